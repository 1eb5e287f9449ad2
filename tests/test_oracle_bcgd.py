"""Pins of the oracle's BCGD-WMMSE (Section VII-F ablation: U, W and V each
by one explicit step, W by the Schulz iteration W (2I - E W)).

The receiver gradient is checked against finite differences of the
objective f (Definition 1 inner product) and must vanish at the MMSE receiver;
the receiver step must be a descent step; the Schulz step obeys
I - E W' = (I - E W)^2 exactly and keeps E^{-1} fixed; a converged WMMSE
point is a fixed point of the whole iteration (stationarity, Definition 2);
and on a single-antenna single-user channel the method reaches the MISO
capacity log2(1 + P ||h||^2 / sigma2)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import ammse_oracle as OM
from instances import instance, random_instance


def _prob(inst):
    p = O.from_instance(inst)
    return p, O.split_v(p, inst["V0"])


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def _hpd(rng, n, scale=1.0):
    X = _cn(rng, (n, n))
    return scale * (X @ X.conj().T + 0.5 * np.eye(n))


def test_receiver_gradient_matches_finite_differences():
    inst = random_instance(41, M=6, cell_users=[2, 2], N=3, d=2, P=[4.0, 6.0], sigma2=0.7,
                           alpha_range=(0.5, 1.5))
    prob, V = _prob(inst)
    rng = np.random.default_rng(3)
    Uu = _cn(rng, (prob.U, prob.N, prob.d))
    Wu = np.stack([_hpd(rng, prob.d) for _ in range(prob.U)])
    g = O.receiver_gradient(prob, Uu, Wu, V)
    f = lambda X: O.objective_f(prob, X, Wu, V)
    for _ in range(5):
        D = _cn(rng, Uu.shape)
        h = 1e-6
        fd = (f(Uu + h * D) - f(Uu - h * D)) / (2 * h)
        assert np.vdot(g, D).real == pytest.approx(fd, rel=1e-7)


def test_receiver_gradient_vanishes_at_mmse_receiver():
    inst = random_instance(42, M=6, cell_users=[3, 1], N=2, d=2, P=[4.0, 2.0])
    prob, V = _prob(inst)
    Uu = O.mmse_receivers(prob, V)
    rng = np.random.default_rng(4)
    Wu = np.stack([_hpd(rng, prob.d) for _ in range(prob.U)])
    g = O.receiver_gradient(prob, Uu, Wu, V)
    assert np.abs(g).max() <= 1e-12 * np.abs(O.receiver_gradient(prob, 0 * Uu, Wu, V)).max()


def test_receiver_step_is_a_descent_step():
    """With the step 1 / (2 alpha ||J||_F ||W||_F) <= 1 / L_U the descent lemma
    holds: f drops by at least gamma ||grad||^2 / 2 per user block."""
    inst = random_instance(43, M=5, cell_users=[3], N=3, d=2, P=20.0, sigma2=0.3,
                           alpha_range=(0.5, 1.5))
    prob, V = _prob(inst)
    rng = np.random.default_rng(5)
    Uu = _cn(rng, (prob.U, prob.N, prob.d))
    Wu = np.stack([_hpd(rng, prob.d, 2.0) for _ in range(prob.U)])
    g = O.receiver_gradient(prob, Uu, Wu, V)
    J = O.rx_covariances(prob, V)
    gam = 1.0 / (2 * prob.alpha * np.linalg.norm(J, axis=(1, 2)) * np.linalg.norm(Wu, axis=(1, 2)))
    f0 = O.objective_f(prob, Uu, Wu, V)
    f1 = O.objective_f(prob, Uu - gam[:, None, None] * g, Wu, V)
    assert f1 <= f0 - 0.5 * float(np.sum(gam * np.sum(np.abs(g) ** 2, axis=(1, 2)))) + 1e-10


def test_schulz_step_squares_the_residual_and_fixes_the_inverse():
    rng = np.random.default_rng(6)
    for n in (1, 2, 4):
        E = _hpd(rng, n)
        W = np.linalg.inv(E) + 0.05 * _hpd(rng, n, 0.1)
        W = 0.5 * (W + W.conj().T)
        I = np.eye(n)
        Wn = O.schulz_step(W, E)
        np.testing.assert_allclose(I - E @ Wn, (I - E @ W) @ (I - E @ W), atol=1e-12)
        Ei = np.linalg.inv(E)
        np.testing.assert_allclose(O.schulz_step(Ei, E), Ei, rtol=1e-12, atol=1e-14)


def test_converged_wmmse_point_is_a_fixed_point():
    """At a stationary point of the WSR problem (WMMSE run to KKT residual
    ~1e-10) every block step of BCGD-WMMSE leaves the point in place."""
    inst = random_instance(44, M=8, cell_users=[3], N=2, d=2, P=10.0, alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    w = O.wmmse(prob, V0, max_iters=3000, eps=0.0)
    assert O.kkt_residual(prob, w["V"]) < 1e-9
    r = O.bcgd_wmmse(prob, w["V"], 10)
    assert np.linalg.norm(r["V"] - w["V"]) <= 1e-9 * np.linalg.norm(w["V"])
    np.testing.assert_allclose(r["trace"], w["wsr"], rtol=1e-12)


def test_miso_single_user_reaches_capacity():
    rng = np.random.default_rng(7)
    M, P, s2 = 6, 5.0, 0.8
    h = _cn(rng, (1, M))
    v0 = _cn(rng, (M, 1))
    v0 *= math.sqrt(P) / np.linalg.norm(v0)
    inst = instance([h], s2, 1.0, P, [1], 1, 1, [v0])
    prob, V0 = _prob(inst)
    cap = math.log2(1 + P * np.vdot(h, h).real / s2)
    r = O.bcgd_wmmse(prob, V0, 400)
    assert r["wsr"] == pytest.approx(cap, rel=1e-12)
    # without extrapolation every step is a descent step on f: WSR never drops
    r0 = O.bcgd_wmmse(prob, V0, 400, extrapolate=False)
    assert r0["wsr"] == pytest.approx(cap, rel=1e-12)
    assert np.all(np.diff(r0["trace"]) >= -1e-12 * cap)


def test_default_rule_matches_ammmse_v_step_on_exact_blocks():
    """When U and W are already block-optimal the U step does nothing and the
    Schulz step keeps W = E^{-1}; with the step rule of Algorithm 3's second
    stage the first V step then equals A-WMMSE's first step (no warm start)."""
    inst = random_instance(45, M=7, cell_users=[2, 2], N=2, d=1, P=[3.0, 5.0])
    prob, V0 = _prob(inst)
    a = O.ammmse(prob, V0, 1, warm_start=False)
    b = O.bcgd_wmmse(prob, V0, 1)
    np.testing.assert_allclose(b["V"], a["V"], rtol=1e-10, atol=1e-12)


def test_eps2_stop_rule():
    """eps2 > 0 ends the run before the first t >= 2 whose relative WSR change
    between V^{t-1} and V^{t-2} is <= eps2; the run up to there is the run
    without a stop test."""
    inst = random_instance(46, M=8, cell_users=[3], N=2, d=2, P=10.0)
    prob, V0 = _prob(inst)
    full = O.bcgd_wmmse(prob, V0, 80)
    tr = full["trace"]
    for eps2 in (1e-2, 1e-4):
        r = O.bcgd_wmmse(prob, V0, 80, eps2=eps2)
        cand = [t for t in range(2, 81) if O.rel_change(tr[t - 1], tr[t - 2]) <= eps2]
        assert cand and r["iters"] == cand[0] - 1
        np.testing.assert_array_equal(r["trace"], tr[:r["iters"] + 1])
