"""Pins of the oracle's step-size rule, stop rule and channel constant.

The fixed step of Algorithm 3 is not given by the paper.  The oracle's default
reading takes, in stage II after the adaptive window, gamma_c = 1 / Lhat_c with
Lhat_c = 2 lambda_max(sum_u (alpha_u / sigma2_u) H_{u,c}^H H_{u,c}) (``step_bound``),
an upper bound of the V-gradient's Lipschitz constant at every iterate (the
argument of Lemma 3, Section VI, on the stacked channel).  The tests below pin
that quantity by closed forms and by its tightness at high SNR, the
consequences Theorem 1 draws from a step within the bound (monotone WSR in
stage II without extrapolation), the stability of the resulting trajectories
at the benchmark sizes, the epsilon_2 stop (Algorithm 3's "until" test, read as
applying only after a stage-II step) and kappa (Section VI) on a multi-cell
instance whose strongest link is a cross link.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import ammse_oracle as OM
from instances import instance, random_instance
from paper_2510_20507_amd import synth


def _prob(inst):
    p = O.from_instance(inst)
    return p, O.split_v(p, inst["V0"])


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def _lipschitz(prob, V, stage2):
    """||2 A_c||_2 per BS at the MMSE receivers of V (W = E^{-1} or I)."""
    Uu = O.mmse_receivers(prob, V)
    if stage2:
        Wu = OM._inv_hermitian(O.mse_at_mmse(prob, Uu, V))
    else:
        Wu = np.broadcast_to(np.eye(prob.d), (prob.U, prob.d, prob.d)).copy()
    A = O.transmit_hessians(prob, Uu, Wu)
    return np.array([2.0 * np.linalg.norm(A[c], 2) for c in range(prob.C)])


# ---------------------------------------------------------------------------
# The bound Lhat_c
# ---------------------------------------------------------------------------

def test_step_bound_miso_closed_form():
    """One user, N = d = 1: Lhat = 2 alpha ||h||^2 / sigma2 (pins the factor 2,
    the weight and the noise power)."""
    rng = np.random.default_rng(1)
    h = _cn(rng, (1, 6))
    v0 = _cn(rng, (6, 1))
    inst = instance([h], 0.7, 1.3, 5.0, [1], 1, 1, [v0])
    prob, _ = _prob(inst)
    assert O.step_bound(prob)[0] == pytest.approx(2 * 1.3 * np.vdot(h, h).real / 0.7, rel=1e-13)


def test_step_bound_orthogonal_users_is_a_maximum_not_a_sum():
    """Users on orthogonal antenna subspaces: the weighted Gram is block
    diagonal, so Lhat = 2 max_u alpha_u ||H_u||_2^2 / sigma2_u."""
    M = 6
    E = np.eye(M)
    H0 = 2.0 * E[0:2]                  # user 0 on antennas 0, 1: ||H_0||_2^2 = 4
    H1 = 1.5 * E[2:4]                  # user 1 on antennas 2, 3: 2.25
    H = np.concatenate([H0, H1]).astype(np.complex128)
    rng = np.random.default_rng(2)
    inst = instance([H], [1.0, 0.5], [1.0, 1.2], 3.0, [2], 2, 2, [_cn(rng, (M, 4))])
    prob, _ = _prob(inst)
    want = 2 * max(1.0 * 4.0 / 1.0, 1.2 * 2.25 / 0.5)
    assert O.step_bound(prob)[0] == pytest.approx(want, rel=1e-13)


def test_step_bound_counts_other_cells_users_and_is_tight_at_high_snr():
    """Two cells, one single-antenna user each, the link from BS 0 to the user
    of cell 1 twice as strong as the direct ones.  At a converged high-SNR point
    the interference is nulled and U W U^H -> 1/sigma2, so ||2 A_0|| approaches
    Lhat_0, which must include the cross user; it never exceeds it."""
    rng = np.random.default_rng(3)
    M = 4
    h00 = _cn(rng, (1, M))            # BS 0 -> user 0 (direct)
    h10 = 2.0 * _cn(rng, (1, M))      # BS 0 -> user 1 (cross, strong)
    h01 = 0.3 * _cn(rng, (1, M))      # BS 1 -> user 0
    h11 = _cn(rng, (1, M))            # BS 1 -> user 1
    H = [np.concatenate([h00, h10]), np.concatenate([h01, h11])]
    V0 = [_cn(rng, (M, 1)), _cn(rng, (M, 1))]
    inst = instance(H, 1.0, 1.0, 1e5, [1, 1], 1, 1, V0)
    prob, V = _prob(inst)
    w = O.wmmse(prob, V, max_iters=400, eps=1e-14)
    L = _lipschitz(prob, w["V"], True)
    Lh = O.step_bound(prob)
    own_only = 2 * np.vdot(h00, h00).real          # what a bound over cell 0's users gives
    assert L[0] <= Lh[0] * (1 + 1e-12)
    assert L[0] >= 0.9 * Lh[0]
    assert L[0] > 1.5 * own_only


@pytest.mark.parametrize("cells,N,d", [([3], 2, 2), ([2, 3], 2, 1), ([3, 1, 2], 1, 1)])
def test_step_bound_dominates_lipschitz_along_iterates(cells, N, d):
    """||2 A_c|| <= Lhat_c <= 2 alpha_max U kappa / sigma2_min (Lemma 3) at every
    iterate of a trajectory, in both stages, and at random feasible points."""
    inst = random_instance(31, M=5, cell_users=cells, N=N, d=d, P=50.0, sigma2=0.4,
                           alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    Lh = O.step_bound(prob)
    L3 = 2 * prob.alpha.max() * prob.U * O.kappa(prob) / prob.sigma2.min()
    assert np.all(Lh <= L3 * (1 + 1e-12))
    pts = [V0]
    r = O.ammmse(prob, V0, 25)
    rng = np.random.default_rng(5)
    for _ in range(4):
        pts.append(O.project_spc(prob, 20 * _cn(rng, V0.shape)))
    V = V0.copy()
    for t in range(15):    # WMMSE iterates as further feasible points
        Uu = O.mmse_receivers(prob, V)
        Wu = OM._inv_hermitian(O.mse_at_mmse(prob, Uu, V))
        V, _ = O.wmmse_precoder(prob, Uu, Wu)
        pts.append(V)
    pts.append(r["V"])
    for X in pts:
        for stage2 in (False, True):
            assert np.all(_lipschitz(prob, X, stage2) <= Lh * (1 + 1e-12))


# ---------------------------------------------------------------------------
# Consequences of the rule (Theorem 1) and stability at the benchmark sizes
# ---------------------------------------------------------------------------

def test_default_rule_is_bound_in_stage2_and_frozen_in_stage1():
    """After the adaptive windows: stage I keeps the last adaptive value, stage
    II uses 1/Lhat; step_rule="frozen" keeps the last adaptive value throughout;
    a positive gamma_c overrides both."""
    inst = random_instance(32, M=8, cell_users=[2, 2], N=2, d=2, P=100.0,
                           alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    r = O.ammmse(prob, V0, 30, force_switch_iter=8)
    g = r["gammas"]
    Lh = O.step_bound(prob)
    np.testing.assert_array_equal(g[3], g[2])         # t = 4: frozen (stage I)
    np.testing.assert_array_equal(g[6], g[2])         # t = 7: still stage I
    assert not np.allclose(g[7], g[2])                # t = 8: re-armed adaptive step
    np.testing.assert_allclose(g[10:], np.broadcast_to(1.0 / Lh, g[10:].shape), rtol=1e-15)
    assert np.all(g[7:10] >= 1.0 / Lh * (1 - 1e-12))  # adaptive steps are never below 1/Lhat
    f = O.ammmse(prob, V0, 30, force_switch_iter=8, step_rule="frozen")["gammas"]
    np.testing.assert_array_equal(f[10:], np.broadcast_to(f[9], f[10:].shape))
    c = O.ammmse(prob, V0, 30, force_switch_iter=8, gamma_c=1e-3)["gammas"]
    np.testing.assert_array_equal(c[10:], 1e-3)


def _rayleigh_30db(i):
    b = synth.rayleigh_sweep(B_per_p=4)
    return b.instance(3 * 4 + i)


def _hexcell(i):
    return synth.hexcell_batch(B=64).instance(i)


@pytest.mark.parametrize("which", ["rayleigh30", "hexcell"])
def test_stage2_monotone_without_extrapolation_at_benchmark_shapes(which):
    """Theorem 1 with the default rule: every stage-II step is within the
    Lipschitz bound, so without extrapolation WSR(V^t) never decreases after
    the switch (64-antenna, 16-user instance at 30 dB; a seven-cell instance)."""
    inst = _rayleigh_30db(0) if which == "rayleigh30" else _hexcell(5)
    prob, V0 = _prob(inst)
    r = O.ammmse(prob, V0, 60, extrapolate=False)
    tr, s = r["trace"], r["switch_iter"]
    assert 2 <= s < 30
    d = np.diff(tr[s:])
    assert np.all(d >= -1e-11 * tr[s + 1:]), d.min()


def test_frozen_rule_oscillates_where_bound_rule_is_stable():
    """64-antenna, 16-user instance at 30 dB, 100 iterations with extrapolation:
    under the bound rule a perturbation of 1e-9 per iterate moves the final WSR
    by < 1e-6 and the last 20 iterations change WSR by < 1e-2 each; under the
    frozen rule the last 20 iterations swing by more than 1 % and the
    perturbation is amplified above 1e-4 (the reason for the default)."""
    inst = _rayleigh_30db(1)
    prob, V0 = _prob(inst)
    rng = np.random.default_rng(9)

    def perturb(t, V):
        return V * (1 + 1e-9 * rng.standard_normal(V.shape))

    out = {}
    for rule in ("bound", "frozen"):
        a = O.ammmse(prob, V0, 100, step_rule=rule)["trace"]
        b = O.ammmse(prob, V0, 100, step_rule=rule, perturb=perturb)["trace"]
        rel = np.abs(np.diff(a[-21:])) / a[-21:-1]
        out[rule] = (abs(a[-1] - b[-1]) / a[-1], rel.max())
    assert out["bound"][0] < 1e-6 and out["bound"][1] < 1e-2
    assert out["frozen"][1] > 1e-2


# ---------------------------------------------------------------------------
# epsilon_2 stop (Algorithm 3, reading R9) and kappa (Section VI)
# ---------------------------------------------------------------------------

def test_eps2_stop_rule_on_trace():
    """With eps2 > 0 the iteration ends before the first t >= 2 whose previous
    V step was a stage-II step and whose relative WSR change between V^{t-1}
    and V^{t-2} is <= eps2 (t - 1 iterations run), and never earlier; the run
    up to there equals the run without a stop test."""
    inst = random_instance(33, M=8, cell_users=[4], N=2, d=2, P=10.0)
    prob, V0 = _prob(inst)
    full = O.ammmse(prob, V0, 120)
    tr, s = full["trace"], full["switch_iter"]
    for eps2 in (1e-2, 1e-3, 1e-5):
        r = O.ammmse(prob, V0, 120, eps2=eps2)
        n = r["iters"]
        # first stage-II step is iteration s, so the test applies from t = s + 1
        cand = [t for t in range(s + 1, 121) if O.rel_change(tr[t - 1], tr[t - 2]) <= eps2]
        assert cand, eps2
        assert n == cand[0] - 1
        np.testing.assert_array_equal(r["trace"], tr[:n + 1])
        assert r["switch_iter"] == s


def test_eps2_never_stops_in_stage1():
    """A tiny relative change during stage I (forced late switch) does not stop
    the run: the first possible stop follows the first stage-II step."""
    inst = random_instance(34, M=8, cell_users=[4], N=2, d=2, P=10.0)
    prob, V0 = _prob(inst)
    r = O.ammmse(prob, V0, 60, eps2=0.5, force_switch_iter=20)
    assert r["iters"] == 20


def test_kappa_on_cross_link():
    """kappa = max over all user-BS pairs of sigma_max(H^H H): channels built as
    a scaled matrix with orthonormal rows have sigma_max(H^H H) = scale^2, and
    the maximum sits on a cross link (BS 1 -> user of cell 0)."""
    rng = np.random.default_rng(6)
    M, N = 6, 2

    def scaled_orth(a):
        Q, _ = np.linalg.qr(_cn(rng, (M, N)))
        return a * Q.conj().T               # N x M, orthonormal rows times a

    H0 = np.concatenate([scaled_orth(1.0), scaled_orth(0.5)])     # BS 0 -> users 0, 1
    H1 = np.concatenate([scaled_orth(3.0), scaled_orth(1.2)])     # BS 1 -> users 0, 1
    inst = instance([H0, H1], 1.0, 1.0, 1.0, [1, 1], N, N, [_cn(rng, (M, 2))] * 2)
    prob, _ = _prob(inst)
    assert O.kappa(prob) == pytest.approx(9.0, rel=1e-13)
