"""Pins of the unrolled-solver oracle (CPU): its forward is Algorithm 3 with
the given steps (checked against the NumPy oracle run with a fixed step and
the same switch), and its autograd gradients agree with central finite
differences of the forward, for the step sizes and along random channel
directions (which also fixes the complex-gradient convention)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2510_20507_amd import synth  # noqa: E402
import oracle as O  # noqa: E402
from oracle import unrolled as UR  # noqa: E402


def _inst(seed=31, M=6, U=3, N=2, d=2, P=10.0):
    b = synth.rayleigh_batch(seed, 1, M=M, U=U, N=N, d=d, P=P, alpha_range=(0.5, 1.5),
                             name="unroll_pin")
    inst = b.instance(0)
    prob = O.from_instance(inst)
    H = prob.Hs[:, 0]                       # [U, N, M]
    V0 = O.split_v(prob, inst["V0"])        # [U, M, d]
    return prob, H, V0


def test_forward_matches_numpy_oracle_with_fixed_step():
    prob, H, V0 = _inst()
    T, g, s = 12, 0.05, 4
    ref = O.ammmse(prob, V0, T, Tc=0, gamma_c=g, force_switch_iter=s)
    wsr, _, _, VT, trace = UR.value_and_grad(H, prob.sigma2, prob.alpha, prob.P[0], V0,
                                             [g] * T, s)
    np.testing.assert_allclose(trace, ref["trace"][:T], rtol=1e-12)
    assert wsr == pytest.approx(ref["wsr"], rel=1e-12)
    np.testing.assert_allclose(VT, ref["V"], rtol=0, atol=1e-12 * np.abs(ref["V"]).max())


def _fd_wsr(prob, H, V0, gammas, s):
    w, _, _, _, _ = UR.value_and_grad(H, prob.sigma2, prob.alpha, prob.P[0], V0, gammas, s)
    return w


@pytest.mark.parametrize("s", [3, 1])
def test_step_size_gradient_matches_finite_differences(s):
    prob, H, V0 = _inst(seed=32)
    T = 8
    gam = np.linspace(0.03, 0.06, T)
    _, gg, _, _, _ = UR.value_and_grad(H, prob.sigma2, prob.alpha, prob.P[0], V0, gam, s)
    for t in range(T):
        h = 1e-6 * gam[t]
        gp, gm = gam.copy(), gam.copy()
        gp[t] += h
        gm[t] -= h
        fd = (_fd_wsr(prob, H, V0, gp, s) - _fd_wsr(prob, H, V0, gm, s)) / (2 * h)
        assert gg[t] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(gg).max()), t


def test_channel_gradient_matches_directional_finite_differences():
    prob, H, V0 = _inst(seed=33)
    T, s = 6, 3
    gam = np.full(T, 0.04)
    _, _, gH, _, _ = UR.value_and_grad(H, prob.sigma2, prob.alpha, prob.P[0], V0, gam, s)
    rng = np.random.default_rng(7)
    for _ in range(3):
        D = rng.standard_normal(H.shape) + 1j * rng.standard_normal(H.shape)
        h = 1e-6
        # the oracle normalises nothing: perturb H of the problem directly
        fp = _fd_wsr(prob, H + h * D, V0, gam, s)
        fm = _fd_wsr(prob, H - h * D, V0, gam, s)
        fd = (fp - fm) / (2 * h)
        an = float(np.real(np.sum(np.conj(gH) * D)))
        assert an == pytest.approx(fd, rel=1e-5)


def test_projection_branch_is_active_in_the_pins():
    """The pinned runs exercise the projection scaling (budget active)."""
    prob, H, V0 = _inst(seed=32)
    _, _, _, VT, _ = UR.value_and_grad(H, prob.sigma2, prob.alpha, prob.P[0], V0,
                                       np.linspace(0.03, 0.06, 8), 3)
    assert np.sum(np.abs(VT) ** 2) == pytest.approx(prob.P[0], rel=1e-12)


def test_switch_iteration_matches_the_numpy_oracle():
    """The eps1 rule on the unrolled solver with a fixed step picks the same
    switch iteration as Algorithm 3 in the NumPy oracle with that fixed step."""
    prob, H, V0 = _inst(seed=37)
    T, g = 20, 0.05
    ref = O.ammmse(prob, V0, T, Tc=0, gamma_c=g)
    s = UR.switch_iter(H, prob.sigma2, prob.alpha, prob.P[0], V0, [g] * T)
    assert 2 <= ref["switch_iter"] <= T
    assert s == ref["switch_iter"]
    assert UR.switch_iter(H, prob.sigma2, prob.alpha, prob.P[0], V0, [g] * T, eps1=0.0) == T + 1
