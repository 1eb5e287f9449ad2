"""Pins of the FP64 oracle against facts fixed by the paper or by mathematics.

Each test is chosen so that a plausible slip in the oracle (a dropped
interference term, a wrong conjugate, a missing factor 2, a wrong cell index,
a reversed projection test) fails at least one of them.  None of them re-types
the oracle's own formula: they use textbook closed forms, finite differences
of an independently written quantity, brute force, invariances and the
monotonicity / stationarity statements of Section VI.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import ammse_oracle as OM
from instances import instance, random_instance, water_filling, weighted_water_filling

pytestmark = []


def _prob(inst):
    p = O.from_instance(inst)
    return p, O.split_v(p, inst["V0"])


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

def _single_user(seed, M, N, d, P, sigma2):
    rng = np.random.default_rng(seed)
    H = (rng.standard_normal((N, M)) + 1j * rng.standard_normal((N, M))) / math.sqrt(2)
    V0 = rng.standard_normal((M, d)) + 1j * rng.standard_normal((M, d))
    V0 *= math.sqrt(P) / np.linalg.norm(V0)
    return instance([H], sigma2, 1.0, P, [1], N, d, [V0]), H


@pytest.mark.parametrize("P", [0.3, 10.0, 1000.0])
def test_rate_of_water_filling_precoder_is_capacity(P):
    """Single-user rate of the SVD/water-filling precoder equals sum log2(1+p s^2/s2)."""
    inst, H = _single_user(1, M=6, N=3, d=3, P=P, sigma2=0.7)
    _, s, Vh = np.linalg.svd(H)
    p, cap = water_filling(s ** 2, P, 0.7)
    V = Vh.conj().T[:, :3] * np.sqrt(p)[None, :]
    prob, _ = _prob(inst)
    assert O.wsr_bits(prob, V[None]) == pytest.approx(cap, rel=1e-12)


@pytest.mark.parametrize("P", [1.0, 10.0, 100.0])
def test_single_user_methods_reach_water_filling_capacity(P):
    """WMMSE and A-MMMSE, single user with d = rank H, converge to capacity."""
    inst, H = _single_user(2, M=5, N=2, d=2, P=P, sigma2=1.0)
    s = np.linalg.svd(H, compute_uv=False)
    _, cap = water_filling(s ** 2, P, 1.0)
    prob, V0 = _prob(inst)
    w = O.wmmse(prob, V0, max_iters=2000, eps=1e-14)
    assert w["wsr"] == pytest.approx(cap, rel=1e-8)
    a = O.ammmse(prob, V0, 1500)
    assert a["wsr"] == pytest.approx(cap, rel=1e-9)
    assert a["wsr"] <= cap * (1 + 1e-12)


def test_miso_mrt_capacity():
    """N = d = 1, one user: optimum log2(1 + P ||h||^2 / sigma2) (MRT)."""
    rng = np.random.default_rng(3)
    h = (rng.standard_normal((1, 7)) + 1j * rng.standard_normal((1, 7))) / math.sqrt(2)
    v0 = (rng.standard_normal((7, 1)) + 1j * rng.standard_normal((7, 1)))
    v0 *= math.sqrt(4.0) / np.linalg.norm(v0)
    inst = instance([h], 0.5, 1.0, 4.0, [1], 1, 1, [v0])
    prob, V0 = _prob(inst)
    cap = math.log2(1 + 4.0 * np.vdot(h, h).real / 0.5)
    assert O.wmmse(prob, V0, max_iters=1000, eps=1e-14)["wsr"] == pytest.approx(cap, rel=1e-9)
    assert O.ammmse(prob, V0, 2000)["wsr"] == pytest.approx(cap, rel=1e-9)


def test_orthogonal_users_weighted_water_filling():
    """Users on disjoint antenna sets (no interference): the optimum is weighted
    water-filling over the users' channel gains; alpha must weight the rates."""
    rng = np.random.default_rng(4)
    M, U = 8, 4
    H = np.zeros((U, M), np.complex128)
    for u in range(U):
        H[u, 2 * u: 2 * u + 2] = (rng.standard_normal(2) + 1j * rng.standard_normal(2)) * 0.6
    alpha = np.array([0.5, 1.5, 1.0, 0.8])
    sig = 1.0
    P = 3.0
    V0 = rng.standard_normal((M, U)) + 1j * rng.standard_normal((M, U))
    V0 *= math.sqrt(P) / np.linalg.norm(V0)
    inst = instance([H], sig, alpha, P, [U], 1, 1, [V0])
    prob, V0u = _prob(inst)
    g = np.sum(np.abs(H) ** 2, axis=1)
    p, opt = weighted_water_filling(g, alpha, P, sig)
    assert np.count_nonzero(p == 0) >= 1          # the weights switch a user off
    w = O.wmmse(prob, V0u, max_iters=5000, eps=1e-15)
    assert w["wsr"] == pytest.approx(opt, rel=1e-6)
    a = O.ammmse(prob, V0u, 3000)
    assert a["wsr"] == pytest.approx(opt, rel=1e-5)
    assert a["wsr"] <= opt * (1 + 1e-9)


# ---------------------------------------------------------------------------
# Identities and derivatives
# ---------------------------------------------------------------------------

def test_rate_definition_matches_covariance_determinants():
    """R_u = log det(all + s2 I) - log det(interference + s2 I), multi-cell."""
    inst = random_instance(5, M=6, cell_users=[2, 3], N=2, d=2, P=[3.0, 5.0], sigma2=0.4)
    prob, V = _prob(inst)
    R = O.user_rates(prob, V)
    for u in range(prob.U):
        tot = 0.4 * np.eye(2)
        intf = 0.4 * np.eye(2)
        for l in range(prob.U):
            Hul = prob.Hs[u, prob.cell[l]]
            Q = Hul @ V[l] @ V[l].conj().T @ Hul.conj().T
            tot = tot + Q
            if l != u:
                intf = intf + Q
        ref = np.linalg.slogdet(tot)[1] - np.linalg.slogdet(intf)[1]
        assert R[u] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_rate_equals_minus_logdet_mmse_error():
    """At the MMSE receiver, R_u = -log det E_u and the general MSE definition
    reduces to I - U^H H V (Woodbury)."""
    inst = random_instance(6, M=5, cell_users=[2, 2], N=3, d=2, P=[4.0, 2.0], sigma2=0.8,
                           alpha_range=(0.5, 1.5))
    prob, V = _prob(inst)
    Uu = O.mmse_receivers(prob, V)
    E_gen = O.mse_matrices(prob, Uu, V)
    E_red = O.mse_at_mmse(prob, Uu, V)
    np.testing.assert_allclose(E_gen, E_red, rtol=0, atol=1e-12)
    R = O.user_rates(prob, V)
    for u in range(prob.U):
        assert R[u] == pytest.approx(-np.linalg.slogdet(E_red[u])[1], rel=1e-11)


def test_mmse_receiver_minimises_mse_trace():
    """U from the receiver equation minimises Tr(W E) for any PD W (Section VI
    stationarity in U): random perturbations can only increase f."""
    inst = random_instance(7, M=4, cell_users=[3], N=2, d=2, P=5.0)
    prob, V = _prob(inst)
    Uu = O.mmse_receivers(prob, V)
    rng = np.random.default_rng(0)
    Wu = []
    for _ in range(prob.U):
        X = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        Wu.append(X @ X.conj().T + np.eye(2))
    Wu = np.array(Wu)
    f0 = O.objective_f(prob, Uu, Wu, V)
    for _ in range(20):
        dU = (rng.standard_normal(Uu.shape) + 1j * rng.standard_normal(Uu.shape)) * 1e-3
        assert O.objective_f(prob, Uu + dU, Wu, V) >= f0 - 1e-12


def test_w_update_minimises_objective():
    """W = E^{-1} minimises Tr(W E) - log det W over PD W."""
    inst = random_instance(8, M=4, cell_users=[3], N=2, d=2, P=5.0)
    prob, V = _prob(inst)
    Uu = O.mmse_receivers(prob, V)
    Wu = OM._inv_hermitian(O.mse_at_mmse(prob, Uu, V))
    f0 = O.objective_f(prob, Uu, Wu, V)
    rng = np.random.default_rng(1)
    for _ in range(20):
        X = (rng.standard_normal(Wu.shape) + 1j * rng.standard_normal(Wu.shape)) * 1e-3
        dW = X + np.conj(np.swapaxes(X, 1, 2))
        assert O.objective_f(prob, Uu, Wu + dW, V) >= f0 - 1e-12


def _dirderiv(fun, V, D, h=1e-6):
    return (fun(V + h * D) - fun(V - h * D)) / (2 * h)


def test_gradient_matches_finite_differences_of_objective():
    """<grad, D> (real inner product of Definition 1) equals the directional
    derivative of f(U, W, .) for fixed U, W, in a two-cell instance."""
    inst = random_instance(9, M=5, cell_users=[2, 1], N=2, d=2, P=[3.0, 3.0], sigma2=0.6,
                           alpha_range=(0.5, 1.5))
    prob, V = _prob(inst)
    rng = np.random.default_rng(2)
    Uu = (rng.standard_normal((prob.U, 2, 2)) + 1j * rng.standard_normal((prob.U, 2, 2)))
    Wu = []
    for _ in range(prob.U):
        X = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        Wu.append(X @ X.conj().T + np.eye(2))
    Wu = np.array(Wu)
    g = O.gradient_v(prob, Uu, Wu, V)
    for _ in range(5):
        D = rng.standard_normal(V.shape) + 1j * rng.standard_normal(V.shape)
        fd = _dirderiv(lambda X: O.objective_f(prob, Uu, Wu, X), V, D)
        assert np.vdot(g, D).real == pytest.approx(fd, rel=1e-7)


def test_gradient_is_minus_wsr_gradient_at_block_optimum():
    """Envelope theorem: at the MMSE receiver and W = E^{-1}, the V gradient
    of f equals minus the gradient of sum alpha R (nats) of the plain rate."""
    inst = random_instance(10, M=4, cell_users=[2, 2], N=2, d=1, P=[2.0, 6.0], sigma2=0.5,
                           alpha_range=(0.5, 1.5))
    prob, V = _prob(inst)
    Uu = O.mmse_receivers(prob, V)
    Wu = OM._inv_hermitian(O.mse_at_mmse(prob, Uu, V))
    g = O.gradient_v(prob, Uu, Wu, V)
    rng = np.random.default_rng(3)
    wsr_nats = lambda X: float(np.dot(prob.alpha, O.user_rates(prob, X)))
    for _ in range(5):
        D = rng.standard_normal(V.shape) + 1j * rng.standard_normal(V.shape)
        fd = _dirderiv(wsr_nats, V, D)
        assert np.vdot(g, D).real == pytest.approx(-fd, rel=1e-7)


def test_step_size_descent_lemma_and_lemma3_bound():
    """With gamma = 1/||2A||_2 the unconstrained gradient step decreases f by at
    least gamma ||grad||^2 / 2 (descent lemma), a step of 2.5/||2A|| along the
    top curvature direction increases f, and ||2A_c|| <= 2 alpha_max U kappa / s2
    (Lemma 3)."""
    inst = random_instance(11, M=6, cell_users=[3], N=2, d=2, P=8.0, sigma2=0.9,
                           alpha_range=(0.5, 1.5))
    prob, V = _prob(inst)
    Uu = O.mmse_receivers(prob, V)
    Wu = OM._inv_hermitian(O.mse_at_mmse(prob, Uu, V))
    A = O.transmit_hessians(prob, Uu, Wu)
    gamma = O.step_sizes(A)[0]
    g = O.gradient_v(prob, Uu, Wu, V, A)
    f = lambda X: O.objective_f(prob, Uu, Wu, X)
    f0 = f(V)
    assert f(V - gamma * g) <= f0 - 0.5 * gamma * np.vdot(g, g).real + 1e-10
    # along the top eigenvector of A, the quadratic model has curvature 1/gamma
    lam, Q = np.linalg.eigh(0.5 * (A[0] + A[0].conj().T))
    D = np.zeros_like(V)
    D[0, :, 0] = Q[:, -1]
    slope = np.vdot(O.gradient_v(prob, Uu, Wu, V, A), D).real
    curv = (f(V + 1e-3 * D) - 2 * f0 + f(V - 1e-3 * D)) / 1e-6
    assert curv == pytest.approx(1.0 / gamma, rel=1e-5)
    L3 = 2 * prob.alpha.max() * prob.U * O.kappa(prob) / prob.sigma2.min()
    assert 1.0 / gamma <= L3


def test_projection_properties():
    """Closed-form projection onto the ball: result power min(p, P), idempotent,
    untouched inside, obtuse-angle property against feasible points."""
    inst = random_instance(12, M=4, cell_users=[2, 3], N=1, d=1, P=[1.0, 2.0])
    prob, V = _prob(inst)
    rng = np.random.default_rng(4)
    X = (rng.standard_normal(V.shape) + 1j * rng.standard_normal(V.shape)) * 2
    PX = O.project_spc(prob, X)
    for c in range(prob.C):
        users = prob.cell == c
        p_in = np.vdot(X[users], X[users]).real
        p_out = np.vdot(PX[users], PX[users]).real
        assert p_out == pytest.approx(min(p_in, prob.P[c]), rel=1e-12)
    np.testing.assert_allclose(O.project_spc(prob, PX), PX, rtol=1e-14, atol=1e-15)
    small = X * 1e-3
    np.testing.assert_array_equal(O.project_spc(prob, small), small)
    for _ in range(20):
        Y = rng.standard_normal(V.shape) + 1j * rng.standard_normal(V.shape)
        Y = O.project_spc(prob, Y * 0.3)
        assert np.vdot(X - PX, Y - PX).real <= 1e-10


def test_omega_printed_values():
    """omega^t = max{(t-2)/(t+1), 0}: 0, 0, 1/4, 2/5, 1/2 for t = 1..5."""
    assert [O.omega_schedule(t) for t in range(1, 6)] == pytest.approx(
        [0.0, 0.0, 0.25, 0.4, 0.5], abs=1e-15)
    assert all(0 <= O.omega_schedule(t) < 1 for t in range(1, 1000))


# ---------------------------------------------------------------------------
# Monotonicity, stationarity, bounds (Section VI)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cells", [[4], [2, 3]])
def test_wmmse_wsr_monotone(cells):
    inst = random_instance(13, M=8, cell_users=cells, N=2, d=2, P=10.0, alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    w = O.wmmse(prob, V0, max_iters=200, eps=1e-12)
    assert np.all(np.diff(w["trace"]) >= -1e-9 * w["trace"][1:])


@pytest.mark.parametrize("cells", [[4], [2, 3]])
def test_ammmse_stage2_monotone_without_extrapolation(cells):
    """Theorem 1 chain: stage II, no extrapolation, gamma = 1/L every iteration
    => WSR(V^t) non-decreasing."""
    inst = random_instance(14, M=8, cell_users=cells, N=2, d=2, P=30.0, alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    r = O.ammmse(prob, V0, 150, Tc=150, extrapolate=False, warm_start=False)
    tr = r["trace"]
    assert np.all(np.diff(tr) >= -1e-10 * tr[1:])
    assert tr[-1] > tr[0]


def test_spc_active_and_kkt_at_convergence_single_cell():
    """Single cell: the budget is met with equality at a stationary point and
    the stationarity residual vanishes (Definition 2)."""
    inst = random_instance(15, M=8, cell_users=[4], N=2, d=2, P=10.0)
    prob, V0 = _prob(inst)
    w = O.wmmse(prob, V0, max_iters=3000, eps=1e-13)
    p = np.vdot(w["V"], w["V"]).real
    assert p == pytest.approx(10.0, rel=1e-9)
    assert O.kkt_residual(prob, w["V"]) < 1e-4
    # Theorem 1 regime: a step no larger than 1/L in every iteration
    a = O.ammmse(prob, V0, 3000, Tc=3000)
    assert np.vdot(a["V"], a["V"]).real == pytest.approx(10.0, rel=1e-9)
    assert O.kkt_residual(prob, a["V"]) < 1e-8
    assert a["wsr"] == pytest.approx(w["wsr"], rel=1e-6)
    # a non-stationary point has a large residual
    assert O.kkt_residual(prob, V0) > 0.1


def test_lemma_bounds_along_iterates():
    """Lemma 1: lambda_min(E) >= s2/(P kappa + s2); Lemma 2: ||U||_F^2 <= d/s2,
    lambda_max(W) <= (P kappa + s2)/s2, for every iterate of A-MMMSE."""
    inst = random_instance(16, M=6, cell_users=[2, 2], N=2, d=2, P=[20.0, 20.0], sigma2=0.3)
    prob, V = _prob(inst)
    kap = O.kappa(prob)
    Pm = prob.P.max()
    r = O.ammmse(prob, V, 1)
    Vt = V
    for t in range(25):
        Uu = O.mmse_receivers(prob, Vt)
        E = O.mse_at_mmse(prob, Uu, Vt)
        for u in range(prob.U):
            ev = np.linalg.eigvalsh(E[u])
            assert ev.min() >= 0.3 / (Pm * kap + 0.3) * (1 - 1e-12)
            assert np.linalg.norm(Uu[u]) ** 2 <= prob.d / 0.3 * (1 + 1e-12)
            assert (1.0 / ev.min()) <= (Pm * kap + 0.3) / 0.3 * (1 + 1e-12)
        r = O.ammmse(prob, Vt, 1, warm_start=False)
        Vt = r["V"]


def test_brute_force_tiny_instance():
    """M = 2, two single-antenna users: dense sampling of the power sphere plus
    local polish gives the global optimum; WMMSE / A-MMMSE never exceed it and
    the best of several starts reaches it."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(17)
    H = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / math.sqrt(2)
    P, s2 = 5.0, 1.0
    alpha = np.array([1.0, 1.3])

    def wsr(x):
        v = (x[:4] + 1j * x[4:]).reshape(2, 2)          # columns v1, v2
        v = v * math.sqrt(P) / np.linalg.norm(v)
        r = 0.0
        for u in range(2):
            sig = abs(H[u] @ v[:, u]) ** 2
            intf = abs(H[u] @ v[:, 1 - u]) ** 2
            r += alpha[u] * math.log2(1 + sig / (s2 + intf))
        return r

    X = rng.standard_normal((200000, 8))
    vals = np.array([wsr(x) for x in X[:20000]])
    best = X[np.argsort(-vals)[:10]]
    brute = max(-minimize(lambda x: -wsr(x), x0, method="Nelder-Mead",
                          options=dict(xatol=1e-12, fatol=1e-14, maxiter=20000)).fun
                for x0 in best)
    results_w, results_a = [], []
    for s in range(6):
        V0 = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        V0 *= math.sqrt(P) / np.linalg.norm(V0)
        inst = instance([H], s2, alpha, P, [2], 1, 1, [V0])
        prob, V0u = _prob(inst)
        results_w.append(O.wmmse(prob, V0u, max_iters=3000, eps=1e-14)["wsr"])
        results_a.append(O.ammmse(prob, V0u, 1500)["wsr"])
    assert max(results_w) <= brute + 1e-7
    assert max(results_a) <= brute + 1e-7
    assert max(results_w) == pytest.approx(brute, rel=1e-6)
    assert max(results_a) == pytest.approx(brute, rel=1e-6)


# ---------------------------------------------------------------------------
# Invariances and structure
# ---------------------------------------------------------------------------

def test_noise_scaling_invariance():
    """(H, s2) -> (c H, c^2 s2) leaves every A-MMMSE iterate's WSR unchanged."""
    inst = random_instance(18, M=6, cell_users=[2, 2], N=2, d=2, P=[5.0, 5.0], sigma2=1.0,
                           alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    r1 = O.ammmse(prob, V0, 40)
    inst2 = dict(inst)
    inst2["H"] = [h * 1e-5 for h in inst["H"]]
    inst2["sigma2"] = inst["sigma2"] * 1e-10
    prob2, _ = _prob(inst2)
    r2 = O.ammmse(prob2, V0, 40)
    np.testing.assert_allclose(r1["trace"], r2["trace"], rtol=1e-9)
    assert r1["switch_iter"] == r2["switch_iter"]


def test_unitary_rotation_invariance():
    """H -> H Q (per BS), V0 -> Q^H V0 leaves the WSR trajectory unchanged."""
    inst = random_instance(19, M=5, cell_users=[3], N=2, d=2, P=4.0)
    prob, V0 = _prob(inst)
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5)))
    inst2 = dict(inst)
    inst2["H"] = [inst["H"][0] @ Q]
    prob2, _ = _prob(inst2)
    V02 = np.einsum("mk,ukd->umd", Q.conj().T, V0)
    r1 = O.ammmse(prob, V0, 30)
    r2 = O.ammmse(prob2, V02, 30)
    np.testing.assert_allclose(r1["trace"], r2["trace"], rtol=1e-9)


def test_user_permutation_invariance():
    """Reordering users inside a cell (with their alpha) changes nothing."""
    inst = random_instance(20, M=6, cell_users=[3], N=2, d=1, P=6.0, alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    perm = [2, 0, 1]
    H = inst["H"][0].reshape(3, 2, 6)[perm].reshape(6, 6)
    V0b = inst["V0"][0][:, perm]
    inst2 = instance([H], inst["sigma2"][perm], inst["alpha"][perm], inst["P"], [3], 2, 1, [V0b])
    prob2, V02 = _prob(inst2)
    r1 = O.ammmse(prob, V0, 30)
    r2 = O.ammmse(prob2, V02, 30)
    np.testing.assert_allclose(r1["trace"], r2["trace"], rtol=1e-10)


def test_decoupled_cells_sum_of_single_cells():
    """No cross-cell channels: the two-cell problem is two independent
    single-cell problems (same steps per BS), so every iterate's WSR is the sum
    - provided both cells switch stage together, which a forced switch ensures."""
    a = random_instance(21, M=5, cell_users=[2], N=2, d=2, P=3.0, alpha_range=(0.5, 1.5))
    b = random_instance(22, M=5, cell_users=[3], N=2, d=2, P=7.0, alpha_range=(0.5, 1.5))
    U = 5
    H0 = np.zeros((U * 2, 5), np.complex128)
    H1 = np.zeros((U * 2, 5), np.complex128)
    H0[:4] = a["H"][0]
    H1[4:] = b["H"][0]
    joint = instance([H0, H1], 1.0, np.concatenate([a["alpha"], b["alpha"]]), [3.0, 7.0],
                     [2, 3], 2, 2, [a["V0"][0], b["V0"][0]])
    pj, Vj = _prob(joint)
    pa, Va = _prob(a)
    pb, Vb = _prob(b)
    rj = O.ammmse(pj, Vj, 30, force_switch_iter=5)
    ra = O.ammmse(pa, Va, 30, force_switch_iter=5)
    rb = O.ammmse(pb, Vb, 30, force_switch_iter=5)
    np.testing.assert_allclose(rj["trace"], ra["trace"] + rb["trace"], rtol=1e-10)


def test_stage_switch_rule_on_trace():
    """The latch fires at the first t >= 2 whose relative WSR change between
    V^{t-1} and V^{t-2} is <= eps1, and never before."""
    inst = random_instance(23, M=8, cell_users=[4], N=2, d=2, P=10.0)
    prob, V0 = _prob(inst)
    for eps1 in (0.3, 0.1, 0.02):
        r = O.ammmse(prob, V0, 40, eps1=eps1)
        tr, s = r["trace"], r["switch_iter"]
        assert s >= 2
        rel = [O.rel_change(tr[t - 1], tr[t - 2]) for t in range(2, s + 1)]
        assert rel[-1] <= eps1
        assert all(x > eps1 for x in rel[:-1])


def test_wmmse_subproblem_optimality():
    """The WMMSE V step solves its convex QCQP: no feasible perturbation lowers
    the subproblem objective f(U, W, .), and lambda (P - p) = 0."""
    inst = random_instance(24, M=6, cell_users=[3], N=2, d=2, P=2.0)
    prob, V = _prob(inst)
    Uu = O.mmse_receivers(prob, V)
    Wu = OM._inv_hermitian(O.mse_at_mmse(prob, Uu, V))
    Vn, lam = O.wmmse_precoder(prob, Uu, Wu)
    p = np.vdot(Vn, Vn).real
    assert lam[0] * (2.0 - p) == pytest.approx(0.0, abs=1e-8)
    assert p <= 2.0 * (1 + 1e-10)
    f0 = O.objective_f(prob, Uu, Wu, Vn)
    rng = np.random.default_rng(6)
    for _ in range(30):
        Y = Vn + 0.05 * (rng.standard_normal(Vn.shape) + 1j * rng.standard_normal(Vn.shape))
        Y = O.project_spc(prob, Y)
        assert O.objective_f(prob, Uu, Wu, Y) >= f0 - 1e-9


# ---------------------------------------------------------------------------
# MMMSE (Section V-B)
# ---------------------------------------------------------------------------

def _sum_mse(prob, V):
    """sum_u alpha_u Tr(E_u) at the MMSE receivers of V (the stage-I objective),
    E_u from the general MSE definition."""
    Uu = O.mmse_receivers(prob, V)
    E = O.mse_matrices(prob, Uu, V)
    return float(sum(prob.alpha[u] * np.trace(E[u]).real for u in range(prob.U)))


@pytest.mark.parametrize("cells", [[4], [2, 3]])
def test_mmmse_stage1_is_descent_on_sum_mse(cells):
    """Block coordinate descent on the sum-MSE problem: with the switch never
    taken, sum alpha Tr(E) at the MMSE receivers does not increase."""
    inst = random_instance(51, M=8, cell_users=cells, N=2, d=2, P=10.0, alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    vals = [_sum_mse(prob, V0)]
    for t in range(1, 9):
        r = O.mmmse(prob, V0, max_iters=t, eps1=-1.0, eps2=0.0)
        assert r["switch_iter"] == -1
        vals.append(_sum_mse(prob, r["V"]))
    assert np.all(np.diff(vals) <= 1e-10 * np.abs(vals[1:]))
    assert vals[-1] < vals[0]


def test_mmmse_with_immediate_switch_is_wmmse():
    inst = random_instance(52, M=8, cell_users=[2, 2], N=2, d=2, P=10.0, alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    a = O.mmmse(prob, V0, max_iters=30, eps2=0.0, force_switch_iter=1)
    b = O.wmmse(prob, V0, max_iters=30, eps=-1.0)
    np.testing.assert_allclose(a["trace"], b["trace"], rtol=1e-13)


def test_mmmse_switch_rule_and_stage2_monotone():
    inst = random_instance(53, M=8, cell_users=[4], N=2, d=2, P=30.0, alpha_range=(0.5, 1.5))
    prob, V0 = _prob(inst)
    r = O.mmmse(prob, V0, max_iters=80, eps1=0.1, eps2=0.0)
    s, tr = r["switch_iter"], r["trace"]
    assert s >= 2
    rel = lambda a, b: abs(a - b) / b
    assert rel(tr[s - 1], tr[s - 2]) <= 0.1
    assert all(rel(tr[t - 1], tr[t - 2]) > 0.1 for t in range(2, s))
    assert np.all(np.diff(tr[s:]) >= -1e-9 * tr[s + 1:])
