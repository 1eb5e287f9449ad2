"""Plain FP64 CPU reference for WSR precoding by WMMSE and A-MMMSE.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import or run this module; the GPU product
path never does, and the two share no code.  Everything here is NumPy
complex128 / float64, written from the equations of the paper (arXiv
2510.20507, "A-MMMSE"), one step at a time, with LAPACK (solve, inv, eigh,
eigvalsh, slogdet) as the only library primitives.

Notation (Section II): C base stations ("cells", K in the paper), users u
ordered cell by cell (the paper's i_k), c(u) the serving BS of user u,
H_{u,j} the N x M channel from BS j to user u, V_u the M x d precoder of user
u, sigma2_u the noise power, alpha_u the priority weight, P_c the sum-power
budget of BS c.  Per instance the precoders are held as a stack
``V[u] = V_u`` of shape [U, M, d].

Readings of the paper where it is silent or ambiguous (each is applied the
same way on the GPU; the list is kept with the design notes):

* R1  In Algorithm 3 the receivers U^t, the MSE matrices and the WSR are
      evaluated at V^{t-1}; the extrapolated point enters only the V step.
* R2  The gradient is taken at the extrapolated point (prox-linear rule with
      extrapolation, Section III).
* R3  The stage test in iteration t compares WSR(V^{t-1}) with WSR(V^{t-2});
      the earliest switch is t = 2.
* R4  The stage switch is a one-way latch.
* R5  The fixed step gamma_c is never given numerically.  The adaptive step
      is computed in the first T_c iterations and again in the first T_c
      iterations of stage II (the weighted problem has a larger Lipschitz
      constant than the unweighted one).  In stage I the later iterations
      keep the last adaptive value of each BS.  In stage II the later
      iterations use gamma_c = 1 / Lhat_c with Lhat_c = 2 lambda_max(sum_u
      (alpha_u / sigma2_u) H_{u,c}^H H_{u,c}), an upper bound of the gradient's
      Lipschitz constant ||2 A_c||_2 at every iterate of either stage (Section
      VI, proof of Lemma 3: lambda_max(W U^H U) <= 1 / sigma2, applied to the
      stacked channel of BS c instead of term by term), so every stage-II step
      meets the descent condition of Theorem 1 (step_rule = "bound").
      step_rule = "frozen" keeps the last adaptive value in stage II as well;
      a positive gamma_c overrides both; rearm_at_switch = False gives the
      single window t <= T_c.
* R6  The step size is one scalar per BS (its expression depends only on the
      BS index).
* R8  The extrapolation counter t is not restarted at the stage switch.
* R9  The epsilon_2 stop test is applied only once the previous V step was a
      stage-II step.
* R10 Natural logarithms inside the objective; WSR reported in bits.
* R12 V^0 is supplied by the caller, scaled to full power.
* R14 The projection leaves V unchanged when its power equals the budget.
* relative-change rule: rel(a, b) = |a - b| / b for b > 0; for b == 0 it is
      0 when a == b and +inf otherwise.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np

LN2 = math.log(2.0)

__all__ = [
    "Problem", "from_instance", "split_v", "join_v", "cross_terms", "user_rates", "wsr_bits",
    "mmse_receivers", "mse_matrices", "mse_at_mmse", "objective_f", "transmit_hessians",
    "gradient_v", "step_sizes", "step_bound", "project_spc", "omega_schedule", "rel_change",
    "ammmse", "wmmse", "wmmse_precoder", "mmmse", "bcgd_wmmse", "receiver_gradient",
    "schulz_step", "rx_covariances", "kkt_residual", "kappa", "solve_batch",
]


class Problem:
    """One channel realisation (Section II system model)."""

    def __init__(self, H: Sequence[np.ndarray], sigma2, alpha, P, cell_users: Sequence[int],
                 N: int, d: int):
        self.C = len(H)
        self.cell_users = [int(x) for x in cell_users]
        self.U = int(sum(self.cell_users))
        self.N = int(N)
        self.d = int(d)
        self.M = int(np.asarray(H[0]).shape[1])
        U, M = self.U, self.M
        # Hs[u, j] = H_{u,j}, the N x M channel from BS j to user u.
        self.Hs = np.stack([np.asarray(Hc, np.complex128).reshape(U, N, M) for Hc in H], axis=1)
        self.sigma2 = np.asarray(sigma2, np.float64).reshape(U)
        self.alpha = np.asarray(alpha, np.float64).reshape(U)
        self.P = np.asarray(P, np.float64).reshape(self.C)
        self.cell = np.repeat(np.arange(self.C), self.cell_users)            # c(u)
        self.local = np.concatenate([np.arange(n) for n in self.cell_users]) if U else \
            np.zeros(0, int)

    def H_serving(self) -> np.ndarray:
        """H_{u,c(u)} for every user: [U, N, M]."""
        return self.Hs[np.arange(self.U), self.cell]


def from_instance(inst: dict) -> "Problem":
    """Build a Problem from a per-instance dict (lists of per-BS blocks)."""
    return Problem(inst["H"], inst["sigma2"], inst["alpha"], inst["P"], inst["cell_users"],
                   inst["N"], inst["d"])


def split_v(prob: Problem, blocks: Sequence[np.ndarray]) -> np.ndarray:
    """Per-BS blocks V_c (M x U_c d) -> per-user stack [U, M, d]."""
    out = np.zeros((prob.U, prob.M, prob.d), np.complex128)
    u = 0
    for c in range(prob.C):
        Vc = np.asarray(blocks[c]).reshape(prob.M, prob.cell_users[c] * prob.d)
        for i in range(prob.cell_users[c]):
            out[u] = Vc[:, i * prob.d:(i + 1) * prob.d]
            u += 1
    return out


def join_v(prob: Problem, Vu: np.ndarray) -> list:
    """Per-user stack [U, M, d] -> per-BS blocks V_c (M x U_c d)."""
    out, u = [], 0
    for c in range(prob.C):
        n = prob.cell_users[c]
        out.append(np.concatenate([Vu[u + i] for i in range(n)], axis=1) if n else
                   np.zeros((prob.M, 0), np.complex128))
        u += n
    return out


# ---------------------------------------------------------------------------
# Rates, receivers, MSE (Sections II and IV)
# ---------------------------------------------------------------------------

def cross_terms(prob: Problem, Vu: np.ndarray) -> np.ndarray:
    """T[u, l] = H_{u,c(l)} V_l, the N x d image of user l's precoder at user u."""
    Hsel = prob.Hs[:, prob.cell]                     # [U, U, N, M]: H_{u,c(l)}
    return np.einsum("ulnm,lmd->ulnd", Hsel, Vu)


def _covariances(T: np.ndarray) -> np.ndarray:
    """C[u, l] = T[u,l] T[u,l]^H  ([U, U, N, N])."""
    return np.einsum("ulnd,ulkd->ulnk", T, T.conj())


def user_rates(prob: Problem, Vu: np.ndarray) -> np.ndarray:
    """Achievable rate R_u in nats (Section II):
    log det(I + H_{u,c(u)} V_u V_u^H H^H (sum_{l != u} H_{u,c(l)} V_l V_l^H H^H
    + sigma2_u I)^{-1})."""
    U, N = prob.U, prob.N
    T = cross_terms(prob, Vu)
    Cv = _covariances(T)
    off = (1.0 - np.eye(U))[:, :, None, None]
    I = np.eye(N)
    R = np.zeros(U)
    for u in range(U):
        Jm = (Cv[u] * off[u]).sum(axis=0) + prob.sigma2[u] * I
        S = Cv[u, u]
        sign, logabs = np.linalg.slogdet(I + S @ np.linalg.inv(Jm))
        R[u] = logabs
    return R


def wsr_bits(prob: Problem, Vu: np.ndarray) -> float:
    """Weighted sum rate sum_u alpha_u R_u in bits per channel use."""
    return float(np.dot(prob.alpha, user_rates(prob, Vu)) / LN2)


def mmse_receivers(prob: Problem, Vu: np.ndarray) -> np.ndarray:
    """Receiver update, equation for U (Section IV):
    U_u = (sum_l H_{u,c(l)} V_l V_l^H H_{u,c(l)}^H + sigma2_u I)^{-1} H_{u,c(u)} V_u."""
    T = cross_terms(prob, Vu)
    Cv = _covariances(T)
    I = np.eye(prob.N)
    Uu = np.zeros((prob.U, prob.N, prob.d), np.complex128)
    for u in range(prob.U):
        J = Cv[u].sum(axis=0) + prob.sigma2[u] * I
        Uu[u] = np.linalg.solve(J, T[u, u])
    return Uu


def mse_matrices(prob: Problem, Uu: np.ndarray, Vu: np.ndarray) -> np.ndarray:
    """MSE matrix E_u for arbitrary receivers (definition of E, Section IV):
    (I - U^H H V_u)(I - U^H H V_u)^H + sum_{l != u} U^H H V_l V_l^H H^H U + sigma2 U^H U."""
    T = cross_terms(prob, Vu)
    Id = np.eye(prob.d)
    E = np.zeros((prob.U, prob.d, prob.d), np.complex128)
    for u in range(prob.U):
        Uh = Uu[u].conj().T
        A = Id - Uh @ T[u, u]
        acc = A @ A.conj().T + prob.sigma2[u] * (Uh @ Uu[u])
        for l in range(prob.U):
            if l != u:
                B = Uh @ T[u, l]
                acc = acc + B @ B.conj().T
        E[u] = acc
    return E


def mse_at_mmse(prob: Problem, Uu: np.ndarray, Vu: np.ndarray) -> np.ndarray:
    """E_u = I - U_u^H H_{u,c(u)} V_u (the form inverted by the W update, valid
    at the MMSE receiver), Hermitian-symmetrised."""
    Hs = prob.H_serving()
    E = np.eye(prob.d)[None] - np.einsum("und,unm,ume->ude", Uu.conj(), Hs, Vu)
    return 0.5 * (E + np.conj(np.swapaxes(E, 1, 2)))


def objective_f(prob: Problem, Uu: np.ndarray, Wu: np.ndarray, Vu: np.ndarray) -> float:
    """f(U, W, V) = sum_u alpha_u (Tr(W_u E_u) - log det W_u) (weighted sum-MSE
    objective, Section IV), with E_u from the general MSE definition."""
    E = mse_matrices(prob, Uu, Vu)
    val = 0.0
    for u in range(prob.U):
        sign, logdet = np.linalg.slogdet(Wu[u])
        val += prob.alpha[u] * (np.trace(Wu[u] @ E[u]).real - logdet)
    return float(val)


# ---------------------------------------------------------------------------
# V step of A-MMMSE (Section V-A)
# ---------------------------------------------------------------------------

def transmit_hessians(prob: Problem, Uu: np.ndarray, Wu: np.ndarray) -> np.ndarray:
    """A_c = sum_l alpha_l H_{l,c}^H U_l W_l U_l^H H_{l,c}  ([C, M, M]); the
    gradient's linear term is 2 A_c V_u and its Lipschitz constant ||2 A_c||_2."""
    A = np.zeros((prob.C, prob.M, prob.M), np.complex128)
    for c in range(prob.C):
        for l in range(prob.U):
            G = Uu[l] @ Wu[l] @ Uu[l].conj().T                # N x N
            Hlc = prob.Hs[l, c]
            A[c] += prob.alpha[l] * (Hlc.conj().T @ G @ Hlc)
    return A


def gradient_v(prob: Problem, Uu: np.ndarray, Wu: np.ndarray, Vu: np.ndarray,
               A: Optional[np.ndarray] = None) -> np.ndarray:
    """Block gradient of f in V (Section V-A):
    grad_u = (sum_l 2 alpha_l H_{l,c(u)}^H U_l W_l U_l^H H_{l,c(u)}) V_u
             - 2 alpha_u H_{u,c(u)}^H U_u W_u.
    The factor 2 follows the real inner product of Definition 1."""
    if A is None:
        A = transmit_hessians(prob, Uu, Wu)
    Hs = prob.H_serving()
    g = np.zeros_like(Vu)
    for u in range(prob.U):
        c = prob.cell[u]
        g[u] = 2.0 * A[c] @ Vu[u] - 2.0 * prob.alpha[u] * (Hs[u].conj().T @ Uu[u] @ Wu[u])
    return g


def step_sizes(A: np.ndarray) -> np.ndarray:
    """gamma_c = 1 / ||2 A_c||_2 (adaptive step, equation for gamma), by a dense
    Hermitian eigenvalue solve of the M x M matrix."""
    out = np.zeros(A.shape[0])
    for c in range(A.shape[0]):
        lam = np.linalg.eigvalsh(2.0 * 0.5 * (A[c] + A[c].conj().T)).max()
        out[c] = 1.0 / lam if lam > 0 else 0.0
    return out


def step_bound(prob: Problem) -> np.ndarray:
    """Lhat_c = 2 lambda_max(sum_u (alpha_u / sigma2_u) H_{u,c}^H H_{u,c}) per BS,
    the sum running over every user (all cells).  With U_u W_u U_u^H <= I /
    sigma2_u (Section VI, proof of Lemma 3, for W = E^{-1}; for W = I from
    sigma2 U^H U <= E <= I at the MMSE receiver), A_c <= sum_u (alpha_u /
    sigma2_u) H_{u,c}^H H_{u,c} in the Loewner order, so ||2 A_c||_2 <= Lhat_c
    for every iterate; Lhat_c <= 2 alpha_max U kappa / sigma2_min (Lemma 3)."""
    out = np.zeros(prob.C)
    for c in range(prob.C):
        B = np.zeros((prob.M, prob.M), np.complex128)
        for u in range(prob.U):
            Huc = prob.Hs[u, c]
            B += (prob.alpha[u] / prob.sigma2[u]) * (Huc.conj().T @ Huc)
        out[c] = 2.0 * np.linalg.eigvalsh(0.5 * (B + B.conj().T)).max()
    return out


def project_spc(prob: Problem, Vu: np.ndarray) -> np.ndarray:
    """Projection onto each BS's sum-power ball (projection equation, Section V-A):
    unchanged if sum_{u in c} ||V_u||_F^2 <= P_c, else scaled by sqrt(P_c / power)."""
    out = Vu.copy()
    for c in range(prob.C):
        users = np.nonzero(prob.cell == c)[0]
        p = float(sum(np.vdot(Vu[u], Vu[u]).real for u in users))
        if p > prob.P[c]:
            s = math.sqrt(prob.P[c] / p)
            out[users] = Vu[users] * s
    return out


def omega_schedule(t: int) -> float:
    """Extrapolation weight omega^t = max{(t-2)/(t+1), 0} (equation for omega)."""
    return max((t - 2.0) / (t + 1.0), 0.0)


def rel_change(a: float, b: float) -> float:
    """|a - b| / b, the relative WSR change of Algorithms 2 and 3."""
    if b > 0:
        return abs(a - b) / b
    return 0.0 if a == b else math.inf


def _inv_hermitian(E: np.ndarray) -> np.ndarray:
    W = np.linalg.inv(E)
    return 0.5 * (W + np.conj(np.swapaxes(W, -1, -2)))


def ammmse(prob: Problem, V0u: np.ndarray, iters: int, eps1: float = 0.1, eps2: float = 0.0,
           Tc: int = 3, gamma_c: Optional[float] = None, extrapolate: bool = True,
           warm_start: bool = True, force_switch_iter: Optional[int] = None,
           rearm_at_switch: bool = True, step_rule: str = "bound", perturb=None) -> dict:
    """A-MMMSE (Algorithm 3), FP64, one instance.

    Per iteration t = 1..iters:
      1. omega^t and the extrapolated point V^ = V^{t-1} + omega^t (V^{t-1} - V^{t-2})
         (V^ = V^{t-1} for t = 1);
      2. U^t by the receiver equation at V^{t-1} (R1);
      3. stage latch: stage I -> II when the relative WSR change between
         V^{t-1} and V^{t-2} is <= eps1 (R3, R4);
      4. W^t = (I - U^H H V^{t-1})^{-1} in stage II, I in stage I;
      5. for t <= Tc (and the first Tc stage-II iterations, R5),
         gamma_c = 1/||2 A_c||_2 per BS; afterwards the last adaptive value
         in stage I and 1 / Lhat_c (``step_bound``) in stage II, or the last
         adaptive value in both stages with step_rule="frozen" (R5, R6);
      6. V^t = Pi_P(V^ - gamma grad f(U^t, W^t, V^)) (R2).
    Returns the final precoders, the WSR trace WSR(V^0..V^T) in bits, the
    iteration of the stage switch (-1 if none) and the number of iterations run.
    ``force_switch_iter = s`` makes the first stage-II iteration exactly s.
    ``warm_start=False`` runs stage II from t = 1 (A-WMMSE).  With Tc = 0 a
    positive ``gamma_c`` must be given.  ``perturb(t, V)``, if given, replaces
    every new iterate V^t by its return value; the tests use it to measure how
    strongly a trajectory amplifies rounding-sized perturbations."""
    if Tc <= 0 and not (gamma_c is not None and gamma_c > 0):
        raise ValueError("Tc = 0 needs a positive fixed step gamma_c")
    if step_rule not in ("bound", "frozen"):
        raise ValueError("step_rule must be 'bound' or 'frozen'")
    bound = None
    V_prev = V0u.copy()
    V_prev2 = V0u.copy()
    trace = [wsr_bits(prob, V_prev)]
    if force_switch_iter is not None:
        stage2 = force_switch_iter <= 1
    else:
        stage2 = not warm_start
    switch_iter = 1 if stage2 else -1
    prev_step_stage2 = False
    gamma = np.zeros(prob.C)
    gammas = []
    Id = np.eye(prob.d)
    iters_run = 0
    for t in range(1, iters + 1):
        if (eps2 > 0 and t >= 2 and prev_step_stage2
                and rel_change(trace[t - 1], trace[t - 2]) <= eps2):
            break
        omega = omega_schedule(t) if extrapolate else 0.0
        Vhat = V_prev + omega * (V_prev - V_prev2) if t >= 2 else V_prev.copy()
        Uu = mmse_receivers(prob, V_prev)
        if not stage2:
            if force_switch_iter is not None:
                trigger = t >= force_switch_iter
            else:
                trigger = t >= 2 and rel_change(trace[t - 1], trace[t - 2]) <= eps1
            if trigger:
                stage2 = True
                switch_iter = t
        if stage2:
            Wu = _inv_hermitian(mse_at_mmse(prob, Uu, V_prev))
        else:
            Wu = np.broadcast_to(Id, (prob.U, prob.d, prob.d)).copy()
        A = transmit_hessians(prob, Uu, Wu)
        adaptive = t <= Tc or (rearm_at_switch and switch_iter >= 1
                                and switch_iter <= t < switch_iter + Tc)
        if adaptive:
            gamma = step_sizes(A)
        elif gamma_c is not None and gamma_c > 0:
            gamma = np.full(prob.C, float(gamma_c))
        elif stage2 and step_rule == "bound":
            if bound is None:
                bound = step_bound(prob)
            gamma = np.where(bound > 0, 1.0 / np.where(bound > 0, bound, 1.0), 0.0)
        gammas.append(gamma.copy())
        grad = gradient_v(prob, Uu, Wu, Vhat, A)
        V_new = project_spc(prob, Vhat - gamma[prob.cell][:, None, None] * grad)
        if perturb is not None:
            V_new = perturb(t, V_new)
        V_prev2, V_prev = V_prev, V_new
        trace.append(wsr_bits(prob, V_new))
        prev_step_stage2 = stage2
        iters_run = t
    return dict(V=V_prev, wsr=trace[-1], trace=np.array(trace), switch_iter=switch_iter,
                iters=iters_run, gammas=np.array(gammas))


# ---------------------------------------------------------------------------
# WMMSE (Algorithm 2) with the dual bisection of the V equation
# ---------------------------------------------------------------------------

def wmmse_precoder(prob: Problem, Uu: np.ndarray, Wu: np.ndarray, mode: str = "reference"
                   ) -> tuple:
    """V update of WMMSE (equation for V with dual lambda_c, Section IV).

    Per BS: A_c as in ``transmit_hessians``, B_u = alpha_u H_{u,c}^H U_u W_u,
    V_u(lambda) = (A_c + lambda I)^{-1} B_u.  lambda_c = 0 when the
    (pseudo-inverse) solution already meets the budget, otherwise bisection on
    the power p(lambda) = sum_m phi_m / (Lambda_m + lambda)^2 with A_c = Q Lambda Q^H
    and phi = row norms of Q^H B.  ``mode="paper"`` stops at interval width
    1e-4 or 100 probes (Section VII-A); ``mode="reference"`` at relative width
    1e-12 or 200 probes.  The feasible end of the interval is returned."""
    A = transmit_hessians(prob, Uu, Wu)
    Hs = prob.H_serving()
    V = np.zeros((prob.U, prob.M, prob.d), np.complex128)
    lambdas = np.zeros(prob.C)
    for c in range(prob.C):
        users = np.nonzero(prob.cell == c)[0]
        if users.size == 0:
            continue
        B = np.concatenate([prob.alpha[u] * (Hs[u].conj().T @ Uu[u] @ Wu[u]) for u in users],
                           axis=1)
        Ac = 0.5 * (A[c] + A[c].conj().T)
        lam, Q = np.linalg.eigh(Ac)
        Phi = Q.conj().T @ B
        phi = np.sum(np.abs(Phi) ** 2, axis=1)
        pos = lam > 1e-12 * max(lam.max(), 0.0)
        p0 = float(np.sum(phi[pos] / lam[pos] ** 2))
        if p0 <= prob.P[c]:
            mu = 0.0
            inv = np.where(pos, 1.0 / np.where(pos, lam, 1.0), 0.0)
        else:
            lo, hi = 0.0, math.sqrt(float(phi.sum()) / prob.P[c])
            probes = 0
            max_probes = 100 if mode == "paper" else 200
            while probes < max_probes:
                if mode == "paper" and hi - lo < 1e-4:
                    break
                if mode != "paper" and hi - lo <= 1e-12 * hi:
                    break
                mid = 0.5 * (lo + hi)
                if float(np.sum(phi / (lam + mid) ** 2)) > prob.P[c]:
                    lo = mid
                else:
                    hi = mid
                probes += 1
            mu = hi
            inv = 1.0 / (lam + mu)
        Vc = Q @ (inv[:, None] * Phi)
        lambdas[c] = mu
        for k, u in enumerate(users):
            V[u] = Vc[:, k * prob.d:(k + 1) * prob.d]
    return V, lambdas


def wmmse(prob: Problem, V0u: np.ndarray, max_iters: int = 500, eps: float = 1e-6,
          mode: str = "reference", perturb=None) -> dict:
    """WMMSE (Algorithm 2): U by the receiver equation, W = E^{-1}, V by the
    dual-bisection solve, until the relative WSR change is <= eps.
    ``perturb(t, V)``, if given, replaces every new iterate (a test hook that
    measures how strongly a trajectory amplifies rounding-sized changes)."""
    V = V0u.copy()
    trace = [wsr_bits(prob, V)]
    it = 0
    for t in range(1, max_iters + 1):
        Uu = mmse_receivers(prob, V)
        Wu = _inv_hermitian(mse_at_mmse(prob, Uu, V))
        V, _ = wmmse_precoder(prob, Uu, Wu, mode)
        if perturb is not None:
            V = perturb(t, V)
        trace.append(wsr_bits(prob, V))
        it = t
        if rel_change(trace[-1], trace[-2]) <= eps:
            break
    return dict(V=V, wsr=trace[-1], trace=np.array(trace), iters=it)


def mmmse(prob: Problem, V0u: np.ndarray, max_iters: int = 500, eps1: float = 0.1,
          eps2: float = 1e-6, mode: str = "reference", force_switch_iter: Optional[int] = None
          ) -> dict:
    """MMMSE (Section V-B, mixed weighted-unweighted sum-MSE): stage I is BCD on
    the sum-MSE problem (W = I: U by the receiver equation, V by the
    eq:mmse_Vk solve with its dual mu found by bisection, i.e. the WMMSE V step
    with W = I); once the relative WSR change between V^{t-1} and V^{t-2} is
    <= eps1 (tested at the start of iteration t, as in Algorithm 3) iteration t
    and the later ones are WMMSE iterations (W = E^{-1}); stop once a stage-II
    step changes the WSR by <= eps2 (relative) or after max_iters."""
    V = V0u.copy()
    trace = [wsr_bits(prob, V)]
    stage2 = force_switch_iter is not None and force_switch_iter <= 1
    switch = 1 if stage2 else -1
    prev_stage2 = False
    it = 0
    for t in range(1, max_iters + 1):
        if prev_stage2 and t >= 2 and rel_change(trace[-1], trace[-2]) <= eps2:
            break
        if not stage2:
            trig = (t >= force_switch_iter) if force_switch_iter is not None else \
                (t >= 2 and rel_change(trace[-1], trace[-2]) <= eps1)
            if trig:
                stage2, switch = True, t
        Uu = mmse_receivers(prob, V)
        if stage2:
            Wu = _inv_hermitian(mse_at_mmse(prob, Uu, V))
        else:
            Wu = np.stack([np.eye(prob.d, dtype=np.complex128)] * prob.U)
        V, _ = wmmse_precoder(prob, Uu, Wu, mode)
        trace.append(wsr_bits(prob, V))
        prev_stage2 = stage2
        it = t
    return dict(V=V, wsr=trace[-1], trace=np.array(trace), iters=it, switch_iter=switch)


# ---------------------------------------------------------------------------
# BCGD-WMMSE (Section VII-F ablation): every block by one explicit step
# ---------------------------------------------------------------------------

def rx_covariances(prob: Problem, Vu: np.ndarray) -> np.ndarray:
    """J_u = sum_l H_{u,c(l)} V_l V_l^H H_{u,c(l)}^H + sigma2_u I (all users l,
    the matrix inverted by the receiver equation of Section IV): [U, N, N]."""
    T = cross_terms(prob, Vu)
    J = _covariances(T).sum(axis=1)
    return J + prob.sigma2[:, None, None] * np.eye(prob.N)[None]


def receiver_gradient(prob: Problem, Uu: np.ndarray, Wu: np.ndarray, Vu: np.ndarray) -> np.ndarray:
    """Block gradient of f in U_u (Definition 1 inner product): f depends on
    U_u through alpha_u Tr(W_u E_u) with E_u = I - U^H H V_u - V_u^H H^H U +
    U^H J_u U, so grad_u = 2 alpha_u (J_u U_u W_u - H_{u,c(u)} V_u W_u)."""
    J = rx_covariances(prob, Vu)
    G = np.einsum("unm,umd->und", prob.H_serving(), Vu)
    return 2.0 * prob.alpha[:, None, None] * (J @ Uu @ Wu - G @ Wu)


def schulz_step(W: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Schulz iteration for E^{-1} (Section VII-F): W (2I - E W), symmetrised."""
    I = np.eye(W.shape[-1])
    Wn = W @ (2.0 * I - E @ W)
    return 0.5 * (Wn + np.conj(np.swapaxes(Wn, -1, -2)))


def bcgd_wmmse(prob: Problem, V0u: np.ndarray, iters: int, Tc: int = 3,
               extrapolate: bool = True, step_rule: str = "bound", eps2: float = 0.0) -> dict:
    """BCGD-WMMSE, the full block-coordinate gradient method of the ablation
    in Section VII-F: U, W and V each take one explicit step per iteration.
    Readings (the section fixes only the W update):
      * start: U^0 the MMSE receivers at V^0 and W^0 = E(U^0, V^0)^{-1};
      * U step: U^t = U^{t-1} - gu_u grad_U f(U^{t-1}, W^{t-1}, V^{t-1}) with
        gu_u = 1 / (2 alpha_u ||J_u||_F ||W_u||_F), J_u the receive covariance
        at V^{t-1}; ||.||_F bounds the spectral norms of the block Lipschitz
        constant 2 alpha_u lambda_max(J_u) lambda_max(W_u) without an
        eigenvalue solve;
      * W step: W^t = W^{t-1} (2I - E_u W^{t-1}) with E_u the MSE matrix of
        (U^t, V^{t-1}) (general definition, Section IV);
      * V step: as Algorithm 3's second stage, at the extrapolated point with
        (U^t, W^t): adaptive step 1/||2 A_c|| for t <= Tc, then 1 / Lhat_c
        (step_rule "bound") or the last adaptive value ("frozen");
      * eps2 > 0: stop before iteration t >= 2 when the relative WSR change
        between V^{t-1} and V^{t-2} is <= eps2 (every step is a second-stage
        step here).
    Returns the final precoders and the WSR trace WSR(V^0..V^T) in bits."""
    if step_rule not in ("bound", "frozen"):
        raise ValueError("step_rule must be 'bound' or 'frozen'")
    V_prev = V0u.copy()
    V_prev2 = V0u.copy()
    Uu = mmse_receivers(prob, V_prev)
    Wu = _inv_hermitian(mse_matrices(prob, Uu, V_prev))
    trace = [wsr_bits(prob, V_prev)]
    gamma = np.zeros(prob.C)
    bound = None
    iters_run = 0
    for t in range(1, iters + 1):
        if eps2 > 0 and t >= 2 and rel_change(trace[t - 1], trace[t - 2]) <= eps2:
            break
        omega = omega_schedule(t) if extrapolate else 0.0
        Vhat = V_prev + omega * (V_prev - V_prev2) if t >= 2 else V_prev.copy()
        J = rx_covariances(prob, V_prev)
        gU = receiver_gradient(prob, Uu, Wu, V_prev)
        nJ = np.linalg.norm(J, axis=(1, 2))
        nW = np.linalg.norm(Wu, axis=(1, 2))
        den = 2.0 * prob.alpha * nJ * nW
        gu = np.where(den > 0, 1.0 / np.where(den > 0, den, 1.0), 0.0)
        Uu = Uu - gu[:, None, None] * gU
        Wu = schulz_step(Wu, mse_matrices(prob, Uu, V_prev))
        A = transmit_hessians(prob, Uu, Wu)
        if t <= Tc:
            gamma = step_sizes(A)
        elif step_rule == "bound":
            if bound is None:
                bound = step_bound(prob)
            gamma = np.where(bound > 0, 1.0 / np.where(bound > 0, bound, 1.0), 0.0)
        grad = gradient_v(prob, Uu, Wu, Vhat, A)
        V_new = project_spc(prob, Vhat - gamma[prob.cell][:, None, None] * grad)
        V_prev2, V_prev = V_prev, V_new
        trace.append(wsr_bits(prob, V_new))
        iters_run = t
    return dict(V=V_prev, U=Uu, W=Wu, wsr=trace[-1], trace=np.array(trace), iters=iters_run)


# ---------------------------------------------------------------------------
# Stationarity and constants (Section VI)
# ---------------------------------------------------------------------------

def kappa(prob: Problem) -> float:
    """kappa = max over all user-BS pairs of sigma_max(H^H H) (Section VI; the
    maximum runs over every channel so that the Lemma 3 bound covers
    multi-cell interference terms)."""
    return float(max(np.linalg.norm(prob.Hs[u, c], 2) ** 2
                     for u in range(prob.U) for c in range(prob.C)))


def kkt_residual(prob: Problem, Vu: np.ndarray) -> float:
    """Stationarity residual of V for the sum-power-constrained problem
    (Definition 2): with g = grad f at the MMSE receivers and W = E^{-1}, per BS
    min_{lambda >= 0} ||g_c + 2 lambda V_c||_F / ||g_c||_F, with lambda = 0
    forced when the budget is not active.  Returns the largest over BSs."""
    Uu = mmse_receivers(prob, Vu)
    Wu = _inv_hermitian(mse_at_mmse(prob, Uu, Vu))
    g = gradient_v(prob, Uu, Wu, Vu)
    worst = 0.0
    for c in range(prob.C):
        users = np.nonzero(prob.cell == c)[0]
        if users.size == 0:
            continue
        gc = g[users].ravel()
        vc = Vu[users].ravel()
        p = float(np.vdot(vc, vc).real)
        gn = float(np.linalg.norm(gc))
        if gn == 0.0:
            continue
        lam = 0.0
        if p >= prob.P[c] * (1.0 - 1e-9) and p > 0:
            lam = max(0.0, -float(np.vdot(vc, gc).real) / (2.0 * p))
        worst = max(worst, float(np.linalg.norm(gc + 2.0 * lam * vc)) / gn)
    return worst


# ---------------------------------------------------------------------------
# Batch driver (process pool over instances, one BLAS thread per worker)
# ---------------------------------------------------------------------------

def _solve_one(args):
    inst, algo, kw = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover - threadpoolctl is optional
        pass
    prob = from_instance(inst)
    V0 = split_v(prob, inst["V0"])
    if algo == "ammmse":
        r = ammmse(prob, V0, **kw)
    elif algo == "wmmse":
        r = wmmse(prob, V0, **kw)
    elif algo == "mmmse":
        r = mmmse(prob, V0, **kw)
    elif algo == "bcgd_wmmse":
        r = bcgd_wmmse(prob, V0, **kw)
    elif algo == "wsr":
        r = dict(wsr=wsr_bits(prob, V0), V=V0)
    else:
        raise ValueError(algo)
    r["V_blocks"] = join_v(prob, r["V"])
    del r["V"]
    return r


def solve_batch(instances: Sequence[dict], algo: str, workers: int = 1, **kw) -> list:
    """Run ``algo`` ("ammmse", "wmmse" or "wsr") on every instance dict; with
    ``workers > 1`` a process pool spreads instances over host cores."""
    jobs = [(inst, algo, kw) for inst in instances]
    if workers <= 1:
        return [_solve_one(j) for j in jobs]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        return pool.map(_solve_one, jobs, chunksize=max(1, len(jobs) // (4 * workers)))
