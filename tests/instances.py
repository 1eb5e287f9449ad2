"""Small hand-built problem instances for the tests (no method arithmetic)."""
import math

import numpy as np

from paper_2510_20507_amd import synth


def instance(H, sigma2, alpha, P, cell_users, N, d, V0):
    """Per-instance dict in the layout of ``synth.Batch.instance``."""
    U = int(sum(cell_users))
    return dict(C=len(H), U=U, M=int(H[0].shape[1]), N=N, d=d, cell_users=list(cell_users),
                H=[np.asarray(h, np.complex128) for h in H],
                V0=[np.asarray(v, np.complex128) for v in V0],
                sigma2=np.broadcast_to(np.asarray(sigma2, float), (U,)).copy(),
                alpha=np.broadcast_to(np.asarray(alpha, float), (U,)).copy(),
                P=np.broadcast_to(np.asarray(P, float), (len(H),)).copy())


def random_instance(seed, M, cell_users, N, d, P=10.0, sigma2=1.0, alpha_range=None):
    rng = np.random.default_rng(seed)
    return synth.rayleigh_instance(rng, M, cell_users, N, d, P, sigma2, alpha_range)


def water_filling(gains, P, sigma2):
    """Textbook water-filling over parallel channels with power gains g_i:
    p_i = (mu - sigma2/g_i)^+, sum p_i = P; returns (p, capacity in bits)."""
    g = np.asarray(gains, float)
    order = np.argsort(-g)
    gs = g[order]
    for k in range(len(gs), 0, -1):
        mu = (P + np.sum(sigma2 / gs[:k])) / k
        if mu - sigma2 / gs[k - 1] > 0:
            break
    p = np.maximum(mu - sigma2 / g, 0.0)
    return p, float(np.sum(np.log2(1.0 + p * g / sigma2)))


def weighted_water_filling(gains, alpha, P, sigma2):
    """max sum_u alpha_u log(1 + p_u g_u / sigma2) s.t. sum p_u = P:
    p_u = (alpha_u / nu - sigma2 / g_u)^+, nu found by bisection on the budget.
    Returns (p, weighted sum rate in bits)."""
    g = np.asarray(gains, float)
    a = np.asarray(alpha, float)
    lo, hi = 1e-300, 1e300
    for _ in range(3000):
        nu = math.sqrt(lo * hi)
        p = np.maximum(a / nu - sigma2 / g, 0.0)
        if p.sum() > P:
            lo = nu
        else:
            hi = nu
        if hi / lo < 1 + 1e-15:
            break
    p = np.maximum(a / hi - sigma2 / g, 0.0)
    return p, float(np.sum(a * np.log2(1.0 + p * g / sigma2)))
