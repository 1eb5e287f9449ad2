"""Unrolled A-MMMSE and its gradient, FP64 (test infrastructure: only the
tests may import this module; the GPU path shares nothing with it).

The unrolled solver runs T iterations of Algorithm 3 on one single-cell
instance with the step size of iteration t supplied from outside (gamma_t,
the learnable step sizes of an unrolled network) instead of the adaptive
rule, the stage switch at a given iteration s (stage I, W = I, for t < s;
stage II, W = E^{-1}, for t >= s; s is decided by the eps1 rule in a plain
forward run and held fixed when differentiating), the extrapolation weight
omega^t and the projection onto the sum-power ball.  The output is the
weighted sum rate of V^T (Section II, bits).

Each step is written with torch complex128 operations in the paper's order
and notation (receiver equation by a linear solve, W = (I - U^H H V)^{-1},
the block gradient of Section V-A, the projection equation); gradients with
respect to the step sizes and the channel come from torch.autograd (the
library's reverse-mode differentiation stands in for the hand derivation).
The switch and the projection branch are piecewise constant and not
differentiated.

Gradient convention: for a real loss L and a complex input z, torch stores
z.grad = dL/dRe(z) + i dL/dIm(z), so that dL = Re(sum(conj(z.grad) * dz)).
"""
from typing import Sequence

import numpy as np
import torch

LN2 = float(np.log(2.0))


def omega(t: int) -> float:
    """Extrapolation weight omega^t = max{(t-2)/(t+1), 0}."""
    return max((t - 2.0) / (t + 1.0), 0.0)


def _herm(A):
    return 0.5 * (A + A.conj().transpose(-1, -2))


def wsr_bits(H, sigma2, alpha, V):
    """WSR (bits) of precoders V [U, M, d] for channels H [U, N, M] of one
    cell: R_u = log det(I + S_u J_u^{-1}), S_u the own-signal covariance and
    J_u the interference-plus-noise covariance (Section II rate)."""
    U, N, _ = H.shape
    T = torch.einsum("unm,lmd->ulnd", H, V)               # H_u V_l
    C = T @ T.conj().transpose(-1, -2)                     # [U, U, N, N]
    I = torch.eye(N, dtype=H.dtype)
    total = 0.0
    for u in range(U):
        Jm = sigma2[u] * I
        for l in range(U):
            if l != u:
                Jm = Jm + C[u, l]
        Su = C[u, u]
        R = torch.linalg.slogdet(I + Su @ torch.linalg.inv(Jm))[1]
        total = total + alpha[u] * R
    return total / LN2


def unrolled_wsr(H, sigma2, alpha, P: float, V0, gammas, switch_iter: int,
                 extrapolate: bool = True):
    """WSR(V^T) of T = len(gammas) unrolled A-MMMSE iterations (see the module
    docstring).  H [U, N, M] and V0 [U, M, d] complex128 tensors, gammas a
    real tensor [T]; stage II from iteration switch_iter (1: from the start,
    T + 1 or more: stage I throughout).  Returns (wsr, V^T, trace of
    WSR(V^0..V^{T-1}) as floats)."""
    U, N, M = H.shape
    d = V0.shape[2]
    Id = torch.eye(d, dtype=H.dtype)
    In = torch.eye(N, dtype=H.dtype)
    Vp, Vq = V0, V0                                         # V^{t-1}, V^{t-2}
    trace = []
    for t in range(1, len(gammas) + 1):
        w = omega(t) if extrapolate else 0.0
        Vh = Vp + w * (Vp - Vq)
        trace.append(float(wsr_bits(H, sigma2, alpha, Vp).detach()))
        # receivers at V^{t-1}: U_u = (sum_l H_u V_l V_l^H H_u^H + sigma2 I)^{-1} H_u V_u
        T = torch.einsum("unm,lmd->ulnd", H, Vp)
        Uu, Wu = [], []
        stage2 = t >= switch_iter
        for u in range(U):
            J = sigma2[u] * In
            for l in range(U):
                J = J + T[u, l] @ T[u, l].conj().T
            Ur = torch.linalg.solve(J, T[u, u])
            Uu.append(Ur)
            if stage2:
                E = _herm(Id - Ur.conj().T @ T[u, u])
                Wu.append(_herm(torch.linalg.inv(E)))
            else:
                Wu.append(Id)
        # block gradient at the extrapolated point (Section V-A)
        A = torch.zeros((M, M), dtype=H.dtype)
        for l in range(U):
            A = A + alpha[l] * (H[l].conj().T @ Uu[l] @ Wu[l] @ Uu[l].conj().T @ H[l])
        G = torch.stack([2.0 * A @ Vh[u] - 2.0 * alpha[u] * (H[u].conj().T @ Uu[u] @ Wu[u])
                         for u in range(U)])
        Vt = Vh - gammas[t - 1] * G
        p = torch.sum(torch.abs(Vt) ** 2)
        if float(p.detach()) > P:
            Vt = Vt * torch.sqrt(P / p)
        Vq, Vp = Vp, Vt
    return wsr_bits(H, sigma2, alpha, Vp), Vp, trace


def switch_iter(H: np.ndarray, sigma2: Sequence[float], alpha: Sequence[float], P: float,
                V0: np.ndarray, gammas: Sequence[float], eps1: float = 0.1,
                extrapolate: bool = True) -> int:
    """The stage-switch iteration the eps1 rule of Algorithm 3 picks for the
    unrolled solver with these step sizes: the first t >= 2 whose relative WSR
    change between V^{t-1} and V^{t-2} is <= eps1 (T + 1 if none).  Before the
    switch the iterates equal those of a run that stays in stage I, so the
    rule is applied to the trace of that run."""
    T = len(gammas)
    with torch.no_grad():
        _, _, trace = unrolled_wsr(torch.tensor(H, dtype=torch.complex128),
                                   torch.tensor(np.asarray(sigma2, float)),
                                   torch.tensor(np.asarray(alpha, float)), float(P),
                                   torch.tensor(V0, dtype=torch.complex128),
                                   torch.tensor(np.asarray(gammas, float)), T + 1, extrapolate)
    for t in range(2, T + 1):
        a, b = trace[t - 1], trace[t - 2]
        rel = abs(a - b) / b if b > 0 else (0.0 if a == b else float("inf"))
        if rel <= eps1:
            return t
    return T + 1


def value_and_grad(H: np.ndarray, sigma2: Sequence[float], alpha: Sequence[float], P: float,
                   V0: np.ndarray, gammas: Sequence[float], switch_iter: int,
                   extrapolate: bool = True):
    """WSR(V^T) and its gradients with respect to the step sizes (length T)
    and the channel (same shape as H, in the convention of the module
    docstring), from NumPy inputs."""
    Ht = torch.tensor(H, dtype=torch.complex128, requires_grad=True)
    gt = torch.tensor(np.asarray(gammas, float), dtype=torch.float64, requires_grad=True)
    s2 = torch.tensor(np.asarray(sigma2, float), dtype=torch.float64)
    al = torch.tensor(np.asarray(alpha, float), dtype=torch.float64)
    V0t = torch.tensor(V0, dtype=torch.complex128)
    wsr, VT, trace = unrolled_wsr(Ht, s2, al, float(P), V0t, gt, switch_iter, extrapolate)
    wsr.backward()
    return (float(wsr.detach()), gt.grad.numpy().copy(), Ht.grad.numpy().copy(),
            VT.detach().numpy(), np.array(trace))
