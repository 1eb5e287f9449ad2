"""Seeded synthetic workloads for multi-cell MU-MIMO downlink precoding.

This module only draws random numbers and lays them out; it contains none of
the precoding method's arithmetic.  Both the FP64 reference used by the tests
and the GPU library consume exactly the arrays produced here.

System model (Section II of the paper): C base stations (cells), each with M
antennas, serving U_c users with N receive antennas and d streams.  The
channel from BS j to user u is an N x M complex matrix H_{u,j}; the precoder of
user u is an M x d complex matrix V_u.

Flat layout shared by every consumer (complex elements are complex128 here;
the GPU side converts to its storage precision):

* ``H``: per instance, C blocks (one per BS c) of the stacked channel
  H_{:,c} = [H_{0,c}; H_{1,c}; ...] of shape (U*N) x M, row-major.
  Users are ordered cell by cell.
* ``V0``: per instance, C blocks of V_c = [V_u for u in cell c] of shape
  M x (U_c*d), row-major, so V_u[m, s] = V_c[m, i*d + s] for the i-th user of
  cell c.
* ``sigma2``, ``alpha``: per instance, U entries (noise power, priority weight).
* ``P``: per instance, C entries (sum-power budget of each BS).
* ``cell_users``: per instance, C entries (users per cell).

Random draws per instance follow a fixed order so that any subset of a batch
can be regenerated: H, then alpha, then V0 (plus geometry first for the
hexagonal layout).  Complex Gaussian CN(0,1) means real and imaginary parts
i.i.d. N(0, 1/2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 20507


def cn01(rng: np.random.Generator, shape) -> np.ndarray:
    """Draw circularly-symmetric CN(0,1) samples (re, im i.i.d. N(0, 1/2))."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * math.sqrt(0.5)


@dataclasses.dataclass
class Batch:
    """A batch of independent channel realisations in the flat layout."""

    C: np.ndarray          # int32 [B] cells
    U: np.ndarray          # int32 [B] users (all cells)
    M: np.ndarray          # int32 [B] BS antennas
    N: np.ndarray          # int32 [B] receive antennas
    d: np.ndarray          # int32 [B] streams per user
    cell_off: np.ndarray   # int32 [B] offset into cell_users
    h_off: np.ndarray      # int64 [B] complex elements
    v_off: np.ndarray      # int64 [B] complex elements
    user_off: np.ndarray   # int64 [B]
    bs_off: np.ndarray     # int64 [B]
    cell_users: np.ndarray  # int32 [sum C]
    H: np.ndarray          # complex128 flat
    sigma2: np.ndarray     # float64 flat [sum U]
    alpha: np.ndarray      # float64 flat [sum U]
    P: np.ndarray          # float64 flat [sum C]
    V0: np.ndarray         # complex128 flat
    name: str = ""

    @property
    def batch(self) -> int:
        return int(self.C.shape[0])

    def instance(self, b: int) -> dict:
        """Per-instance views: lists of per-BS blocks, as described above."""
        C, U, M, N, d = (int(x[b]) for x in (self.C, self.U, self.M, self.N, self.d))
        cu = [int(x) for x in self.cell_users[self.cell_off[b]: self.cell_off[b] + C]]
        h0, v0 = int(self.h_off[b]), int(self.v_off[b])
        H = [self.H[h0 + c * U * N * M: h0 + (c + 1) * U * N * M].reshape(U * N, M)
             for c in range(C)]
        V = []
        off = v0
        for c in range(C):
            n = M * cu[c] * d
            V.append(self.V0[off: off + n].reshape(M, cu[c] * d))
            off += n
        u0, s0 = int(self.user_off[b]), int(self.bs_off[b])
        return dict(C=C, U=U, M=M, N=N, d=d, cell_users=cu, H=H, V0=V,
                    sigma2=self.sigma2[u0: u0 + U].copy(),
                    alpha=self.alpha[u0: u0 + U].copy(),
                    P=self.P[s0: s0 + C].copy())

    def subset(self, idx: Sequence[int]) -> "Batch":
        """A new batch holding the listed instances (re-packed contiguously)."""
        insts = [self.instance(int(b)) for b in idx]
        return pack(insts, name=self.name + "[subset]")

    def total_flops_per_iter(self) -> np.ndarray:
        """Work per instance-iteration of the two channel products (8 flops per
        complex multiply-add): 2 * 8 * (U*N) * M * (U*d), summed over BSs of the
        per-BS products (U*N x M) by (M x U_c*d)."""
        return 16.0 * (self.U * self.N).astype(np.float64) * self.M * (self.U * self.d)


def pack(insts: List[dict], name: str = "") -> Batch:
    """Pack per-instance dicts (as returned by ``Batch.instance``) into a Batch."""
    B = len(insts)
    C = np.array([i["C"] for i in insts], np.int32)
    U = np.array([i["U"] for i in insts], np.int32)
    M = np.array([i["M"] for i in insts], np.int32)
    N = np.array([i["N"] for i in insts], np.int32)
    d = np.array([i["d"] for i in insts], np.int32)
    cell_off = np.zeros(B, np.int32)
    h_off = np.zeros(B, np.int64)
    v_off = np.zeros(B, np.int64)
    user_off = np.zeros(B, np.int64)
    bs_off = np.zeros(B, np.int64)
    cu, Hs, Vs, s2, al, Ps = [], [], [], [], [], []
    co = ho = vo = uo = so = 0
    for b, inst in enumerate(insts):
        cell_off[b], h_off[b], v_off[b], user_off[b], bs_off[b] = co, ho, vo, uo, so
        cu.extend(inst["cell_users"])
        for Hc in inst["H"]:
            Hs.append(np.ascontiguousarray(Hc, np.complex128).ravel())
            ho += Hc.size
        for Vc in inst["V0"]:
            Vs.append(np.ascontiguousarray(Vc, np.complex128).ravel())
            vo += Vc.size
        s2.append(np.asarray(inst["sigma2"], np.float64))
        al.append(np.asarray(inst["alpha"], np.float64))
        Ps.append(np.asarray(inst["P"], np.float64))
        co += inst["C"]
        uo += inst["U"]
        so += inst["C"]
    cat = lambda xs, dt: (np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return Batch(C=C, U=U, M=M, N=N, d=d, cell_off=cell_off, h_off=h_off, v_off=v_off,
                 user_off=user_off, bs_off=bs_off,
                 cell_users=np.array(cu, np.int32), H=cat(Hs, np.complex128),
                 sigma2=cat(s2, np.float64), alpha=cat(al, np.float64), P=cat(Ps, np.float64),
                 V0=cat(Vs, np.complex128), name=name)


def scale_to_power(X: np.ndarray, P: float) -> np.ndarray:
    """Feasible initial precoder: a random block scaled so its power is exactly P."""
    p = float(np.vdot(X, X).real)
    return X * math.sqrt(P / p) if p > 0 else X


def rayleigh_instance(rng: np.random.Generator, M: int, cell_users: Sequence[int], N: int,
                      d: int, P, sigma2: float = 1.0,
                      alpha_range: Optional[tuple] = None) -> dict:
    """i.i.d. Rayleigh channels, CN(0,1) entries; draw order H, alpha, V0."""
    C = len(cell_users)
    U = int(sum(cell_users))
    H = [cn01(rng, (U * N, M)) for _ in range(C)]
    if alpha_range is None:
        alpha = np.ones(U)
    else:
        alpha = rng.uniform(alpha_range[0], alpha_range[1], size=U)
    Pv = np.broadcast_to(np.asarray(P, np.float64), (C,)).copy()
    V0 = [scale_to_power(cn01(rng, (M, cell_users[c] * d)), Pv[c]) for c in range(C)]
    return dict(C=C, U=U, M=M, N=N, d=d, cell_users=list(cell_users), H=H, V0=V0,
                sigma2=np.full(U, float(sigma2)), alpha=alpha, P=Pv)


def rayleigh_batch(seed: int, B: int, M: int, U: int, N: int, d: int, P: float,
                   sigma2: float = 1.0, alpha_range: Optional[tuple] = None,
                   name: str = "") -> Batch:
    """Single-cell batch of B instances with identical shapes."""
    rng = np.random.default_rng(seed)
    insts = [rayleigh_instance(rng, M, [U], N, d, P, sigma2, alpha_range) for _ in range(B)]
    return pack(insts, name=name)


def db_to_lin(db: float) -> float:
    return 10.0 ** (db / 10.0)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def single_small(seed: int = BASE_SEED + 1000) -> Batch:
    """One instance, single cell: M=8, 4 users, N=2, d=2, sigma2=1, P=10, alpha=1."""
    return rayleigh_batch(seed, 1, M=8, U=4, N=2, d=2, P=10.0, name="single_small_m8u4n2d2")


SWEEP_DB = (0.0, 10.0, 20.0, 30.0)


def rayleigh_sweep(B_per_p: int = 256, seed_base: int = BASE_SEED + 2000,
                   M: int = 64, U: int = 16, N: int = 4, d: int = 4,
                   sweep_db: Sequence[float] = SWEEP_DB) -> Batch:
    """Single-cell Rayleigh batch, B_per_p instances for each SNR in the sweep.

    M=64, 16 users, N=4, d=4, sigma2=1, alpha ~ U[0.5, 1.5], P in {0,10,20,30} dB.
    The sweep index k uses seed ``seed_base + k``; instances are concatenated
    in sweep order."""
    parts = []
    for k, db in enumerate(sweep_db):
        rng = np.random.default_rng(seed_base + k)
        parts.extend(rayleigh_instance(rng, M, [U], N, d, db_to_lin(db), 1.0, (0.5, 1.5))
                     for _ in range(B_per_p))
    return pack(parts, name=f"rayleigh_m{M}u{U}n{N}d{d}_sweep{len(sweep_db)}x{B_per_p}")


def rayleigh_large(B: int = 512, seed: int = BASE_SEED + 4000) -> Batch:
    """Single-cell Rayleigh batch: M=256, 64 users, N=2, d=2, P=20 dB,
    sigma2=1, alpha ~ U[0.5, 1.5]."""
    return rayleigh_batch(seed, B, M=256, U=64, N=2, d=2, P=100.0, alpha_range=(0.5, 1.5),
                          name=f"rayleigh_m256u64n2d2_b{B}")


# --- 7-cell hexagonal layout with path loss and shadowing -------------------

HEX_ISD_M = 500.0
HEX_MIN_DIST_M = 35.0
HEX_SHADOW_DB = 8.0
HEX_NOISE_W = 10.0 ** ((-174.0 + 10.0 * math.log10(10e6)) / 10.0) * 1e-3   # -104 dBm
HEX_P_W = 10.0 ** (46.0 / 10.0) * 1e-3                                      # 46 dBm


def hex_sites(isd: float = HEX_ISD_M) -> np.ndarray:
    """Centre site plus the first ring of six at distance ``isd`` (metres)."""
    pts = [(0.0, 0.0)]
    for k in range(6):
        ang = math.pi / 6 + k * math.pi / 3
        pts.append((isd * math.cos(ang), isd * math.sin(ang)))
    return np.array(pts)


def _uniform_in_hexagon(rng: np.random.Generator, R: float, min_dist: float) -> np.ndarray:
    """Uniform point in a hexagon of circumradius R centred at 0 (flat-topped
    vertices at angles 0, 60, ...), at least ``min_dist`` from the centre.
    Rejection sampling from the bounding box."""
    h = R * math.sqrt(3.0) / 2.0
    while True:
        x = rng.uniform(-R, R)
        y = rng.uniform(-h, h)
        ax, ay = abs(x), abs(y)
        inside = ay <= h and (math.sqrt(3.0) * ax + ay) <= math.sqrt(3.0) * R
        if inside and math.hypot(x, y) >= min_dist:
            return np.array([x, y])


def pathloss_db(dist_m: np.ndarray) -> np.ndarray:
    """128.1 + 37.6 log10(distance in km) dB."""
    return 128.1 + 37.6 * np.log10(np.asarray(dist_m) / 1000.0)


def hexcell_instance(rng: np.random.Generator) -> dict:
    """One 7-cell instance.  Draw order: M, N, users per cell, user positions,
    shadowing, small-scale fading, V0.  d = min(N, 2); alpha = 1."""
    M = int(rng.choice([16, 32, 64, 128]))
    N = int(rng.choice([1, 2, 4]))
    d = min(N, 2)
    C = 7
    cell_users = [int(x) for x in rng.integers(2, 13, size=C)]
    U = sum(cell_users)
    sites = hex_sites()
    R = HEX_ISD_M / math.sqrt(3.0)          # hexagon circumradius
    pos = []
    for c in range(C):
        for _ in range(cell_users[c]):
            pos.append(sites[c] + _uniform_in_hexagon(rng, R, HEX_MIN_DIST_M))
    pos = np.array(pos)                                          # [U, 2]
    dist = np.linalg.norm(pos[:, None, :] - sites[None, :, :], axis=2)   # [U, C]
    dist = np.maximum(dist, HEX_MIN_DIST_M)
    shadow = rng.standard_normal((U, C)) * HEX_SHADOW_DB
    gain_amp = 10.0 ** (-(pathloss_db(dist) + shadow) / 20.0)       # [U, C]
    H = []
    for c in range(C):
        Hc = cn01(rng, (U * N, M))
        Hc *= np.repeat(gain_amp[:, c], N)[:, None]
        H.append(Hc)
    alpha = np.ones(U)
    P = np.full(C, HEX_P_W)
    V0 = [scale_to_power(cn01(rng, (M, cell_users[c] * d)), P[c]) for c in range(C)]
    return dict(C=C, U=U, M=M, N=N, d=d, cell_users=cell_users, H=H, V0=V0,
                sigma2=np.full(U, HEX_NOISE_W), alpha=alpha, P=P)


def hexcell_batch(B: int = 4096, seed: int = BASE_SEED + 3000) -> Batch:
    """Uneven batch: 7-cell hexagonal layout, ISD 500 m, per-instance
    M in {16,32,64,128}, N in {1,2,4}, d=min(N,2), users per cell U{2..12},
    path loss 128.1+37.6 log10(d_km) dB, 8 dB log-normal shadowing,
    noise -174 dBm/Hz over 10 MHz, 46 dBm per BS."""
    rng = np.random.default_rng(seed)
    return pack([hexcell_instance(rng) for _ in range(B)], name=f"hexcell7_b{B}")


def unrolled_batch(B: int = 1024, seed: int = BASE_SEED + 5000) -> Batch:
    """Single-cell Rayleigh batch for unrolled differentiation: M=64, 16 users,
    N=4, d=4, P=20 dB, sigma2=1, alpha ~ U[0.5, 1.5]."""
    return rayleigh_batch(seed, B, M=64, U=16, N=4, d=4, P=100.0, alpha_range=(0.5, 1.5),
                          name=f"rayleigh_m64u16n4d4_p20_b{B}")
