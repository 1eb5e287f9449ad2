// Device-side helpers shared by the solve kernels of libammse (gfx950).
#pragma once

#include <math.h>

#include "ammse_internal.h"

namespace ammse_dev {


template <class R>
struct cx {
  R x, y;
};

template <class R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R>
__device__ __forceinline__ cx<R> scal(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <class R>
__device__ __forceinline__ cx<R> cj(cx<R> a) { return {a.x, -a.y}; }
// a * conj(b)
template <class R>
__device__ __forceinline__ cx<R> mulc(cx<R> a, cx<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <class R>
__device__ __forceinline__ R nrm2(cx<R> a) { return a.x * a.x + a.y * a.y; }

using zd = cx<double>;

template <class R>
__device__ __forceinline__ zd to_d(cx<R> a) { return {(double)a.x, (double)a.y}; }
template <class R>
__device__ __forceinline__ cx<R> from_d(zd a) { return {(R)a.x, (R)a.y}; }

template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)u, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave (all lanes active); every lane receives the
// same value: DPP moves within each 16-lane row, then the four row sums.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp64<0xB1>(v);     // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);     // quad_perm [2,3,0,1]
  v += dpp64<0x124>(v);    // row_ror 4
  v += dpp64<0x128>(v);    // row_ror 8
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum over the 16 lanes of each DPP row (every lane of the row receives it).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp64<0xB1>(v);     // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);     // quad_perm [2,3,0,1]
  v += dpp64<0x124>(v);    // row_ror 4
  v += dpp64<0x128>(v);    // row_ror 8
  return v;
}

// Sum over the block (a multiple of 64 threads, at most 512); every thread
// receives the same value.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}


// ---------------------------------------------------------------------------
// 4 x 4 complex double helpers (row-major, fully unrolled)
// ---------------------------------------------------------------------------

// In-place Cholesky A = L L^H (lower); false if a pivot is not positive/finite.
__device__ __forceinline__ bool chol4(zd* A) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double s = A[j * 4 + j].x;
#pragma unroll
    for (int k = 0; k < j; ++k) s -= nrm2(A[j * 4 + k]);
    ok = ok && (s > 0.0) && isfinite(s);
    const double l = sqrt(fmax(s, 1e-300));
    const double il = 1.0 / l;
    A[j * 4 + j] = {l, 0.0};
#pragma unroll
    for (int i = j + 1; i < 4; ++i) {
      zd t = A[i * 4 + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t = t - mulc(A[i * 4 + k], A[j * 4 + k]);
      A[i * 4 + j] = scal(il, t);
    }
#pragma unroll
    for (int i = 0; i < j; ++i) A[i * 4 + j] = {0.0, 0.0};
  }
  return ok;
}

// X <- L^{-1} X (forward substitution), L lower with real diagonal.
__device__ __forceinline__ void trsm_lower(const zd* L, zd* X) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      zd t = X[i * 4 + c];
#pragma unroll
      for (int k = 0; k < i; ++k) t = t - L[i * 4 + k] * X[k * 4 + c];
      X[i * 4 + c] = scal(1.0 / L[i * 4 + i].x, t);
    }
  }
}

// X <- L^{-H} X (back substitution with the conjugate transpose).
__device__ __forceinline__ void trsm_lower_h(const zd* L, zd* X) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int i = 3; i >= 0; --i) {
      zd t = X[i * 4 + c];
#pragma unroll
      for (int k = i + 1; k < 4; ++k) t = t - cj(L[k * 4 + i]) * X[k * 4 + c];
      X[i * 4 + c] = scal(1.0 / L[i * 4 + i].x, t);
    }
  }
}

// ---------------------------------------------------------------------------
// Largest eigenvalue of a symmetric tridiagonal matrix by multisection on
// Sturm counts (256 probe points per round, all threads cooperate).
// ---------------------------------------------------------------------------
// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a and off-diagonal b (LDS arrays of AMMSE_MAX_LANCZOS entries, m of
// them used): sign changes of the leading principal minors of s (T - x I),
// p_k = (a_k - x) p_{k-1} - b_{k-1}^2 p_{k-2} with p_{-1} = 1, computed
// without divisions (s scales the entries to magnitude <= 1) in blocks of
// eight steps whose loads are issued together (steps from m on are skipped),
// rescaled by powers of two after each block.
__device__ inline int sturm_below(const double* a, const double* b, int m, double x, double s) {
  static_assert(AMMSE_MAX_LANCZOS % 8 == 0, "blocks of eight stay inside the arrays");
  const double big = 0x1p400, small = 0x1p-400;
  const double xs = x * s;
  double pm = 0.0, pc = 1.0;
  unsigned cnt = 0;
  for (int i = 0; i < m; i += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      av[u] = a[i + u];
      bv[u] = b[(i + u > 0) ? i + u - 1 : 0];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double bs = bv[u] * s;
      const double pn = fma(av[u] * s - xs, pc, -(bs * bs) * pm);
      const bool act = i + u < m;
      const unsigned ch = (unsigned)(((unsigned long long)__double_as_longlong(pn) ^
                                      (unsigned long long)__double_as_longlong(pc)) >> 63);
      cnt += act ? ch : 0u;
      pm = act ? pc : pm;
      pc = act ? pn : pc;
    }
    const double mag = fmax(fabs(pc), fabs(pm));
    const double f = (mag > big) ? small : ((mag < small) ? big : 1.0);
    pc *= f;
    pm *= f;
  }
  return (int)cnt;
}

// la, lb: diagonal and off-diagonal in LDS; imin: an LDS int used for the
// reduction; stops when the bracket is narrower than rtol * lambda.  Every
// thread of the block must call it.
// With th_prev > 0 (the value for a leading block, a lower bound of the new
// one) and conv != NULL, one round of probes over [th_prev, th_prev (1 + ltol)]
// first tests whether the value moved by less than ltol (*conv).
__device__ inline double tridiag_lmax(const double* la, const double* lb, int m, int* imin,
                                     double rtol = 1e-16, double th_prev = 0.0,
                                     double ltol = 0.0, bool* conv = nullptr) {
  double lo = 1e300, hi = -1e300;
  if (conv) *conv = false;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? fabs(lb[i - 1]) : 0.0) + (i < m - 1 ? fabs(lb[i]) : 0.0);
    lo = fmin(lo, la[i] - r);
    hi = fmax(hi, la[i] + r);
  }
  const double sc = 1.0 / fmax(fmax(fabs(lo), fabs(hi)), 1e-300);
  double qlo = -1e300;
  if (conv && th_prev > 0.0) {
    const double n1 = (double)blockDim.x;
    if (threadIdx.x == 0) *imin = blockDim.x;
    __syncthreads();
    const double x = th_prev * (1.0 + ltol * (double)(threadIdx.x + 1) / n1);
    if (sturm_below(la, lb, m, x, sc) == m) atomicMin(imin, (int)threadIdx.x);
    __syncthreads();
    const int t = *imin;
    __syncthreads();
    if (t < (int)blockDim.x) {
      *conv = true;
      return th_prev * (1.0 + ltol * (double)(t + 1) / n1);
    }
    qlo = th_prev * (1.0 + ltol);
  }
  hi += 1e-300 + fabs(hi) * 1e-15;
  if (qlo > lo) lo = fmin(qlo, hi);
  for (int round = 0; round < 8; ++round) {
    const double w = hi - lo;
    if (!(w > fabs(hi) * rtol)) break;
    if (threadIdx.x == 0) *imin = blockDim.x;
    __syncthreads();
    const double x = lo + w * (double)(threadIdx.x + 1) / (double)(blockDim.x + 1);
    if (sturm_below(la, lb, m, x, sc) == m) atomicMin(imin, (int)threadIdx.x);
    __syncthreads();
    const int t = *imin;
    const double nhi = (t < (int)blockDim.x) ? lo + w * (double)(t + 1) / (double)(blockDim.x + 1) : hi;
    const double nlo = (t > 0) ? lo + w * (double)t / (double)(blockDim.x + 1) : lo;
    lo = nlo;
    hi = nhi;
    __syncthreads();
  }
  return hi;
}

// ---------------------------------------------------------------------------
// Per-user receiver / weight algebra (Section IV equations for U and W)
// ---------------------------------------------------------------------------
// Input: J = I + sum of interference covariances (normalised noise), padded
// to 4 x 4 with identity; F = own-signal image G_own (N x d), zero padded.
// Output: UW = J^{-1} G_own (= U W), E = (I + G_own^H J^{-1} G_own)^{-1}
// (= the MSE matrix at the MMSE receiver), *rate = log det E^{-1} (nats).
// Returns false when a factorisation fails.
__device__ __forceinline__ bool user_receiver(zd* J, zd* F, zd* UW, zd* E, double* rate) {
  zd X[16];
  bool ok = chol4(J);
  trsm_lower(J, F);                           // F = L^{-1} G_own
#pragma unroll
  for (int i = 0; i < 4; ++i)                 // X = I + F^H F
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      zd t = {(i == j) ? 1.0 : 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 4; ++k) t = t + mulc(F[k * 4 + j], F[k * 4 + i]);
      X[i * 4 + j] = t;
    }
  trsm_lower_h(J, F);                         // UW = J^{-1} G_own
  ok = chol4(X) && ok;                        // E^{-1} = I + F^H F = Lw Lw^H
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) r += 2.0 * log(X[i * 4 + i].x);
  zd Li[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) Li[i] = {((i % 5) == 0) ? 1.0 : 0.0, 0.0};
  trsm_lower(X, Li);                          // Li = Lw^{-1}
#pragma unroll
  for (int i = 0; i < 4; ++i)                 // E = Li^H Li
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      zd t = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 4; ++k) t = t + mulc(Li[k * 4 + j], Li[k * 4 + i]);
      E[i * 4 + j] = t;
    }
#pragma unroll
  for (int i = 0; i < 16; ++i) UW[i] = F[i];
  *rate = r;
  return ok;
}

// D = alpha U W U^H and Y = alpha U W (padded 4 x 4): stage I uses W = I
// (U = UW E), stage II uses W = E^{-1} (U W = UW, U W U^H = UW E UW^H).
__device__ __forceinline__ void user_weights(const zd* UW, const zd* E, bool stage2, double a,
                                             zd* Dout, zd* Yout) {
  zd T[16];                                   // T = UW E  (= U)
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      zd t = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 4; ++k) t = t + UW[i * 4 + k] * E[k * 4 + j];
      T[i * 4 + j] = t;
    }
  const zd* Ur = stage2 ? UW : T;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      zd t = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 4; ++k) t = t + mulc(T[i * 4 + k], Ur[j * 4 + k]);
      Dout[i * 4 + j] = scal(a, t);
      Yout[i * 4 + j] = scal(a, Ur[i * 4 + j]);
    }
  // exactly Hermitian D (the step-size operator must be symmetric)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Dout[i * 4 + i].y = 0.0;
#pragma unroll
    for (int j = i + 1; j < 4; ++j) {
      const zd x = Dout[i * 4 + j], y = Dout[j * 4 + i];
      const zd m = {0.5 * (x.x + y.x), 0.5 * (x.y - y.y)};
      Dout[i * 4 + j] = m;
      Dout[j * 4 + i] = cj(m);
    }
  }
}

// complex double from lane `src` (every lane of the wave must execute it)
__device__ __forceinline__ zd shz(zd v, int src) {
  return {__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}

// ---------------------------------------------------------------------------
// 4 x 4 complex double matrices spread over a 16-lane group: lane base + 4a + b
// holds entry (a, b).  All functions must be executed by the whole wave.
// The 16-lane groups are the DPP rows of the wave, so row-local patterns use
// DPP moves (a broadcast of one lane of the row; a broadcast within the quad
// of lanes that holds one matrix row) or a bit-mask swizzle; only transposed
// reads go through the general lane permutation.
// ---------------------------------------------------------------------------
// Component-wise select (a select of whole structs can end up as a select of
// stack addresses)
__device__ __forceinline__ zd sel(bool c, zd a, zd b) {
  return {c ? a.x : b.x, c ? a.y : b.y};
}

struct Lane4 {
  int base, a, b;
  __device__ __forceinline__ zd at(zd v, int r, int c) const { return shz(v, base + 4 * r + c); }
};

template <int PAT>
__device__ __forceinline__ double swz64(double v) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_swizzle((int)u, PAT);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_swizzle((int)(u >> 32), PAT);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// entry (K, K) to every lane of the group (DPP row_newbcast)
template <int K>
__device__ __forceinline__ zd l4_diag(zd v) {
  return {dpp64<0x150 + 5 * K>(v.x), dpp64<0x150 + 5 * K>(v.y)};
}
// entry (a, K) of the lane's own row a (DPP quad_perm [K, K, K, K])
template <int K>
__device__ __forceinline__ zd l4_rowq(zd v) {
  return {dpp64<0x55 * K>(v.x), dpp64<0x55 * K>(v.y)};
}
// entry (K, b) of the lane's own column b (bit-mask swizzle: keep lane bits
// 0, 1 and 4, set bits 2-3 to K)
template <int K>
__device__ __forceinline__ zd l4_colk(zd v) {
  constexpr int PAT = 0x13 | ((4 * K) << 5);
  return {swz64<PAT>(v.x), swz64<PAT>(v.y)};
}

// Quotient i / n for 0 <= i < 2^22 from rn = 1 / n (float, n >= 1), without
// the integer division sequence: (i + 1/2) / n is at least 1 / (2n) away from
// every integer, more than the float rounding of the product can move it, so
// truncation gives the exact quotient.
__device__ __forceinline__ int quot(int i, float rn) { return (int)(((float)i + 0.5f) * rn); }

// 1 / sqrt(x) for finite x >= 1e-300: the hardware estimate refined by two
// Newton steps y <- y + y (1 - x y^2) / 2, which square the relative error
// (to about one unit in the last place), in 7 dependent operations instead of
// a correctly rounded square root followed by a correctly rounded division
// (about 22 on this target, on the Cholesky factorisations' critical path).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * y;
  double e = fma(-x * y, h, 0.5);               // (1 - x y^2) / 2
  y = fma(y, e, y);
  h = 0.5 * y;
  e = fma(-x * y, h, 0.5);
  return fma(y, e, y);
}

// Cholesky step K of a Hermitian matrix: the trailing block is updated as a
// whole, so row K above the diagonal still holds conj(column K) and supplies
// L[b][K] = conj(A[K][b]) / l without a transposed read.
template <int K>
__device__ __forceinline__ void chol16_step(const Lane4& L, zd& A, bool& ok, double& ik) {
  const double dkk = l4_diag<K>(A).x;
  const zd rk = l4_colk<K>(A);                  // A[K][b]
  ok = ok && (dkk > 0.0) && isfinite(dkk);
  const double il = rsqrt_nr(fmin(fmax(dkk, 1e-300), __DBL_MAX__));   // 1 / l
  ik = il;
  // lane-dependent updates through per-lane factors (no divergent branches):
  // column K from the diagonal down is scaled by 1/l (the diagonal becomes
  // dkk / l = l, made real), the trailing block loses L[a][K] conj(L[b][K])
  const double f = (L.b == K && L.a >= K) ? il : 1.0;
  A = scal(f, A);
  A.y = (L.a == K && L.b == K) ? 0.0 : A.y;
  const zd lak = l4_rowq<K>(A);                 // L[a][K]
  const zd pr = lak * rk;
  const double g = (L.a > K && L.b > K) ? il : 0.0;
  A = {fma(-g, pr.x, A.x), fma(-g, pr.y, A.y)};
}

// In place Cholesky (lower) of a Hermitian matrix; ok is cleared when a pivot
// is not positive/finite.
// id: the reciprocals of the diagonal of the factor (for the solves below).
__device__ __forceinline__ zd chol16(const Lane4& L, zd A, bool& ok, double (&id)[4]) {
  chol16_step<0>(L, A, ok, id[0]);
  chol16_step<1>(L, A, ok, id[1]);
  chol16_step<2>(L, A, ok, id[2]);
  chol16_step<3>(L, A, ok, id[3]);
  return sel(L.b > L.a, zd{0.0, 0.0}, A);
}
__device__ __forceinline__ zd chol16(const Lane4& L, zd A, bool& ok) {
  double id[4];
  return chol16(L, A, ok, id);
}

// lq: entry (a, K) of the factor with its diagonal zeroed (so rows a <= K
// are left alone by the update).
template <int K>
__device__ __forceinline__ void trsm16_step(const Lane4& L, const zd& lq, double ik, zd& X) {
  X = scal((L.a == K) ? ik : 1.0, X);
  const zd xkb = l4_colk<K>(X);
  X = X - lq * xkb;
}

// X <- Lo^{-1} X (forward substitution, Lo lower with real diagonal whose
// reciprocals are id)
__device__ __forceinline__ zd trsm16(const Lane4& L, zd Lo, const double (&id)[4], zd X) {
  const double i0 = id[0], i1 = id[1], i2 = id[2], i3 = id[3];
  const zd Lz = sel(L.a == L.b, zd{0.0, 0.0}, Lo);   // strictly lower part
  const zd q0 = l4_rowq<0>(Lz), q1 = l4_rowq<1>(Lz), q2 = l4_rowq<2>(Lz);
  trsm16_step<0>(L, q0, i0, X);
  trsm16_step<1>(L, q1, i1, X);
  trsm16_step<2>(L, q2, i2, X);
  return scal((L.a == 3) ? i3 : 1.0, X);
}

template <int K>
// lka: entry (K, a) of the factor with its diagonal zeroed (zero for rows a >= K).
__device__ __forceinline__ void trsm16h_step(const Lane4& L, const zd& lka, double ik, zd& X) {
  X = scal((L.a == K) ? ik : 1.0, X);
  const zd xkb = l4_colk<K>(X);
  X = X - cj(lka) * xkb;
}

// X <- Lo^{-H} X (back substitution with the conjugate transpose)
__device__ __forceinline__ zd trsm16h(const Lane4& L, zd Lo, const double (&id)[4], zd X) {
  const double i0 = id[0], i1 = id[1], i2 = id[2], i3 = id[3];
  const zd Lz = sel(L.a == L.b, zd{0.0, 0.0}, Lo);   // strictly lower part
  const zd t1 = L.at(Lz, 1, L.a), t2 = L.at(Lz, 2, L.a), t3 = L.at(Lz, 3, L.a);   // Lo[k][a]
  trsm16h_step<3>(L, t3, i3, X);
  trsm16h_step<2>(L, t2, i2, X);
  trsm16h_step<1>(L, t1, i1, X);
  return scal((L.a == 0) ? i0 : 1.0, X);
}

__device__ __forceinline__ void diag_recip(zd Lo, double (&id)[4]) {
  id[0] = 1.0 / l4_diag<0>(Lo).x;
  id[1] = 1.0 / l4_diag<1>(Lo).x;
  id[2] = 1.0 / l4_diag<2>(Lo).x;
  id[3] = 1.0 / l4_diag<3>(Lo).x;
}
__device__ __forceinline__ zd trsm16(const Lane4& L, zd Lo, zd X) {
  double id[4];
  diag_recip(Lo, id);
  return trsm16(L, Lo, id, X);
}
__device__ __forceinline__ zd trsm16h(const Lane4& L, zd Lo, zd X) {
  double id[4];
  diag_recip(Lo, id);
  return trsm16h(L, Lo, id, X);
}

// A^H B, A B, A B^H
__device__ __forceinline__ zd mm_hn(const Lane4& L, zd A, zd B) {
  const zd a0 = L.at(A, 0, L.a), a1 = L.at(A, 1, L.a), a2 = L.at(A, 2, L.a), a3 = L.at(A, 3, L.a);
  const zd b0 = l4_colk<0>(B), b1 = l4_colk<1>(B), b2 = l4_colk<2>(B), b3 = l4_colk<3>(B);
  return ((cj(a0) * b0 + cj(a1) * b1) + (cj(a2) * b2 + cj(a3) * b3));
}
__device__ __forceinline__ zd mm_nn(const Lane4& L, zd A, zd B) {
  (void)L;
  const zd a0 = l4_rowq<0>(A), a1 = l4_rowq<1>(A), a2 = l4_rowq<2>(A), a3 = l4_rowq<3>(A);
  const zd b0 = l4_colk<0>(B), b1 = l4_colk<1>(B), b2 = l4_colk<2>(B), b3 = l4_colk<3>(B);
  return ((a0 * b0 + a1 * b1) + (a2 * b2 + a3 * b3));
}
__device__ __forceinline__ zd mm_nh(const Lane4& L, zd A, zd B) {
  const zd a0 = l4_rowq<0>(A), a1 = l4_rowq<1>(A), a2 = l4_rowq<2>(A), a3 = l4_rowq<3>(A);
  const zd b0 = L.at(B, L.b, 0), b1 = L.at(B, L.b, 1), b2 = L.at(B, L.b, 2), b3 = L.at(B, L.b, 3);
  return ((mulc(a0, b0) + mulc(a1, b1)) + (mulc(a2, b2) + mulc(a3, b3)));
}

__device__ __forceinline__ double rel_change(double a, double b) {
  if (b > 0) return fabs(a - b) / b;
  return (a == b) ? 0.0 : INFINITY;
}


// ---------------------------------------------------------------------------
// Wave-level Lanczos helpers: sums, Sturm counts and the largest eigenvalue of
// the tridiagonal matrix, inside one wave (no block barriers)
// ---------------------------------------------------------------------------

// Three wave sums at once (the same additions as wave_sum for each value,
// interleaved level by level).
__device__ __forceinline__ void wave_sum3_dpp(double& a, double& b, double& c) {
  a += dpp64<0xB1>(a);
  b += dpp64<0xB1>(b);
  c += dpp64<0xB1>(c);
  a += dpp64<0x4E>(a);
  b += dpp64<0x4E>(b);
  c += dpp64<0x4E>(c);
  a += dpp64<0x124>(a);
  b += dpp64<0x124>(b);
  c += dpp64<0x124>(c);
  a += dpp64<0x128>(a);
  b += dpp64<0x128>(b);
  c += dpp64<0x128>(c);
  a = (read_lane(a, 0) + read_lane(a, 16)) + (read_lane(a, 32) + read_lane(a, 48));
  b = (read_lane(b, 0) + read_lane(b, 16)) + (read_lane(b, 32) + read_lane(b, 48));
  c = (read_lane(c, 0) + read_lane(c, 16)) + (read_lane(c, 32) + read_lane(c, 48));
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix held in
// LDS as 64 pairs tp[k] = (a_k, b_{k-1}^2) (entries of magnitude <= 1, b_{-1}
// = 0; entries from m on padded with a = 8, b = 0, which adds eigenvalues
// above every probe and leaves the count unchanged).  Sign changes of the
// leading principal minors p_k(x) = det(T_k - x I), p_{-1} = 1, computed
// without divisions (p_k = (a_k - x) p_{k-1} - b_{k-1}^2 p_{k-2}) in blocks
// of eight steps (the eight pairs are loaded together; blocks past m read
// padding) and rescaled by powers of two after each block to stay in range.
__device__ __forceinline__ int sturm_count(const double2* tp, int m, double x) {
  const double big = 0x1p400, small = 0x1p-400;
  double pm = 0.0, pc = 1.0;
  auto sgn = [](double v) { return (unsigned)((unsigned long long)__double_as_longlong(v) >> 63); };
  unsigned cnt = 0;
  for (int i = 0; i < m; i += 8) {                // i <= 56: every k below 64
    double2 e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = tp[i + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double pn = fma(e[u].x - x, pc, -e[u].y * pm);
      cnt += sgn(pn) ^ sgn(pc);
      pm = pc;
      pc = pn;
    }
    const double mag = fmax(fabs(pc), fabs(pm));
    const double f = (mag > big) ? small : ((mag < small) ? big : 1.0);
    pc *= f;
    pm *= f;
  }
  return (int)cnt;
}

__device__ __forceinline__ double wave_min_dpp(double v) {
  v = fmin(v, dpp64<0xB1>(v));
  v = fmin(v, dpp64<0x4E>(v));
  v = fmin(v, dpp64<0x124>(v));
  v = fmin(v, dpp64<0x128>(v));
  return fmin(fmin(read_lane(v, 0), read_lane(v, 16)), fmin(read_lane(v, 32), read_lane(v, 48)));
}
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp64<0xB1>(v));
  v = fmax(v, dpp64<0x4E>(v));
  v = fmax(v, dpp64<0x124>(v));
  v = fmax(v, dpp64<0x128>(v));
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// Largest eigenvalue, to relative width 1e-10, of the m x m symmetric
// tridiagonal matrix with diagonal ta and off-diagonal tb (lane i: entry i),
// by multisection inside one wave (64 probes per round on Sturm counts of the
// matrix scaled by 1/tmax, tmax >= every |a_i| + |b_i|; tp: 64 pairs of LDS
// owned by the calling wave).  With a previous estimate th_prev > 0 (the
// value for a leading block, which bounds the new one from below) the first
// round places 16 probes ltol/16 apart above th_prev and 48 in geometric
// progression up to the Gershgorin bound, so that a small and a large move of
// the value are bracketed in one round; when the value lies within
// th_prev (1 + ltol), *conv reports convergence.
__device__ __forceinline__ double wave_tridiag_lmax(double ta, double tb, int m, double tmax,
                                                    double th_prev, double ltol, double2* tp,
                                                    bool* conv) {
  const int lane = threadIdx.x & 63;
  const double rtol = 1e-10;
  const double is = 1.0 / tmax;
  const double an = (lane < m) ? ta * is : 8.0;
  const double bn = (lane < m - 1) ? tb * is : 0.0;
  const double bup = __shfl_up(bn, 1, 64);      // by every lane (no divergent shuffle)
  const double bl_ = (lane > 0) ? bup : 0.0;    // b_{lane-1}
  tp[lane] = make_double2(an, bl_ * bl_);
  *conv = false;
  // Gershgorin interval
  const double rad = fabs(bl_) + fabs(bn);
  const double glo = wave_min_dpp((lane < m) ? an - rad : 1e300);
  const double ghi = wave_max_dpp((lane < m) ? an + rad : -1e300);
  double hi = ghi + fabs(ghi) * 1e-6 + 1e-300;
  double lo = glo;
  const double t0 = th_prev * is;
  if (t0 > 0.0) {
    // probe l: t0 (1 + f_l), f_l = ltol (l + 1) / 16 for l < 16, then
    // ltol 2^(g (l - 15) / 48) with ltol 2^g = hi / t0 - 1 (g clamped to
    // [2, 120]; probes above hi only confirm the bound)
    const float g = fminf(fmaxf(__log2f((float)((hi / t0 - 1.0) / ltol)), 2.f), 120.f);
    const double f = (lane < 16) ? ltol * (double)(lane + 1) * (1.0 / 16.0)
                                 : ltol * (double)exp2f(g * (float)(lane - 15) * (1.0f / 48.0f));
    const double x = t0 * (1.0 + f);
    const unsigned long long mask = __ballot(sturm_count(tp, m, x) == m);
    if (mask) {
      const int t = __ffsll((long long)mask) - 1;
      const double xt = read_lane(x, t);
      if (t < 16) {
        *conv = true;
        return xt * tmax;
      }
      hi = xt;
      lo = (t > 0) ? read_lane(x, t - 1) : t0;
    } else {
      lo = read_lane(x, 63);
    }
  }
  const double fr = (double)(lane + 1) * (1.0 / 65.0);
  for (int round = 0; round < 10; ++round) {
    const double w = hi - lo;
    if (!(w > fabs(hi) * rtol)) break;
    const double x = lo + w * fr;
    const unsigned long long mask = __ballot(sturm_count(tp, m, x) == m);
    const int t = mask ? (__ffsll((long long)mask) - 1) : 64;
    const double nhi = (t < 64) ? read_lane(x, t) : hi;
    const double nlo = (t > 0) ? read_lane(x, t - 1) : lo;
    lo = nlo;
    hi = nhi;
  }
  return hi * tmax;
}

}  // namespace ammse_dev
