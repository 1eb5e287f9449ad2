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

// Sum over the block (a multiple of 64 threads, at most 512); every thread
// receives the same value.
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
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
__device__ inline int sturm_below(const double* a, const double* b, int m, double x) {
  int cnt = 0;
  double q = a[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < m; ++i) {
    if (q == 0.0) q = 1e-300;
    q = a[i] - x - b[i - 1] * b[i - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// la, lb: diagonal and off-diagonal in LDS; imin: an LDS int used for the
// reduction; stops when the bracket is narrower than rtol * lambda.  Every
// thread of the block must call it.
__device__ inline double tridiag_lmax(const double* la, const double* lb, int m, int* imin,
                                     double rtol = 1e-16) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? fabs(lb[i - 1]) : 0.0) + (i < m - 1 ? fabs(lb[i]) : 0.0);
    lo = fmin(lo, la[i] - r);
    hi = fmax(hi, la[i] + r);
  }
  hi += 1e-300 + fabs(hi) * 1e-15;
  for (int round = 0; round < 8; ++round) {
    const double w = hi - lo;
    if (!(w > fabs(hi) * rtol)) break;
    if (threadIdx.x == 0) *imin = blockDim.x;
    __syncthreads();
    const double x = lo + w * (double)(threadIdx.x + 1) / (double)(blockDim.x + 1);
    if (sturm_below(la, lb, m, x) == m) atomicMin(imin, (int)threadIdx.x);
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
// ---------------------------------------------------------------------------
struct Lane4 {
  int base, a, b;
  __device__ __forceinline__ zd at(zd v, int r, int c) const { return shz(v, base + 4 * r + c); }
};

// In place Cholesky (lower); ok is cleared when a pivot is not positive/finite.
__device__ __forceinline__ zd chol16(const Lane4& L, zd A, bool& ok) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double dkk = L.at(A, k, k).x;
    ok = ok && (dkk > 0.0) && isfinite(dkk);
    const double l = sqrt(fmax(dkk, 1e-300));
    if (L.b == k && L.a > k) A = scal(1.0 / l, A);
    if (L.a == k && L.b == k) A = {l, 0.0};
    const zd lak = L.at(A, L.a, k), lbk = L.at(A, L.b, k);
    if (L.a > k && L.b > k) A = A - mulc(lak, lbk);
  }
  if (L.b > L.a) A = {0.0, 0.0};
  return A;
}

// X <- Lo^{-1} X (forward substitution, Lo lower with real diagonal)
__device__ __forceinline__ zd trsm16(const Lane4& L, zd Lo, zd X) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double lkk = L.at(Lo, k, k).x;
    if (L.a == k) X = scal(1.0 / lkk, X);
    const zd xkb = L.at(X, k, L.b), lak = L.at(Lo, L.a, k);
    if (L.a > k) X = X - lak * xkb;
  }
  return X;
}

// X <- Lo^{-H} X (back substitution with the conjugate transpose)
__device__ __forceinline__ zd trsm16h(const Lane4& L, zd Lo, zd X) {
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    const double lkk = L.at(Lo, k, k).x;
    if (L.a == k) X = scal(1.0 / lkk, X);
    const zd xkb = L.at(X, k, L.b), lka = L.at(Lo, k, L.a);
    if (L.a < k) X = X - cj(lka) * xkb;
  }
  return X;
}

// A^H B, A B, A B^H
__device__ __forceinline__ zd mm_hn(const Lane4& L, zd A, zd B) {
  zd c = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) c = c + cj(L.at(A, k, L.a)) * L.at(B, k, L.b);
  return c;
}
__device__ __forceinline__ zd mm_nn(const Lane4& L, zd A, zd B) {
  zd c = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) c = c + L.at(A, L.a, k) * L.at(B, k, L.b);
  return c;
}
__device__ __forceinline__ zd mm_nh(const Lane4& L, zd A, zd B) {
  zd c = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) c = c + mulc(L.at(A, L.a, k), L.at(B, L.b, k));
  return c;
}

__device__ __forceinline__ double rel_change(double a, double b) {
  if (b > 0) return fabs(a - b) / b;
  return (a == b) ? 0.0 : INFINITY;
}


}  // namespace ammse_dev
