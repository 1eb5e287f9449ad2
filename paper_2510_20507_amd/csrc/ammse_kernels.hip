// Fused A-MMMSE solve kernel for gfx950 (generic path, FP64 and FP32).
//
// One workgroup of 256 threads owns one channel realisation for the whole
// solve: all iterations of Algorithm 3 run inside one launch, so the batch of
// independent instances is the data-parallel axis and no state crosses
// workgroups.  Per iteration t:
//   G_c  = S H_{:,c} V_c^{t-1}       channel product per BS (S = diag(1/sigma_u),
//                                     which normalises every user to unit noise)
//   per user: interference-plus-noise covariance J-_u, Cholesky, rate, E, U, W
//   WSR(V^{t-1}) = sum alpha_u R_u    -> stage latch (eps1), optional eps2 stop
//   step size 1/||2 A_c||_2 by Lanczos on A_c = H^H S D S H (adaptive window)
//   Z_c  = S (D G^_c - Y_c)          with G^ = (1+w) G^{t-1} - w G^{t-2} (linearity)
//   Grad = 2 H_{:,c}^H Z_c            second channel product per BS
//   V^t  = Pi_P(V^ - gamma Grad)      extrapolated step and projection per BS
//
// Receiver/weight algebra (Section IV equations for U and W) is evaluated in
// the cancellation-free form: with F = L^{-1} G_own (J- = L L^H),
// W = E^{-1} = I + F^H F, R_u = log det W, U W = J-^{-1} G_own,
// U = (U W) E.  These are identities of the paper's expressions (Woodbury),
// chosen because I - U^H H V loses digits at high SNR in short precision.
// All N x N and d x d work is in double, zero-padded to 4 x 4 so that every
// loop has a compile-time bound.

#include <math.h>

#include "ammse_internal.h"

#include "ammse_device.h"

namespace {
using namespace ammse_dev;

constexpr int KC = 16;   // k-chunk of the channel products
constexpr int TM = 64;   // output tile rows
constexpr int TN = 64;   // output tile columns

template <class R>
struct Smem {
  cx<R> As[KC * (TM + 1)];
  cx<R> Bs[KC * (TN + 1)];
  double invsig[AMMSE_MAX_USERS];
  double alpha[AMMSE_MAX_USERS];
  double rate[AMMSE_MAX_USERS];
  int cellOf[AMMSE_MAX_USERS];
  int local[AMMSE_MAX_USERS];
  int cu[AMMSE_MAX_CELLS];
  int colOff[AMMSE_MAX_CELLS + 1];
  double Pc[AMMSE_MAX_CELLS];
  double gamma[AMMSE_MAX_CELLS];
  double la[AMMSE_MAX_LANCZOS];
  double lb[AMMSE_MAX_LANCZOS];
  zd h[AMMSE_MAX_LANCZOS];
  double red[16];
  int fail;
  int imin;
};

// C (m x n) = alpha * op(A) * B, row i of C further scaled by rowscale[i / rs_div]
// when rowscale != nullptr.  op(A) = A (m x k, row-major, lda) or, with CONJA,
// A^H where A is stored k x m row-major (lda).  B is k x n row-major (ldb).
// All operands in global memory, staged through LDS tiles of 64 x 16.
template <class R, bool CONJA>
__device__ void block_gemm(int m, int n, int k, const cx<R>* __restrict__ A, long lda,
                           const cx<R>* __restrict__ B, long ldb, cx<R>* __restrict__ Cm,
                           long ldc, R alpha, const double* rowscale, int rs_div, cx<R>* As,
                           cx<R>* Bs) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  for (int i0 = 0; i0 < m; i0 += TM) {
    for (int j0 = 0; j0 < n; j0 += TN) {
      cx<R> acc[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = {R(0), R(0)};
      for (int k0 = 0; k0 < k; k0 += KC) {
        for (int e = tid; e < TM * KC; e += AMMSE_BLOCK) {
          int row, kk;
          if (CONJA) {
            row = e % TM;
            kk = e / TM;
          } else {
            kk = e % KC;
            row = e / KC;
          }
          const int gi = i0 + row, gk = k0 + kk;
          cx<R> v = {R(0), R(0)};
          if (gi < m && gk < k) v = CONJA ? cj(A[(long)gk * lda + gi]) : A[(long)gi * lda + gk];
          As[kk * (TM + 1) + row] = v;
        }
        for (int e = tid; e < KC * TN; e += AMMSE_BLOCK) {
          const int col = e % TN, kk = e / TN;
          const int gj = j0 + col, gk = k0 + kk;
          cx<R> v = {R(0), R(0)};
          if (gj < n && gk < k) v = B[(long)gk * ldb + gj];
          Bs[kk * (TN + 1) + col] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < KC; ++kk) {
          cx<R> a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = As[kk * (TM + 1) + ty + 16 * i];
#pragma unroll
          for (int j = 0; j < 4; ++j) b[j] = Bs[kk * (TN + 1) + tx + 16 * j];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              acc[i][j].x += a[i].x * b[j].x - a[i].y * b[j].y;
              acc[i][j].y += a[i].x * b[j].y + a[i].y * b[j].x;
            }
        }
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gi = i0 + ty + 16 * i;
        if (gi >= m) continue;
        R s = alpha;
        if (rowscale) s *= (R)rowscale[gi / rs_div];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gj = j0 + tx + 16 * j;
          if (gj < n) Cm[(long)gi * ldc + gj] = scal(s, acc[i][j]);
        }
      }
    }
  }
}

typedef float floatx4_t __attribute__((ext_vector_type(4)));

// FP32 variant on MFMA (v_mfma_f32_16x16x4f32): same LDS staging, each wave
// computes a 16 x 64 strip of the 64 x 64 output tile; a complex product is
// three real accumulators (Re*Re, Im*Im, Re*Im + Im*Re).
template <bool CONJA>
__device__ void block_gemm_mfma(int m, int n, int k, const cx<float>* __restrict__ A, long lda,
                                const cx<float>* __restrict__ B, long ldb,
                                cx<float>* __restrict__ Cm, long ldc, float alpha,
                                const double* rowscale, int rs_div, cx<float>* As,
                                cx<float>* Bs) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  for (int i0 = 0; i0 < m; i0 += TM) {
    for (int j0 = 0; j0 < n; j0 += TN) {
      floatx4_t P[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < 3; ++q) P[j][q] = floatx4_t{0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < k; k0 += KC) {
        for (int e = tid; e < TM * KC; e += AMMSE_BLOCK) {
          int row, kk;
          if (CONJA) {
            row = e % TM;
            kk = e / TM;
          } else {
            kk = e % KC;
            row = e / KC;
          }
          const int gi = i0 + row, gk = k0 + kk;
          cx<float> v = {0.f, 0.f};
          if (gi < m && gk < k) v = CONJA ? cj(A[(long)gk * lda + gi]) : A[(long)gi * lda + gk];
          As[kk * (TM + 1) + row] = v;
        }
        for (int e = tid; e < KC * TN; e += AMMSE_BLOCK) {
          const int col = e % TN, kk = e / TN;
          const int gj = j0 + col, gk = k0 + kk;
          cx<float> v = {0.f, 0.f};
          if (gj < n && gk < k) v = B[(long)gk * ldb + gj];
          Bs[kk * (TN + 1) + col] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
          const cx<float> a = As[(kk + lk) * (TM + 1) + 16 * wave + li];
          cx<float> b[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) b[j] = Bs[(kk + lk) * (TN + 1) + 16 * j + li];
#pragma unroll
          for (int j = 0; j < 4; ++j)
            P[j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[j].x, P[j][0], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            P[j][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[j].y, P[j][1], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            P[j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[j].y, P[j][2], 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            P[j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[j].x, P[j][2], 0, 0, 0);
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + 16 * wave + 4 * lk + r;
        if (gi >= m) continue;
        float s = alpha;
        if (rowscale) s *= (float)rowscale[gi / rs_div];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gj = j0 + 16 * j + li;
          if (gj < n) Cm[(long)gi * ldc + gj] = {s * (P[j][0][r] - P[j][1][r]), s * P[j][2][r]};
        }
      }
    }
  }
}

// Channel product dispatch: MFMA for FP32 storage, LDS-tiled FMA for FP64.
template <class R, bool CONJA>
__device__ __forceinline__ void channel_gemm(int m, int n, int k, const cx<R>* A, long lda,
                                             const cx<R>* B, long ldb, cx<R>* Cm, long ldc,
                                             R alpha, const double* rowscale, int rs_div,
                                             cx<R>* As, cx<R>* Bs) {
  if constexpr (sizeof(R) == 4) {
    block_gemm_mfma<CONJA>(m, n, k, A, lda, B, ldb, Cm, ldc, alpha, rowscale, rs_div, As, Bs);
  } else {
    block_gemm<R, CONJA>(m, n, k, A, lda, B, ldb, Cm, ldc, alpha, rowscale, rs_div, As, Bs);
  }
}

// ---------------------------------------------------------------------------
// The fused kernel
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(AMMSE_BLOCK) void ammse_solve_kernel(ammse_kparams_t p) {
  __shared__ Smem<R> sm;
  const ammse_desc_t D = p.desc[blockIdx.x];
  const int tid = threadIdx.x;
  const int C = D.C, U = D.U, M = D.M, N = D.N, d = D.d, un = D.un;
  const int b = D.b;

  // ---- per-instance tables in LDS
  for (int u = tid; u < U; u += AMMSE_BLOCK) {
    sm.invsig[u] = 1.0 / sqrt(p.sigma2[D.user_off + u]);
    sm.alpha[u] = p.alpha[D.user_off + u];
  }
  if (tid == 0) {
    int col = 0, u = 0;
    for (int c = 0; c < C; ++c) {
      const int n = p.cell_users[D.cell_off + c];
      sm.cu[c] = n;
      sm.colOff[c] = col;
      sm.Pc[c] = p.wsr_only ? 0.0 : p.P[D.bs_off + c];
      sm.gamma[c] = 0.0;
      for (int i = 0; i < n; ++i, ++u) {
        sm.cellOf[u] = c;
        sm.local[u] = i;
      }
      col += n * d;
    }
    sm.colOff[C] = col;
    sm.fail = 0;
  }
  __syncthreads();

  const ammse_ws_layout_t L = ammse_ws_layout((int)sizeof(R), U, M, N, d, p.lanczos_steps);
  char* ws = p.ws + D.ws_off;
  cx<R>* Gp = (cx<R>*)(ws + L.Gp);
  cx<R>* Gq = (cx<R>*)(ws + L.Gq);
  cx<R>* Z = (cx<R>*)(ws + L.Z);
  cx<R>* Vq = (cx<R>*)(ws + L.Vq);
  cx<R>* Gr = (cx<R>*)(ws + L.Gr);
  zd* Jm = (zd*)(ws + L.Jm);
  zd* Dm = (zd*)(ws + L.Dm);
  zd* Ym = (zd*)(ws + L.Ym);
  zd* Lq = (zd*)(ws + L.Lq);
  zd* Lw = (zd*)(ws + L.Lw);
  zd* Ly1 = (zd*)(ws + L.Ly1);
  zd* Ly2 = (zd*)(ws + L.Ly2);
  const cx<R>* H = (const cx<R>*)p.H + D.h_off;
  cx<R>* V = (cx<R>*)p.V + D.v_off;
  const long Vtot = (long)M * D.ud;

  auto channel_product = [&](cx<R>* G, const cx<R>* Vsrc) {
    for (int c = 0; c < C; ++c) {
      const int nc = sm.cu[c] * d;
      if (nc == 0) continue;
      channel_gemm<R, false>(un, nc, M, H + (long)c * un * M, M, Vsrc + (long)M * sm.colOff[c], nc,
                           G + (long)un * sm.colOff[c], nc, R(1), sm.invsig, N, sm.As, sm.Bs);
    }
  };

  // Per-user receiver algebra on G (normalised products of the current V).
  // Writes alpha_u R_u into sm.rate; keeps UW and E in the caller's registers.
  auto interference_cov = [&](const cx<R>* G) {
    const int np = N * (N + 1) / 2;
    for (int e = tid; e < U * np; e += AMMSE_BLOCK) {
      const int u = e / np;
      int q = e % np, n1 = 0;
      while (q >= N - n1) {
        q -= N - n1;
        ++n1;
      }
      const int n2 = n1 + q;
      const int cown = sm.cellOf[u], j0 = sm.local[u] * d;
      zd acc = {0.0, 0.0};
      for (int c = 0; c < C; ++c) {
        const int nc = sm.cu[c] * d;
        const cx<R>* Gc = G + (long)un * sm.colOff[c];
        const cx<R>* r1 = Gc + (long)(u * N + n1) * nc;
        const cx<R>* r2 = Gc + (long)(u * N + n2) * nc;
        for (int j = 0; j < nc; ++j) {
          if (c == cown && j >= j0 && j < j0 + d) continue;
          acc = acc + mulc(to_d(r1[j]), to_d(r2[j]));
        }
      }
      if (n1 == n2) acc = {acc.x + 1.0, 0.0};
      Jm[u * 16 + n1 * 4 + n2] = acc;
      Jm[u * 16 + n2 * 4 + n1] = cj(acc);
    }
    __syncthreads();
  };

  auto user_rates = [&](const cx<R>* G, zd* UW, zd* E) {
    if (tid < U) {
      const int u = tid;
      zd J[16], F[16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          J[i * 4 + j] = (i < N && j < N) ? Jm[u * 16 + i * 4 + j]
                                          : zd{(i == j) ? 1.0 : 0.0, 0.0};
          F[i * 4 + j] = {0.0, 0.0};
        }
      const int c = sm.cellOf[u], nc = sm.cu[c] * d, j0 = sm.local[u] * d;
      const cx<R>* Gc = G + (long)un * sm.colOff[c];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          if (i < N && s < d) F[i * 4 + s] = to_d(Gc[(long)(u * N + i) * nc + j0 + s]);
      double r;
      const bool ok = user_receiver(J, F, UW, E, &r);
      sm.rate[u] = sm.alpha[u] * r;
      if (!ok) atomicOr(&sm.fail, AMMSE_INST_CHOLESKY);
    }
  };

  // WSR in bits of the rates in sm.rate (all threads get the value).
  auto wsr_sum = [&]() {
    double v = 0.0;
    for (int u = tid; u < U; u += AMMSE_BLOCK) v += sm.rate[u];
    return block_sum(v, sm.red) * (1.0 / M_LN2);
  };

  // D_u = alpha U W U^H, Y_u = alpha U W into the workspace (padded 4 x 4).
  auto user_weights_ws = [&](const zd* UW, const zd* E, bool stage2) {
    if (tid < U) {
      zd Dl[16], Yl[16];
      user_weights(UW, E, stage2, sm.alpha[tid], Dl, Yl);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        Dm[tid * 16 + i] = Dl[i];
        Ym[tid * 16 + i] = Yl[i];
      }
    }
    __syncthreads();
  };

  // lambda_max(A_c), A_c = H_c^H S D S H_c, by plain three-term Lanczos (the
  // largest Ritz value converges without re-orthogonalisation).  Products
  // with H use several threads per row / column (a power of two within one
  // wave, combined by shuffles); the three inner products of a step are
  // reduced together.  FP64 forms ||w - alpha q - beta p|| explicitly, FP32
  // uses beta^2 = ||w||^2 - alpha^2 - 2 beta_prev Re(p^H w) + beta_prev^2.
  auto lanczos_lmax = [&](int c) {
    const cx<R>* __restrict__ Hc = H + (long)c * un * M;
    zd* qv = Lq;
    zd* pv = Lq + M;
    zd* wv = Lq + 2 * M;
    int tpr = 1;
    while (tpr < 64 && tpr * 2 * un <= AMMSE_BLOCK) tpr *= 2;
    int tpc = 1;
    while (tpc < 64 && tpc * 2 * M <= AMMSE_BLOCK) tpc *= 2;
    for (int i = tid; i < M; i += AMMSE_BLOCK) {
      qv[i] = {1.0 + 0.5 * sin(0.731 * i + 0.25), 0.3 * cos(1.37 * i + 0.5)};
      pv[i] = {0.0, 0.0};
    }
    double nn = 0.0;
    for (int i = tid; i < M; i += AMMSE_BLOCK) nn += nrm2(qv[i]);
    nn = block_sum(nn, sm.red);
    for (int i = tid; i < M; i += AMMSE_BLOCK) qv[i] = scal(1.0 / sqrt(nn), qv[i]);
    __syncthreads();
    const int m = min(p.lanczos_steps, M);
    constexpr bool exact_beta = sizeof(R) == 8;
    const double ltol = exact_beta ? 1e-14 : 1e-8;
    const double rtol = exact_beta ? 1e-16 : 1e-10;
    const int first = exact_beta ? 8 : 12, every = exact_beta ? 8 : 4;
    double beta_prev = 0.0, tmax = 0.0, theta = 0.0;
    for (int j = 0; j < m; ++j) {
      {  // y1 = S H q
        const int part = tid & (tpr - 1);
        for (int r = tid / tpr; r < un; r += AMMSE_BLOCK / tpr) {
          const cx<R>* __restrict__ hr = Hc + (long)r * M;
          zd acc = {0.0, 0.0};
#pragma unroll 4
          for (int i = part; i < M; i += tpr) acc = acc + to_d(hr[i]) * qv[i];
          for (int o = 1; o < tpr; o <<= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
          }
          if (part == 0) Ly1[r] = scal(sm.invsig[r / N], acc);
        }
      }
      __syncthreads();
      for (int r = tid; r < un; r += AMMSE_BLOCK) {   // y2 = S D y1
        const int u = r / N, n = r - u * N;
        zd acc = {0.0, 0.0};
        for (int k = 0; k < N; ++k) acc = acc + Dm[u * 16 + n * 4 + k] * Ly1[u * N + k];
        Ly2[r] = scal(sm.invsig[u], acc);
      }
      __syncthreads();
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      {  // w = H^H y2 and the inner products
        const int part = tid & (tpc - 1);
        for (int i = tid / tpc; i < M; i += AMMSE_BLOCK / tpc) {
          zd acc = {0.0, 0.0};
#pragma unroll 4
          for (int r = part; r < un; r += tpc) acc = acc + cj(to_d(Hc[(long)r * M + i])) * Ly2[r];
          for (int o = 1; o < tpc; o <<= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
          }
          if (part == 0) {
            wv[i] = acc;
            const zd q = qv[i], pp = pv[i];
            s0 += nrm2(acc);
            s1 += q.x * acc.x + q.y * acc.y;
            s2 += pp.x * acc.x + pp.y * acc.y;
          }
        }
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      __syncthreads();
      if ((tid & 63) == 0) {
        sm.red[(tid >> 6)] = s0;
        sm.red[4 + (tid >> 6)] = s1;
        sm.red[8 + (tid >> 6)] = s2;
      }
      __syncthreads();
      const double ww = (sm.red[0] + sm.red[1]) + (sm.red[2] + sm.red[3]);
      const double al = (sm.red[4] + sm.red[5]) + (sm.red[6] + sm.red[7]);
      const double pw = (sm.red[8] + sm.red[9]) + (sm.red[10] + sm.red[11]);
      double bb;
      if (exact_beta) {
        double nr = 0.0;
        for (int i = tid; i < M; i += AMMSE_BLOCK) {
          const zd w = wv[i] - scal(al, qv[i]) - scal(beta_prev, pv[i]);
          wv[i] = w;
          nr += nrm2(w);
        }
        bb = sqrt(block_sum(nr, sm.red));
      } else {
        bb = sqrt(fmax(ww - al * al - 2.0 * beta_prev * pw + beta_prev * beta_prev, 0.0));
      }
      if (tid == 0) {
        sm.la[j] = al;
        sm.lb[j] = bb;
      }
      const int msz = j + 1;
      tmax = fmax(tmax, fabs(al) + bb);
      const bool breakdown = !(bb > 1e-13 * tmax);
      bool stop = breakdown;
      if (breakdown || (msz >= first && (msz % every) == 0) || msz == m) {
        __syncthreads();
        const double th = (tmax > 0.0) ? tridiag_lmax(sm.la, sm.lb, msz, &sm.imin, rtol) : 0.0;
        stop = stop || fabs(th - theta) <= ltol * fabs(th);
        theta = th;
      }
      if (stop) break;
      __syncthreads();
      const double ib = 1.0 / bb;
      for (int i = tid; i < M; i += AMMSE_BLOCK) {
        const zd w = exact_beta ? wv[i] : wv[i] - scal(al, qv[i]) - scal(beta_prev, pv[i]);
        pv[i] = qv[i];
        qv[i] = scal(ib, w);
      }
      beta_prev = bb;
      __syncthreads();
    }
    __syncthreads();
    return theta;
  };

  // ---- initial state: G^0, copies for the t = 1 extrapolation
  channel_product(Gp, V);
  __syncthreads();
  const int T = p.wsr_only ? 0 : p.max_iters;
  if (!p.wsr_only) {
    const int nv = (int)Vtot, ng = un * D.ud;
#pragma unroll 4
    for (int e = tid; e < nv; e += AMMSE_BLOCK) Vq[e] = V[e];
#pragma unroll 4
    for (int e = tid; e < ng; e += AMMSE_BLOCK) Gq[e] = Gp[e];
  }
  __syncthreads();

  int fsw = p.force_switch_iter;
  if (p.force_switch && p.force_switch[b] > 0) fsw = p.force_switch[b];
  bool stage2 = (fsw >= 1) ? (fsw <= 1) : (p.warm_start == 0);
  int switch_iter = stage2 ? 1 : -1;
  bool prev_step_stage2 = false;
  double wsr_prev = 0.0, wsr_prev2 = 0.0;   // WSR(V^{t-1}), WSR(V^{t-2})
  int iters_run = 0;
  int status = 0;
  zd UW[16], E[16];

  for (int t = 1; t <= T; ++t) {
    // receivers and rate of V^{t-1}
    interference_cov(Gp);
    user_rates(Gp, UW, E);
    __syncthreads();
    wsr_prev2 = wsr_prev;
    wsr_prev = wsr_sum();
    if (p.trace) {
      if (tid == 0) p.trace[(long)b * p.trace_len + (t - 1)] = wsr_prev;
    }
    if (sm.fail) {
      status |= sm.fail;
      break;
    }
    if (!isfinite(wsr_prev)) {
      status |= AMMSE_INST_NONFINITE;
      break;
    }
    if (p.eps2 > 0 && t >= 2 && prev_step_stage2 && rel_change(wsr_prev, wsr_prev2) <= p.eps2)
      break;
    if (!stage2) {
      const bool trig = (fsw >= 1) ? (t >= fsw)
                                   : (t >= 2 && rel_change(wsr_prev, wsr_prev2) <= p.eps1);
      if (trig) {
        stage2 = true;
        switch_iter = t;
      }
    }
    user_weights_ws(UW, E, stage2);

    // step size
    const bool adaptive = t <= p.T_c || (p.rearm && switch_iter >= 1 && t >= switch_iter &&
                                         t < switch_iter + p.T_c);
    if (adaptive) {
      for (int c = 0; c < C; ++c) {
        const double lm = (sm.cu[c] > 0) ? lanczos_lmax(c) : 0.0;
        if (tid == 0) sm.gamma[c] = (lm > 0.0) ? 1.0 / (2.0 * lm) : 0.0;
        __syncthreads();
      }
    } else if (p.gamma_c > 0.0) {
      if (tid < C) sm.gamma[tid] = p.gamma_c;
      __syncthreads();
    }

    // Z = S (D G^ - Y), G^ = (1+w) G^{t-1} - w G^{t-2}
    const double om = p.extrapolate ? fmax((t - 2.0) / (t + 1.0), 0.0) : 0.0;
    for (int c = 0; c < C; ++c) {
      const int nc = sm.cu[c] * d;
      const long base = (long)un * sm.colOff[c];
      // flat element loop (consecutive threads along a row, rows wrap)
      const int ne = un * nc;
      for (int e = tid; e < ne; e += AMMSE_BLOCK) {
        const int r = e / nc, j = e - r * nc;
        const int u = r / N, n = r - u * N;
        zd acc = {0.0, 0.0};
        const long g0 = base + (long)(u * N) * nc + j;
#pragma unroll
        for (int k = 0; k < AMMSE_MAX_RX; ++k) {
          if (k < N) {
            const cx<R> a = Gp[g0 + (long)k * nc], q = Gq[g0 + (long)k * nc];
            const zd gh = {(1.0 + om) * (double)a.x - om * (double)q.x,
                           (1.0 + om) * (double)a.y - om * (double)q.y};
            acc = acc + Dm[u * 16 + n * 4 + k] * gh;
          }
        }
        const int j0 = sm.local[u] * d;
        if (sm.cellOf[u] == c && j >= j0 && j < j0 + d) acc = acc - Ym[u * 16 + n * 4 + (j - j0)];
        Z[base + e] = from_d<R>(scal(sm.invsig[u], acc));
      }
    }
    __syncthreads();

    // gradient: Gr_c = 2 H_c^H Z_c
    for (int c = 0; c < C; ++c) {
      const int nc = sm.cu[c] * d;
      if (nc == 0) continue;
      channel_gemm<R, true>(M, nc, un, H + (long)c * un * M, M, Z + (long)un * sm.colOff[c], nc,
                          Gr + (long)M * sm.colOff[c], nc, R(2), nullptr, 1, sm.As, sm.Bs);
    }
    __syncthreads();

    // extrapolated projected step per BS
    for (int c = 0; c < C; ++c) {
      const int nc = sm.cu[c] * d;
      const long base = (long)M * sm.colOff[c];
      const long n = (long)M * nc;
      const double g = sm.gamma[c];
      double pw = 0.0;
      const int ni = (int)n;
      cx<R>* __restrict__ Vb = V + base;
      cx<R>* __restrict__ Vqb = Vq + base;
      cx<R>* __restrict__ Grb = Gr + base;
#pragma unroll 4
      for (int e = tid; e < ni; e += AMMSE_BLOCK) {
        const zd v = to_d(Vb[e]), vq = to_d(Vqb[e]), gr = to_d(Grb[e]);
        const zd x = {(1.0 + om) * v.x - om * vq.x - g * gr.x, (1.0 + om) * v.y - om * vq.y - g * gr.y};
        const cx<R> xs = from_d<R>(x);
        Grb[e] = xs;
        pw += nrm2(to_d(xs));
      }
      pw = block_sum(pw, sm.red);
      const double s = (pw > sm.Pc[c]) ? sqrt(sm.Pc[c] / pw) : 1.0;
#pragma unroll 4
      for (int e = tid; e < ni; e += AMMSE_BLOCK) {
        Vqb[e] = Vb[e];
        Vb[e] = from_d<R>(scal(s, to_d(Grb[e])));
      }
    }
    __syncthreads();

    // G^{t} = S H V^t ; keep G^{t-1}
    {
      cx<R>* tmp = Gq;
      Gq = Gp;
      Gp = tmp;
    }
    channel_product(Gp, V);
    __syncthreads();
    prev_step_stage2 = stage2;
    iters_run = t;
  }

  // ---- WSR of the returned precoders
  double wsr_final;
  if (iters_run == T && !status) {
    interference_cov(Gp);
    user_rates(Gp, UW, E);
    __syncthreads();
    wsr_final = wsr_sum();
    if (sm.fail) status |= sm.fail;
    if (!isfinite(wsr_final)) status |= AMMSE_INST_NONFINITE;
    if (p.trace && tid == 0) p.trace[(long)b * p.trace_len + T] = wsr_final;
  } else {
    wsr_final = wsr_prev;   // stopped early: V holds V^{iters_run}, WSR already known
  }
  // zero-power check
  for (int c = 0; c < C; ++c) {
    const long base = (long)M * sm.colOff[c];
    const long n = (long)M * sm.cu[c] * d;
    double pw = 0.0;
    for (int e = tid; e < (int)n; e += AMMSE_BLOCK) pw += nrm2(to_d(V[base + e]));
    pw = block_sum(pw, sm.red);
    if (n > 0 && pw == 0.0) status |= AMMSE_INST_ZERO_POWER;
  }
  if (tid == 0) {
    p.wsr[b] = wsr_final;
    if (p.iters) p.iters[b] = iters_run;
    if (p.switch_iter) p.switch_iter[b] = p.wsr_only ? -1 : switch_iter;
    if (p.status) p.status[b] = status;
  }
  if (p.trace) {
    const int last = (iters_run == T && !(status & (AMMSE_INST_CHOLESKY | AMMSE_INST_NONFINITE)))
                         ? T : iters_run;
    for (int k = last + 1 + tid; k <= T; k += AMMSE_BLOCK)
      p.trace[(long)b * p.trace_len + k] = NAN;
  }
}

}  // namespace

size_t ammse_general_lds_bytes(int precision) {
  return precision == AMMSE_PREC_FP64 ? sizeof(Smem<double>) : sizeof(Smem<float>);
}

hipError_t ammse_launch_fp64(const ammse_kparams_t& p, hipStream_t s) {
  hipLaunchKernelGGL(ammse_solve_kernel<double>, dim3(p.batch), dim3(AMMSE_BLOCK), 0, s, p);
  return hipGetLastError();
}

hipError_t ammse_launch_fp32(const ammse_kparams_t& p, hipStream_t s) {
  hipLaunchKernelGGL(ammse_solve_kernel<float>, dim3(p.batch), dim3(AMMSE_BLOCK), 0, s, p);
  return hipGetLastError();
}
