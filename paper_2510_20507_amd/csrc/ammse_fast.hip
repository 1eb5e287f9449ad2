// LDS-resident A-MMMSE solve kernel on MFMA (FP32 storage), gfx950.
//
// For single-cell instances whose stacked channel H (U*N x M), precoders
// (M x U*d) and channel product (U*N x U*d) fit in LDS together, one
// workgroup of 256 threads (4 waves) loads H once and keeps it in LDS for
// all iterations; HBM is touched only to read H, V0 and the per-user
// scalars and to write the results.  The two complex channel products per
// iteration run on v_mfma_f32_16x16x4f32: a complex product is three real
// accumulators (Re*Re, Im*Im, Re*Im + Im*Re), fed from interleaved complex
// LDS tiles.  Each wave owns whole 16-row strips of the outputs, so the
// iteration state lives in registers in the MFMA output layout:
//   G^{t-1}, G^{t-2} (for the extrapolated product by linearity) and
//   V^{t-1}, V^{t-2} (for the extrapolated precoder).
// A lane holds 4 consecutive rows of one column; with N in {1, 2, 4} these
// are whole users, so Z = S (D G^ - Y) is formed in registers.
//
// Per iteration (Algorithm 3 with the readings of the generic kernel):
//   Gs <- G^{t-1}; per-user J-, Cholesky, rate, U, W (double);
//   WSR(V^{t-1}), stage latch, adaptive step by Lanczos on H in LDS;
//   Z -> LDS; Grad = 2 H^H Z (MFMA); V^t = Pi(V^ - gamma Grad) in registers;
//   V^t -> LDS; G^t = S H V^t (MFMA).

#include "ammse_device.h"

namespace {
using namespace ammse_dev;

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int MB_, int UNB_, int UDB_>
struct Shape {
  static constexpr int MB = MB_, UNB = UNB_, UDB = UDB_;
  static constexpr int M = 16 * MB, UN = 16 * UNB, UD = 16 * UDB;
  static constexpr int HLD = M + 2;                 // padded LDS row strides (complex)
  static constexpr int BROWS = (M > UN) ? M : UN;
  static constexpr int BLD = UD + 2;
  static constexpr int GLD = UD + 2;
  static constexpr int GRB = UNB / 4;               // row blocks per wave in G
  static constexpr int VRB = MB / 4;                // row blocks per wave in V / Grad
  static constexpr int MAXU = UN;                   // U <= U*N
  static_assert(MB % 4 == 0 && UNB % 4 == 0, "row blocks must split over 4 waves");
  // LDS carve (bytes)
  static constexpr size_t oH = 0;
  static constexpr size_t oB = oH + sizeof(float2) * UN * HLD;
  static constexpr size_t oG = oB + sizeof(float2) * BROWS * BLD;
  static constexpr size_t oD = oG + sizeof(float2) * UN * GLD;
  static constexpr size_t oY = oD + sizeof(float2) * MAXU * 16;
  static constexpr size_t oJ = oY + sizeof(float2) * MAXU * 16;     // J-: U*N*N <= 4*U*N
  static constexpr size_t oQ = oJ + sizeof(zd) * 4 * UN;            // 3 Lanczos vectors
  static constexpr size_t oY1 = oQ + sizeof(zd) * 3 * M;
  static constexpr size_t oY2 = oY1 + sizeof(zd) * UN;
  static constexpr size_t oS = oY2 + sizeof(zd) * UN;               // invsig, alpha, rate
  static constexpr size_t oL = oS + sizeof(double) * 3 * MAXU;      // la, lb
  static constexpr size_t oR = oL + sizeof(double) * 2 * AMMSE_MAX_LANCZOS;
  static constexpr size_t bytes = oR + sizeof(double) * 8 + 16;
};

__device__ __forceinline__ float2 c2(float x, float y) { return make_float2(x, y); }

// g[i] for a run-time i in [0, 4) without dynamic register indexing.
__device__ __forceinline__ float2 pick4(const float2 (&g)[4], int i) {
  float2 r = g[0];
  r = (i == 1) ? g[1] : r;
  r = (i == 2) ? g[2] : r;
  r = (i == 3) ? g[3] : r;
  return r;
}

// One wave: P[i][j] (three real accumulators) += op(A) B for the wave's row
// blocks i (global row block wave + 4 i) and all column blocks j.
// op(A)[r][k] = A[r*lda + k], or conj(A[k*lda + r]) with CONJA.
template <int NRB, int NCB, bool CONJA>
__device__ __forceinline__ void wave_cgemm(const float2* __restrict__ A, int lda,
                                           const float2* __restrict__ B, int ldb, int K,
                                           int wave, floatx4 (&P)[NRB][NCB][3]) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < NRB; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) P[i][j][q] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int k0 = 0; k0 < K; k0 += 4) {
    float2 a[NRB], b[NCB];
    const int kk = k0 + lk;
#pragma unroll
    for (int i = 0; i < NRB; ++i) {
      const int r = 16 * (wave + 4 * i) + li;
      if (CONJA) {
        const float2 h = A[kk * lda + r];
        a[i] = c2(h.x, -h.y);
      } else {
        a[i] = A[r * lda + kk];
      }
    }
#pragma unroll
    for (int j = 0; j < NCB; ++j) b[j] = B[kk * ldb + 16 * j + li];
#pragma unroll
    for (int i = 0; i < NRB; ++i)
#pragma unroll
      for (int j = 0; j < NCB; ++j)
        P[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, b[j].x, P[i][j][0], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NRB; ++i)
#pragma unroll
      for (int j = 0; j < NCB; ++j)
        P[i][j][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, b[j].y, P[i][j][1], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NRB; ++i)
#pragma unroll
      for (int j = 0; j < NCB; ++j)
        P[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, b[j].y, P[i][j][2], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NRB; ++i)
#pragma unroll
      for (int j = 0; j < NCB; ++j)
        P[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, b[j].x, P[i][j][2], 0, 0, 0);
  }
}

template <class S>
__global__ __launch_bounds__(256) void ammse_fast_kernel(ammse_kparams_t p) {
  extern __shared__ __align__(16) char smem[];
  float2* Hs = (float2*)(smem + S::oH);
  float2* Bs = (float2*)(smem + S::oB);
  float2* Gs = (float2*)(smem + S::oG);
  float2* Ds = (float2*)(smem + S::oD);
  float2* Ys = (float2*)(smem + S::oY);
  zd* Jm = (zd*)(smem + S::oJ);
  zd* Lq = (zd*)(smem + S::oQ);
  zd* Ly1 = (zd*)(smem + S::oY1);
  zd* Ly2 = (zd*)(smem + S::oY2);
  double* invsig = (double*)(smem + S::oS);
  double* alpha = invsig + S::MAXU;
  double* rate = alpha + S::MAXU;
  double* la = (double*)(smem + S::oL);
  double* lb = la + AMMSE_MAX_LANCZOS;
  double* red = (double*)(smem + S::oR);
  int* misc = (int*)(red + 8);      // [0] fail flag, [1] multisection index

  constexpr int M = S::M, UN = S::UN, UD = S::UD;
  const ammse_desc_t Dd = p.desc[blockIdx.x];
  const int U = Dd.U, N = Dd.N, d = Dd.d;
  const int b = Dd.b;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;

  const float2* Hg = (const float2*)p.H + Dd.h_off;
  float2* Vg = (float2*)p.V + Dd.v_off;
  const double Pc = p.wsr_only ? 0.0 : p.P[Dd.bs_off];

  for (int u = tid; u < U; u += 256) {
    invsig[u] = 1.0 / sqrt(p.sigma2[Dd.user_off + u]);
    alpha[u] = p.alpha[Dd.user_off + u];
  }
  if (tid == 0) misc[0] = 0;
  for (int e = tid; e < UN * M; e += 256) Hs[(e / M) * S::HLD + (e % M)] = Hg[e];
  for (int e = tid; e < M * UD; e += 256) Bs[(e / UD) * S::BLD + (e % UD)] = Vg[e];
  __syncthreads();

  // register state in the MFMA output layout:
  // element [i][j][r] is row 16 (wave + 4 i) + 4 lk + r, column 16 j + li
  float2 Vp[S::VRB][S::UDB][4], Vq[S::VRB][S::UDB][4];
  float2 Gp[S::GRB][S::UDB][4], Gq[S::GRB][S::UDB][4];
#pragma unroll
  for (int i = 0; i < S::VRB; ++i)
#pragma unroll
    for (int j = 0; j < S::UDB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
        Vp[i][j][r] = Bs[row * S::BLD + col];
        Vq[i][j][r] = Vp[i][j][r];
      }

  // G = S H V (from Bs) into Gp, and the copy in Gs for the per-user phase
  auto product_G = [&]() {
    floatx4 P[S::GRB][S::UDB][3];
    wave_cgemm<S::GRB, S::UDB, false>(Hs, S::HLD, Bs, S::BLD, M, wave, P);
#pragma unroll
    for (int i = 0; i < S::GRB; ++i)
#pragma unroll
      for (int j = 0; j < S::UDB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
          const float s = (float)invsig[row / N];
          const float2 g = c2(s * (P[i][j][0][r] - P[i][j][1][r]), s * P[i][j][2][r]);
          Gq[i][j][r] = Gp[i][j][r];
          Gp[i][j][r] = g;
          Gs[row * S::GLD + col] = g;
        }
  };

  // receivers and rates of the precoders whose product is in Gs
  zd UW[16], E[16];
  auto receivers = [&]() {
    const int np = N * (N + 1) / 2;
    for (int e = tid; e < U * np; e += 256) {
      const int u = e / np;
      int q = e % np, n1 = 0;
      while (q >= N - n1) {
        q -= N - n1;
        ++n1;
      }
      const int n2 = n1 + q;
      const float2* r1 = Gs + (u * N + n1) * S::GLD;
      const float2* r2 = Gs + (u * N + n2) * S::GLD;
      const int j0 = u * d;
      zd acc = {0.0, 0.0};
      for (int j = 0; j < UD; ++j) {
        if (j >= j0 && j < j0 + d) continue;
        acc.x += (double)r1[j].x * r2[j].x + (double)r1[j].y * r2[j].y;
        acc.y += (double)r1[j].y * r2[j].x - (double)r1[j].x * r2[j].y;
      }
      if (n1 == n2) acc = {acc.x + 1.0, 0.0};
      Jm[(u * N + n1) * N + n2] = acc;
      Jm[(u * N + n2) * N + n1] = cj(acc);
    }
    __syncthreads();
    // user u on thread (u % 4) * 64 + u / 4: spreads the users over the 4 SIMDs
    const int u = (tid & 63) * 4 + (tid >> 6);
    if ((tid & 63) < (U + 3) / 4 && u < U) {
      zd J[16], F[16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          J[i * 4 + j] = (i < N && j < N) ? Jm[(u * N + i) * N + j]
                                          : zd{(i == j) ? 1.0 : 0.0, 0.0};
          F[i * 4 + j] = {0.0, 0.0};
          if (i < N && j < d) {
            const float2 g = Gs[(u * N + i) * S::GLD + u * d + j];
            F[i * 4 + j] = {(double)g.x, (double)g.y};
          }
        }
      double rr;
      const bool ok = user_receiver(J, F, UW, E, &rr);
      rate[u] = alpha[u] * rr;
      if (!ok) atomicOr(&misc[0], AMMSE_INST_CHOLESKY);
    }
  };
  auto wsr_sum = [&]() {
    double v = 0.0;
    for (int u = tid; u < U; u += 256) v += rate[u];
    return block_sum(v, red) * (1.0 / M_LN2);
  };
  auto weights = [&](bool stage2) {
    const int u = (tid & 63) * 4 + (tid >> 6);
    if ((tid & 63) < (U + 3) / 4 && u < U) {
      zd Dl[16], Yl[16];
      user_weights(UW, E, stage2, alpha[u], Dl, Yl);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        Ds[u * 16 + i] = c2((float)Dl[i].x, (float)Dl[i].y);
        Ys[u * 16 + i] = c2((float)Yl[i].x, (float)Yl[i].y);
      }
    }
    __syncthreads();
  };

  // lambda_max(H^H S D S H) by plain Lanczos, everything in LDS
  auto lanczos = [&]() {
    zd* qa = Lq;
    zd* qb = Lq + M;
    zd* qc = Lq + 2 * M;
    for (int i = tid; i < M; i += 256) {
      qb[i] = {1.0 + 0.5 * sin(0.731 * i + 0.25), 0.3 * cos(1.37 * i + 0.5)};
      qa[i] = {0.0, 0.0};
    }
    double nn = 0.0;
    for (int i = tid; i < M; i += 256) nn += nrm2(qb[i]);
    nn = block_sum(nn, red);
    for (int i = tid; i < M; i += 256) qb[i] = scal(1.0 / sqrt(nn), qb[i]);
    __syncthreads();
    const int m = min(p.lanczos_steps, M);
    const double ltol = 1e-10;
    double beta_prev = 0.0, tmax = 0.0, theta = 0.0;
    constexpr int TPR = 256 / UN;          // threads per row of H
    constexpr int TPC = 256 / M;           // threads per column of H
    for (int j = 0; j < m; ++j) {
      {  // y1 = S H q
        const int r = tid / TPR, part = tid % TPR;
        zd acc = {0.0, 0.0};
        for (int c = part; c < M; c += TPR) {
          const float2 h = Hs[r * S::HLD + c];
          acc = acc + zd{(double)h.x, (double)h.y} * qb[c];
        }
#pragma unroll
        for (int o = 1; o < TPR; o <<= 1) {
          acc.x += __shfl_xor(acc.x, o, 64);
          acc.y += __shfl_xor(acc.y, o, 64);
        }
        if (part == 0) Ly1[r] = scal(invsig[r / N], acc);
      }
      __syncthreads();
      for (int r = tid; r < UN; r += 256) {   // y2 = S D y1
        const int u = r / N, n = r % N;
        zd acc = {0.0, 0.0};
        for (int k = 0; k < N; ++k) {
          const float2 dd = Ds[u * 16 + n * 4 + k];
          acc = acc + zd{(double)dd.x, (double)dd.y} * Ly1[u * N + k];
        }
        Ly2[r] = scal(invsig[u], acc);
      }
      __syncthreads();
      double al = 0.0;
      {  // w = H^H y2
        const int c = tid / TPC, part = tid % TPC;
        zd acc = {0.0, 0.0};
        for (int r = part; r < UN; r += TPC) {
          const float2 h = Hs[r * S::HLD + c];
          acc = acc + zd{(double)h.x, -(double)h.y} * Ly2[r];
        }
#pragma unroll
        for (int o = 1; o < TPC; o <<= 1) {
          acc.x += __shfl_xor(acc.x, o, 64);
          acc.y += __shfl_xor(acc.y, o, 64);
        }
        if (part == 0) {
          qc[c] = acc;
          al = qb[c].x * acc.x + qb[c].y * acc.y;
        }
      }
      al = block_sum(al, red);
      double bb = 0.0;
      for (int i = tid; i < M; i += 256) {
        const zd w = qc[i] - scal(al, qb[i]) - scal(beta_prev, qa[i]);
        qc[i] = w;
        bb += nrm2(w);
      }
      bb = sqrt(block_sum(bb, red));
      if (tid == 0) {
        la[j] = al;
        lb[j] = bb;
      }
      const int msz = j + 1;
      tmax = fmax(tmax, fabs(al) + bb);
      const bool breakdown = !(bb > 1e-13 * tmax);
      if (breakdown || (msz % 8) == 0 || msz == m) {
        __syncthreads();
        const double th = (tmax > 0.0) ? tridiag_lmax(la, lb, msz, &misc[1]) : 0.0;
        const bool conv = fabs(th - theta) <= ltol * fabs(th);
        theta = th;
        if (breakdown || conv) break;
      }
      const double ib = 1.0 / bb;
      for (int i = tid; i < M; i += 256) {
        qa[i] = qb[i];
        qb[i] = scal(ib, qc[i]);
      }
      beta_prev = bb;
      __syncthreads();
    }
    __syncthreads();
    return theta;
  };

  product_G();
  __syncthreads();
#pragma unroll
  for (int i = 0; i < S::GRB; ++i)
#pragma unroll
    for (int j = 0; j < S::UDB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) Gq[i][j][r] = Gp[i][j][r];

  const int T = p.wsr_only ? 0 : p.max_iters;
  int fsw = p.force_switch_iter;
  if (p.force_switch && p.force_switch[b] > 0) fsw = p.force_switch[b];
  bool stage2 = (fsw >= 1) ? (fsw <= 1) : (p.warm_start == 0);
  int switch_iter = stage2 ? 1 : -1;
  bool prev_step_stage2 = false;
  double wsr_prev = 0.0, wsr_prev2 = 0.0, gamma = 0.0;
  int iters_run = 0, status = 0;

  for (int t = 1; t <= T; ++t) {
    receivers();
    __syncthreads();
    wsr_prev2 = wsr_prev;
    wsr_prev = wsr_sum();
    if (p.trace && tid == 0) p.trace[(long)b * p.trace_len + (t - 1)] = wsr_prev;
    if (misc[0]) {
      status |= misc[0];
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
    weights(stage2);
    const bool adaptive = t <= p.T_c || (p.rearm && switch_iter >= 1 && t >= switch_iter &&
                                         t < switch_iter + p.T_c);
    if (adaptive) {
      const double lm = lanczos();
      gamma = (lm > 0.0) ? 1.0 / (2.0 * lm) : 0.0;
    } else if (p.gamma_c > 0.0) {
      gamma = p.gamma_c;
    }

    // Z = S (D G^ - Y) from the registers, into Bs
    const float om = p.extrapolate ? (float)fmax((t - 2.0) / (t + 1.0), 0.0) : 0.f;
#pragma unroll
    for (int i = 0; i < S::GRB; ++i)
#pragma unroll
      for (int j = 0; j < S::UDB; ++j) {
        float2 gh[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          gh[r] = c2((1.f + om) * Gp[i][j][r].x - om * Gq[i][j][r].x,
                     (1.f + om) * Gp[i][j][r].y - om * Gq[i][j][r].y);
        const int row0 = 16 * (wave + 4 * i) + 4 * lk, col = 16 * j + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + r, u = row / N, n = row % N, base = u * N - row0;
          float zx = 0.f, zy = 0.f;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (k < N) {
              const float2 dd = Ds[u * 16 + n * 4 + k];
              const float2 g = pick4(gh, base + k);
              zx += dd.x * g.x - dd.y * g.y;
              zy += dd.x * g.y + dd.y * g.x;
            }
          }
          const int s = col - u * d;
          if (s >= 0 && s < d) {
            const float2 y = Ys[u * 16 + n * 4 + s];
            zx -= y.x;
            zy -= y.y;
          }
          const float is = (float)invsig[u];
          Bs[row * S::BLD + col] = c2(is * zx, is * zy);
        }
      }
    __syncthreads();

    // gradient and the extrapolated projected step, in registers
    {
      floatx4 P[S::VRB][S::UDB][3];
      wave_cgemm<S::VRB, S::UDB, true>(Hs, S::HLD, Bs, S::BLD, UN, wave, P);
      const float g2 = (float)(2.0 * gamma);
      double pw = 0.0;
#pragma unroll
      for (int i = 0; i < S::VRB; ++i)
#pragma unroll
        for (int j = 0; j < S::UDB; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float gx = P[i][j][0][r] - P[i][j][1][r], gy = P[i][j][2][r];
            const float2 v = Vp[i][j][r], q = Vq[i][j][r];
            const float2 x = c2((1.f + om) * v.x - om * q.x - g2 * gx,
                                (1.f + om) * v.y - om * q.y - g2 * gy);
            Vq[i][j][r] = x;     // temporarily holds V~
            pw += (double)x.x * x.x + (double)x.y * x.y;
          }
      pw = block_sum(pw, red);
      const float sc = (pw > Pc) ? (float)sqrt(Pc / pw) : 1.f;
#pragma unroll
      for (int i = 0; i < S::VRB; ++i)
#pragma unroll
        for (int j = 0; j < S::UDB; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float2 x = Vq[i][j][r];
            const float2 vn = c2(sc * x.x, sc * x.y);
            Vq[i][j][r] = Vp[i][j][r];
            Vp[i][j][r] = vn;
            const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
            Bs[row * S::BLD + col] = vn;
          }
    }
    __syncthreads();
    product_G();
    __syncthreads();
    prev_step_stage2 = stage2;
    iters_run = t;
  }

  double wsr_final;
  if (iters_run == T && !status) {
    receivers();
    __syncthreads();
    wsr_final = wsr_sum();
    if (misc[0]) status |= misc[0];
    if (!isfinite(wsr_final)) status |= AMMSE_INST_NONFINITE;
    if (p.trace && tid == 0) p.trace[(long)b * p.trace_len + T] = wsr_final;
  } else {
    wsr_final = wsr_prev;
  }
  double pw = 0.0;
#pragma unroll
  for (int i = 0; i < S::VRB; ++i)
#pragma unroll
    for (int j = 0; j < S::UDB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float2 v = Vp[i][j][r];
        pw += (double)v.x * v.x + (double)v.y * v.y;
        if (!p.wsr_only) {
          const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
          Vg[row * UD + col] = v;
        }
      }
  pw = block_sum(pw, red);
  if (pw == 0.0) status |= AMMSE_INST_ZERO_POWER;
  if (tid == 0) {
    p.wsr[b] = wsr_final;
    if (p.iters) p.iters[b] = iters_run;
    if (p.switch_iter) p.switch_iter[b] = p.wsr_only ? -1 : switch_iter;
    if (p.status) p.status[b] = status;
  }
  if (p.trace) {
    const int last = (iters_run == T && !(status & (AMMSE_INST_CHOLESKY | AMMSE_INST_NONFINITE)))
                         ? T : iters_run;
    for (int k = last + 1 + tid; k <= T; k += 256) p.trace[(long)b * p.trace_len + k] = NAN;
  }
}

using Shape64 = Shape<4, 4, 4>;   // M = 64, U*N = 64, U*d = 64

}  // namespace

// Instance shapes served by the LDS-resident kernel.
bool ammse_fast_eligible(int C, int U, int M, int N, int d) {
  return C == 1 && M == Shape64::M && U * N == Shape64::UN && U * d == Shape64::UD &&
         (N == 1 || N == 2 || N == 4);
}

size_t ammse_fast_lds_bytes() { return Shape64::bytes; }

hipError_t ammse_launch_fast_fp32(const ammse_kparams_t& p, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)ammse_fast_kernel<Shape64>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)Shape64::bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(ammse_fast_kernel<Shape64>, dim3(p.batch), dim3(256), Shape64::bytes, s, p);
  return hipGetLastError();
}
