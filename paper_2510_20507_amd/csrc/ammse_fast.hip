// LDS-resident A-MMMSE solve kernel on MFMA (FP32 storage), gfx950.
//
// For single-cell instances with M = 64 and U*N = U*d = 64, one workgroup of
// 256 threads (4 waves) owns one instance for the whole solve; H stays in
// LDS for all iterations and HBM is touched only to read H, V0 and the
// per-user scalars and to write the results.  LDS use is kept under 80 KiB
// so that two instances share a compute unit and one instance's serial
// phases overlap the other's matrix products.
//
// Channel products: v_mfma_f32_16x16x4f32, a complex product being three
// real accumulators (Re*Re, Im*Im, Re*Im + Im*Re) fed from interleaved
// complex LDS tiles.  Each wave owns whole 16-row strips of the outputs, so
// the iteration state stays in registers in the MFMA output layout:
//   G^{t-1}, G^{t-2}  (the extrapolated product follows by linearity)
//   V^{t-1}, V^{t-2}  (the extrapolated precoder)
// A lane holds 4 consecutive rows of one column.  Four consecutive rows form
// a "block user": one user for N = 4, two for N = 2, four for N = 1; its
// N x N and d x d algebra is done as one block-diagonal 4 x 4 problem.
//
// Per-user algebra (Section IV equations for U and W, in the Woodbury form
// used throughout this library) runs lane-parallel in double: the 16 lanes
// of a 4-lane-row group hold the 16 entries of a 4 x 4 complex matrix and
// exchange them with cross-lane shuffles.  The interference-plus-noise
// covariance of every user is reduced directly from the G registers.
//
// Per iteration t (Algorithm 3):
//   J- from registers (reduce-scatter over the 16 lanes of a row group);
//   Cholesky, rate, U, W per block user; WSR(V^{t-1}); stage latch;
//   adaptive step by Lanczos on H in LDS;  Z = S (D G^ - Y) -> LDS;
//   Grad = 2 H^H Z (MFMA);  V^t = Pi(V^ - gamma Grad) in registers -> LDS;
//   G^t = S H V^t (MFMA), own blocks -> LDS.

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
  static constexpr int GRB = UNB / 4;               // row blocks per wave in G
  static constexpr int VRB = MB / 4;                // row blocks per wave in V / Grad
  static constexpr int NG = UN / 4;                 // block users (4 rows each)
  static_assert(MB % 4 == 0 && UNB % 4 == 0, "row blocks must split over 4 waves");
  // LDS carve (bytes)
  static constexpr size_t oH = 0;
  static constexpr size_t oB = oH + sizeof(float2) * UN * HLD;
  static constexpr size_t oF = oB + sizeof(float2) * BROWS * BLD;   // own blocks of G
  static constexpr size_t oD = oF + sizeof(float2) * NG * 16;       // D per block user
  static constexpr size_t oY = oD + sizeof(float2) * NG * 16;       // Y per block user
  static constexpr size_t oQ = oY + sizeof(float2) * NG * 16;       // S H H^H S (UN x UN)
  static constexpr size_t QLD = UN + 2;
  static constexpr size_t oC = oQ + sizeof(float2) * UN * QLD;      // C per block user (D = C C^H)
  static constexpr size_t oS = oC + sizeof(zd) * NG * 16;           // invsig, alpha per row
  static constexpr size_t oL = oS + sizeof(double) * 2 * UN;        // la, lb
  static constexpr size_t oR = oL + sizeof(double) * 2 * AMMSE_MAX_LANCZOS;
  static constexpr size_t bytes = oR + sizeof(double) * 8 + 16;
  // Lanczos vectors alias the product-operand area, which is free between
  // the last product of an iteration and the Z build.
  static_assert(sizeof(zd) * 2 * UN + 64 * sizeof(double) <= sizeof(float2) * BROWS * BLD,
                "Lanczos area");
};

__device__ __forceinline__ float2 c2(float x, float y) { return make_float2(x, y); }

// One wave: P[i][j] (three real accumulators) = op(A) B for the wave's row
// blocks i (global row block wave + 4 i) and all column blocks j.
// op(A)[r][k] = A[r*lda + k], or conj(A[k*lda + r]) with CONJA; B[k][j] is
// B[k*ldb + j], or conj(B[j*ldb + k]) with CONJBT.
template <int NRB, int NCB, bool CONJA, bool CONJBT = false>
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
    for (int j = 0; j < NCB; ++j) {
      if (CONJBT) {
        const float2 h = B[(16 * j + li) * ldb + kk];
        b[j] = c2(h.x, -h.y);
      } else {
        b[j] = B[kk * ldb + 16 * j + li];
      }
    }
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

// Largest eigenvalue of a symmetric tridiagonal matrix (la, lb in LDS, m x m)
// by multisection inside one wave: 64 probes per round on Sturm counts.

__device__ __forceinline__ double wave_tridiag_lmax(const double* la, const double* lb, int m,
                                                    double rtol) {
  const int lane = threadIdx.x & 63;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? fabs(lb[i - 1]) : 0.0) + (i < m - 1 ? fabs(lb[i]) : 0.0);
    lo = fmin(lo, la[i] - r);
    hi = fmax(hi, la[i] + r);
  }
  hi += fabs(hi) * 1e-6 + 1e-300;
  for (int round = 0; round < 8; ++round) {
    const double w = hi - lo;
    if (!(w > fabs(hi) * rtol)) break;
    const double x = lo + w * (double)(lane + 1) / 65.0;
    const bool full = sturm_below(la, lb, m, x) == m;
    const unsigned long long mask = __ballot(full);
    const int t = mask ? (__ffsll((long long)mask) - 1) : 64;
    const double nhi = (t < 64) ? lo + w * (double)(t + 1) / 65.0 : hi;
    const double nlo = (t > 0) ? lo + w * (double)t / 65.0 : lo;
    lo = nlo;
    hi = nhi;
  }
  return hi;
}

template <class S>
__global__ __launch_bounds__(256, 1) void ammse_fast_kernel(ammse_kparams_t p) {
  extern __shared__ __align__(16) char smem[];
  float2* Hs = (float2*)(smem + S::oH);
  float2* Bs = (float2*)(smem + S::oB);
  float2* Fs = (float2*)(smem + S::oF);
  float2* Ds = (float2*)(smem + S::oD);
  float2* Ys = (float2*)(smem + S::oY);
  float2* Qs = (float2*)(smem + S::oQ);
  zd* Cs = (zd*)(smem + S::oC);
  double* invsig = (double*)(smem + S::oS);    // per row: 1/sigma of the row's user
  double* alpha = invsig + S::UN;              // per row: alpha of the row's user
  double* la = (double*)(smem + S::oL);
  double* lb = la + AMMSE_MAX_LANCZOS;
  double* red = (double*)(smem + S::oR);
  int* misc = (int*)(red + 8);                 // [0] fail flag, [1] multisection index
  zd* Lq = (zd*)Bs;                            // Lanczos vectors (alias, see Shape)

  constexpr int M = S::M, UN = S::UN, UD = S::UD;
  const ammse_desc_t Dd = p.desc[blockIdx.x];
  const int N = Dd.N, d = Dd.d;
  const int lgN = __builtin_ctz(N), lgd = __builtin_ctz(d);   // N, d in {1, 2, 4}
  const int b = Dd.b;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const Lane4 L4{lane & ~15, li >> 2, li & 3};

  const float2* Hg = (const float2*)p.H + Dd.h_off;
  float2* Vg = (float2*)p.V + Dd.v_off;
  const double Pc = p.wsr_only ? 0.0 : p.P[Dd.bs_off];

  for (int r = tid; r < UN; r += 256) {
    invsig[r] = 1.0 / sqrt(p.sigma2[Dd.user_off + r / N]);
    alpha[r] = p.alpha[Dd.user_off + r / N];
  }
  for (int e = tid; e < S::NG * 16; e += 256) Fs[e] = c2(0.f, 0.f);
  if (tid == 0) misc[0] = 0;
  for (int e = tid; e < UN * M; e += 256) Hs[(e / M) * S::HLD + (e % M)] = Hg[e];
  for (int e = tid; e < M * UD; e += 256) Bs[(e / UD) * S::BLD + (e % UD)] = Vg[e];
  __syncthreads();

  // register state: element [i][j][r] is row 16 (wave + 4 i) + 4 lk + r,
  // column 16 j + li
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

  // Q = S H H^H S for the step-size operator, once per solve
  {
    floatx4 P[S::GRB][S::UNB][3];
    wave_cgemm<S::GRB, S::UNB, false, true>(Hs, S::HLD, Hs, S::HLD, M, wave, P);
#pragma unroll
    for (int i = 0; i < S::GRB; ++i)
#pragma unroll
      for (int j = 0; j < S::UNB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
          const float s = (float)(invsig[row] * invsig[col]);
          Qs[row * S::QLD + col] = c2(s * (P[i][j][0][r] - P[i][j][1][r]), s * P[i][j][2][r]);
        }
    __syncthreads();
    for (int e = tid; e < UN * UN; e += 256) {      // exactly Hermitian
      const int r = e / UN, c = e % UN;
      if (r < c) {
        const float2 x = Qs[r * S::QLD + c], y = Qs[c * S::QLD + r];
        const float2 mm = c2(0.5f * (x.x + y.x), 0.5f * (x.y - y.y));
        Qs[r * S::QLD + c] = mm;
        Qs[c * S::QLD + r] = c2(mm.x, -mm.y);
      } else if (r == c) {
        Qs[r * S::QLD + c].y = 0.f;
      }
    }
    __syncthreads();
  }

  // G = S H V (V in Bs) into Gp (previous Gp to Gq); own blocks into Fs
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
          const float s = (float)invsig[row];
          const float2 g = c2(s * (P[i][j][0][r] - P[i][j][1][r]), s * P[i][j][2][r]);
          Gq[i][j][r] = Gp[i][j][r];
          Gp[i][j][r] = g;
          const int u = row >> lgN, c = col - (u << lgd);
          if (c >= 0 && c < d) {
            const int g4 = row >> 2, u0 = (g4 * 4) >> lgN;
            Fs[g4 * 16 + r * 4 + ((u - u0) << lgN) + c] = g;
          }
        }
  };

  // Per block user (i = row block of this wave, group lk): J-, Cholesky,
  // rate, UW = J-^{-1} G_own and E = (I + G_own^H J-^{-1} G_own)^{-1}.
  // Returns the weighted rate contribution of this lane (diagonal lanes).
  zd UWr[S::GRB], Er[S::GRB], Lir[S::GRB];
  auto receivers = [&]() {
    double rsum = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < S::GRB; ++i) {
      const int row0 = 16 * (wave + 4 * i) + 4 * lk;
      // partial J over this lane's columns, all 16 entries (a, b)
      zd s[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) s[e] = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < S::UDB; ++j) {
        const int col = 16 * j + li;
        zd g[4];
        bool own[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          g[r] = {(double)Gp[i][j][r].x, (double)Gp[i][j][r].y};
          own[r] = (col >> lgd) == ((row0 + r) >> lgN);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const bool use = ((row0 + a) >> lgN == (row0 + c) >> lgN) && !own[a];
            const zd t = mulc(g[a], g[c]);
            if (use) s[a * 4 + c] = s[a * 4 + c] + t;
          }
      }
      // reduce-scatter over the 16 lanes: lane li ends with entry li
#pragma unroll
      for (int step = 0; step < 4; ++step) {
        const int bit = 8 >> step;                 // 8, 4, 2, 1
        const int half = bit;                      // entries exchanged
        const bool hi = (li & bit) != 0;
#pragma unroll
        for (int e = 0; e < half; ++e) {
          const zd keep = hi ? s[e + half] : s[e];
          const zd send = hi ? s[e] : s[e + half];
          const zd got = {__shfl_xor(send.x, bit, 64), __shfl_xor(send.y, bit, 64)};
          s[e] = keep + got;
        }
      }
      zd J = s[0];
      if (L4.a == L4.b) J = {J.x + 1.0, 0.0};
      const float2 fo = Fs[(row0 >> 2) * 16 + li];
      zd F = {(double)fo.x, (double)fo.y};
      const zd Lo = chol16(L4, J, ok);
      F = trsm16(L4, Lo, F);                      // L^{-1} G_own
      zd X = mm_hn(L4, F, F);                     // I + F^H F
      if (L4.a == L4.b) X = {X.x + 1.0, 0.0};
      UWr[i] = trsm16h(L4, Lo, F);                // J-^{-1} G_own
      const zd Lw = chol16(L4, X, ok);
      if (L4.a == L4.b) rsum += alpha[row0 + L4.a] * 2.0 * log(Lw.x);
      const zd Li = trsm16(L4, Lw, zd{(L4.a == L4.b) ? 1.0 : 0.0, 0.0});
      Er[i] = mm_hn(L4, Li, Li);                  // E = Lw^{-H} Lw^{-1}
      Lir[i] = Li;
    }
    if (!ok) atomicOr(&misc[0], AMMSE_INST_CHOLESKY);
    return rsum;
  };

  // D = alpha U W U^H and Y = alpha U W per block user, into LDS
  auto weights = [&](bool stage2) {
#pragma unroll
    for (int i = 0; i < S::GRB; ++i) {
      const int row0 = 16 * (wave + 4 * i) + 4 * lk;
      const zd T = mm_nn(L4, UWr[i], Er[i]);     // U
      const zd Ur = stage2 ? UWr[i] : T;
      zd Dv = mm_nh(L4, T, Ur);
      const zd Dt = L4.at(Dv, L4.b, L4.a);
      Dv = {0.5 * (Dv.x + Dt.x), 0.5 * (Dv.y - Dt.y)};   // exactly Hermitian
      const double al = alpha[row0 + L4.a];
      const int g4 = row0 >> 2;
      Ds[g4 * 16 + li] = c2((float)(al * Dv.x), (float)(al * Dv.y));
      Ys[g4 * 16 + li] = c2((float)(al * Ur.x), (float)(al * Ur.y));
      // D = C C^H: C = sqrt(alpha) U (stage I) or sqrt(alpha) UW Lw^{-H} (stage II)
      const zd Cv = stage2 ? mm_nh(L4, UWr[i], Lir[i]) : T;
      Cs[g4 * 16 + li] = scal(sqrt(al), Cv);
    }
    __syncthreads();
  };

  // lambda_max(A), A = H^H S D S H.  With D = C C^H (C block diagonal) and
  // Q = S H H^H S (formed once per solve), lambda_max(A) = lambda_max(K) for
  // the U N x U N matrix K = C^H Q C; plain Lanczos on K, two block barriers
  // per step.  Row r of K is handled by 4 lanes (16 columns each); the
  // Lanczos vectors stay in registers (every lane of a row holds its entry);
  // u = C x goes through LDS for the dense product with Q;
  //   beta^2 = ||y||^2 - alpha^2 - 2 beta_prev Re(p^H y) + beta_prev^2.
  auto lanczos = [&]() {
    static_assert(UN == 64, "16-row strips per wave");
    zd* uv = Lq;                                  // u = C x
    double* part = (double*)(Lq + UN);            // [4 waves][4] partial sums
    const int sub = lane & 3, idx = 16 * wave + (lane >> 2), gq = lane & ~15;
    const int g4 = idx >> 2, a4 = idx & 3;
    zd cr[4], cc[4];                              // row a4 of C, column a4 of C
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cr[k] = Cs[g4 * 16 + a4 * 4 + k];
      cc[k] = Cs[g4 * 16 + k * 4 + a4];
    }
    zd x = {1.0 + 0.5 * sin(0.731 * idx + 0.25), 0.3 * cos(1.37 * idx + 0.5)};
    const double nn = block_sum((sub == 0) ? nrm2(x) : 0.0, red);
    x = scal(1.0 / sqrt(nn), x);
    zd pp = {0.0, 0.0};
    auto put_u = [&]() {                          // u = C x for row idx
      zd u = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 4; ++k) u = u + cr[k] * shz(x, gq + 4 * k + sub);
      if (sub == 0) uv[idx] = u;
    };
    put_u();
    __syncthreads();
    const int m = min(p.lanczos_steps, UN);
    const double ltol = 1e-8;
    double beta_prev = 0.0, tmax = 0.0, theta = 0.0;
    for (int j = 0; j < m; ++j) {
      zd z = {0.0, 0.0};
#pragma unroll 4
      for (int k = 0; k < 16; ++k) {
        const int c = 16 * sub + ((k + idx) & 15);
        const float2 q = Qs[idx * S::QLD + c];
        z = z + zd{(double)q.x, (double)q.y} * uv[c];
      }
      z.x += __shfl_xor(z.x, 1, 64);
      z.y += __shfl_xor(z.y, 1, 64);
      z.x += __shfl_xor(z.x, 2, 64);
      z.y += __shfl_xor(z.y, 2, 64);
      zd y = {0.0, 0.0};                          // y = C^H z in the block user
#pragma unroll
      for (int k = 0; k < 4; ++k) y = y + cj(cc[k]) * shz(z, gq + 4 * k + sub);
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      if (sub == 0) {
        s0 = nrm2(y);
        s1 = x.x * y.x + x.y * y.y;
        s2 = pp.x * y.x + pp.y * y.y;
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      if (lane == 0) {
        part[wave * 4 + 0] = s0;
        part[wave * 4 + 1] = s1;
        part[wave * 4 + 2] = s2;
      }
      __syncthreads();
      double yy = 0.0, al = 0.0, py = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        yy += part[q * 4 + 0];
        al += part[q * 4 + 1];
        py += part[q * 4 + 2];
      }
      const double bb = sqrt(fmax(yy - al * al - 2.0 * beta_prev * py + beta_prev * beta_prev, 0.0));
      if (tid == 0) {
        la[j] = al;
        lb[j] = bb;
      }
      const int msz = j + 1;
      tmax = fmax(tmax, fabs(al) + bb);
      const bool breakdown = !(bb > 1e-12 * tmax);
      bool stop = breakdown;
      if (breakdown || (msz >= 12 && (msz % 4) == 0) || msz == m) {
        __syncthreads();
        if (wave == 0) {
          const double th = (tmax > 0.0) ? wave_tridiag_lmax(la, lb, msz, 1e-10) : 0.0;
          if (lane == 0) red[7] = th;
        }
        __syncthreads();
        const double th = red[7];
        stop = stop || fabs(th - theta) <= ltol * fabs(th);
        theta = th;
      }
      if (stop) break;
      const zd xn = scal(1.0 / bb, y - scal(al, x) - scal(beta_prev, pp));
      pp = x;
      x = xn;
      beta_prev = bb;
      put_u();
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
    const double rs = receivers();
    wsr_prev2 = wsr_prev;
    wsr_prev = block_sum(rs, red) * (1.0 / M_LN2);
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
    for (int i = 0; i < S::GRB; ++i) {
      const int row0 = 16 * (wave + 4 * i) + 4 * lk, g4 = row0 >> 2, u0 = row0 >> lgN;
      float2 dm[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) dm[r][k] = Ds[g4 * 16 + r * 4 + k];
#pragma unroll
      for (int j = 0; j < S::UDB; ++j) {
        float2 gh[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          gh[r] = c2((1.f + om) * Gp[i][j][r].x - om * Gq[i][j][r].x,
                     (1.f + om) * Gp[i][j][r].y - om * Gq[i][j][r].y);
        const int col = 16 * j + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float zx = 0.f, zy = 0.f;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            zx += dm[r][k].x * gh[k].x - dm[r][k].y * gh[k].y;
            zy += dm[r][k].x * gh[k].y + dm[r][k].y * gh[k].x;
          }
          const int u = (row0 + r) >> lgN, c = col - (u << lgd);
          if (c >= 0 && c < d) {
            const float2 y = Ys[g4 * 16 + r * 4 + ((u - u0) << lgN) + c];
            zx -= y.x;
            zy -= y.y;
          }
          const float is = (float)invsig[row0 + r];
          Bs[(row0 + r) * S::BLD + col] = c2(is * zx, is * zy);
        }
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
    const double rs = receivers();
    wsr_final = block_sum(rs, red) * (1.0 / M_LN2);
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
