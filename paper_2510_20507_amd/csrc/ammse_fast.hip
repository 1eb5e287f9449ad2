// LDS-resident A-MMMSE solve kernel on MFMA (FP32 storage), gfx950.
//
// For single-cell instances with M = 64 and U*N = U*d = 64, one workgroup of
// 256 threads (4 waves) owns one instance for the whole solve; HBM is touched
// only to read H, V0 and the per-user scalars (and H, V0 once more at the
// end) and to write the results.
//
// The precoder is carried implicitly, V^t = c_t V^0 + H^H S X^t, so that one
// product with Q = S H H^H S per iteration gives G^t = S H V^t (see the
// iteration below); V^T is rebuilt with one product by H^H at the end.
//
// Products: v_mfma_f32_16x16x4f32, a complex product being three real
// products (Re*Re, Im*Im, (Re + Im)*(Re + Im)) fed from interleaved complex
// LDS tiles.  Each wave owns whole 16-row strips of the outputs, so the
// iteration state stays in registers in the MFMA output layout:
//   G^{t-1}, G^{t-2}  (the extrapolated G follows by linearity)
//   X^{t-1}           (X^{t-2} and G^0 in LDS, per lane)
// each held divided by a per-matrix scale, so that the projection factor is
// applied to scalars rather than to every entry.
// A lane holds 4 consecutive rows of one column.  Four consecutive rows form
// a "block user": one user for N = 4, two for N = 2, four for N = 1; its
// N x N and d x d algebra is done as one block-diagonal 4 x 4 problem.
//
// Per-user algebra (Section IV equations for U and W, in the Woodbury form
// used throughout this library) runs lane-parallel in double: the 16 lanes
// of a DPP row hold the 16 entries of a 4 x 4 complex matrix and exchange
// them with DPP moves and swizzles.  The interference-plus-noise covariance
// of every user is reduced directly from the G registers.
//
// Per iteration t (Algorithm 3):
//   J- from registers (reduce-scatter over the 16 lanes of a row group);
//   Cholesky, U, W per block user; WSR(V^{t-1}) when a test needs it; stage
//   latch; adaptive step by Lanczos on K = C^H Q C (formed in LDS), after the
//   adaptive windows of stage II 1/Lhat (computed before the solve by
//   ammse_fast_bound_kernel);
//   Z' = D G^ - Y -> LDS;  P = Q Z' (MFMA);  in the epilogue
//   G~ = G^ - 2 gamma P, X~ = X^ - 2 gamma Z', the projection norm, and the
//   projection factor applied to G~, X~ and c.

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
  static constexpr int CST = 17;                                    // padded stride of C blocks (zd)
  static constexpr size_t oS = oC + sizeof(zd) * NG * CST;          // invsig, alpha per row
  static constexpr size_t oL = oS + sizeof(double) * 2 * UN;        // la, lb
  static constexpr size_t oR = oL + sizeof(double) * 2 * AMMSE_MAX_LANCZOS;
  static constexpr size_t oVq = oR + sizeof(double) * 16 + 16;     // X^{t-2}, per lane
  static constexpr size_t oP2 = oVq + sizeof(float2) * 256 * VRB * UDB * 4;  // Lanczos partials
  static constexpr size_t bytes = oP2 + sizeof(zd) * 4 * UN;
  static_assert(bytes <= 160 * 1024, "LDS of one CU");
  // During the step-size computation (between the receivers and the Z build)
  // K = C^H Q C and a float copy of the Lanczos vector alias the
  // product-operand area, the partial products alias C, and the tridiagonal
  // pairs alias la/lb.
  static_assert(sizeof(double) * 2 * AMMSE_MAX_LANCZOS >= 16 * 64, "tridiagonal pairs");
  static_assert(UN * UN + UN <= BROWS * BLD, "K and the Lanczos vector copy");
};

using Shape64 = Shape<4, 4, 4>;   // M = 64, U*N = 64, U*d = 64

__device__ __forceinline__ float2 c2(float x, float y) { return make_float2(x, y); }

// One wave: P[i][j] (three real accumulators) = op(A) B for the wave's row
// blocks i (global row block wave + 4 i) and all column blocks j.
// op(A)[r][k] = A[r*lda + k], or conj(A[k*lda + r]) with CONJA; B[k][j] is
// B[k*ldb + j], or conj(B[j*ldb + k]) with CONJBT.
// Three real products per complex product (Gauss): P0 = Ar Br, P1 = Ai Bi,
// P2 = (Ar + Ai)(Br + Bi); Re = P0 - P1, Im = P2 - P0 - P1 (see cplx_at).
template <int NRB, int NCB, int K, bool CONJA, bool CONJBT = false>
__device__ __forceinline__ void wave_cgemm(const float2* __restrict__ A, int lda,
                                           const float2* __restrict__ B, int ldb,
                                           int wave, floatx4 (&P)[NRB][NCB][3]) {
  static_assert(K % 8 == 0, "two k-steps per loop trip");
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < NRB; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) P[i][j][q] = floatx4{0.f, 0.f, 0.f, 0.f};
  auto load = [&](int k0, float2 (&a)[NRB], float2 (&b)[NCB]) {
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
  };
  auto step = [&](const float2 (&a)[NRB], const float2 (&b)[NCB]) {
    float as[NRB], bs[NCB];
#pragma unroll
    for (int i = 0; i < NRB; ++i) as[i] = a[i].x + a[i].y;
#pragma unroll
    for (int j = 0; j < NCB; ++j) bs[j] = b[j].x + b[j].y;
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
        P[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[i], bs[j], P[i][j][2], 0, 0, 0);
  };
  // operands of the next k-step are fetched before the current one's MFMAs
  float2 a0[NRB], b0[NCB], a1[NRB], b1[NCB];
  load(0, a0, b0);
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 8) {
    load(k0 + 4, a1, b1);
    step(a0, b0);
    if (k0 + 8 < K) load(k0 + 8, a0, b0);
    step(a1, b1);
  }
}

// Complex entry r of an accumulator triple from wave_cgemm.
__device__ __forceinline__ float2 cplx_at(const floatx4 (&P)[3], int r) {
  return c2(P[0][r] - P[1][r], P[2][r] - P[0][r] - P[1][r]);
}

// ---------------------------------------------------------------------------
// Wave-level helpers (64 lanes, no LDS traffic)
// ---------------------------------------------------------------------------

// Value of lane l (l uniform over the wave).
__device__ __forceinline__ double rlane(double v, int l) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ zd rlane(zd v, int l) { return {rlane(v.x, l), rlane(v.y, l)}; }

// Sum over the 64 lanes; every lane receives the same value (the row sums
// of lanes 0, 16, 32, 48 added in a fixed order).
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp64<0xB1>(v);     // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp64<0x4E>(v);     // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp64<0x124>(v);    // row_ror 4
  v += dpp64<0x128>(v);    // row_ror 8
  return (rlane(v, 0) + rlane(v, 16)) + (rlane(v, 32) + rlane(v, 48));
}

// Sum over the 256-thread block (four waves); every thread receives the
// same value.  red: four doubles of LDS, which the caller must not hand to
// another call before every wave has passed a further barrier (one barrier
// per call).
__device__ __forceinline__ double block_sum4(double v, double* red) {
  v = wave_sum_dpp(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Position of entry (row, col) of G inside the 4 x 4 block of its row group
// when col is one of the row's own streams (block-diagonal packing of the
// users' N x d own blocks, N = d), else -1.
__device__ __forceinline__ int own_entry(int row, int col, int lgN, int lgd) {
  const int u = row >> lgN, c = col - (u << lgd);
  const int u0 = (row & ~3) >> lgN;
  return (c >= 0 && c < (1 << lgd)) ? (row & 3) * 4 + ((u - u0) << lgN) + c : -1;
}

// Value of lane (lane ^ BIT) within the 16-lane row, BIT in {1, 2, 4, 8}.
template <int BIT>
__device__ __forceinline__ float xor_lane(float v) {
  const int u = __float_as_int(v);
  int r;
  if (BIT == 1) r = __builtin_amdgcn_mov_dpp(u, 0xB1, 0xF, 0xF, false);        // quad_perm [1,0,3,2]
  else if (BIT == 2) r = __builtin_amdgcn_mov_dpp(u, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  else if (BIT == 4) r = __builtin_amdgcn_ds_swizzle(u, 0x1F | (4 << 10));     // swizzle xor 4
  else r = __builtin_amdgcn_mov_dpp(u, 0x128, 0xF, 0xF, false);                // row_ror 8
  return __int_as_float(r);
}

// One level of the 16-lane reduce-scatter of 16 complex partial sums: the
// lane keeps one half of s[0 .. 2 BIT) and adds the partner's copy of it.
template <int BIT>
__device__ __forceinline__ void rs_level(float2 (&s)[16], int li) {
  const bool hi = (li & BIT) != 0;
#pragma unroll
  for (int e = 0; e < BIT; ++e) {
    const float2 keep = hi ? s[e + BIT] : s[e];
    const float2 send = hi ? s[e] : s[e + BIT];
    s[e] = c2(keep.x + xor_lane<BIT>(send.x), keep.y + xor_lane<BIT>(send.y));
  }
}

// The kernel body for N = d = 2^LGN (compile-time, so that the user and
// own-stream index arithmetic folds).
template <class S, int LGN>
__device__ __forceinline__ void fast_body(const ammse_kparams_t& p) {
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
  double* la = (double*)(smem + S::oL);         // tridiagonal pairs of the step size
  double* red = (double*)(smem + S::oR);
  // red: three slots of four partial sums ([0], [4], [8]; a slot is reused
  // only across further barriers) and two Lanczos values ([12], [13])
  int* misc = (int*)(red + 16);                // [0] fail flag, [1], [2] Lanczos stop flags

  constexpr int M = S::M, UN = S::UN, UD = S::UD;
  const ammse_desc_t Dd = p.desc[blockIdx.x];
  constexpr int lgN = LGN, lgd = LGN, N = 1 << LGN, d = 1 << LGN;   // N = d in {1, 2, 4}
  const int b = Dd.b;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const Lane4 L4{lane & ~15, li >> 2, li & 3};

  const float2* Hg = (const float2*)p.H + Dd.h_off;
  float2* Vg = (float2*)p.V + Dd.v_off;
  const double Pc = p.wsr_only ? 0.0 : p.P[Dd.bs_off];
  const double iPc = (Pc > 0.0) ? 1.0 / Pc : 0.0;

  for (int r = tid; r < UN; r += 256) {
    invsig[r] = 1.0 / sqrt(p.sigma2[Dd.user_off + r / N]);
    alpha[r] = p.alpha[Dd.user_off + r / N];
  }
  for (int e = tid; e < S::NG * 16; e += 256) Fs[e] = c2(0.f, 0.f);
  if (tid == 0) misc[0] = 0;
  for (int e = tid; e < UN * M; e += 256) Hs[(e / M) * S::HLD + (e % M)] = Hg[e];
  for (int e = tid; e < M * UD; e += 256) Bs[(e / UD) * S::BLD + (e % UD)] = Vg[e];
  __syncthreads();

  // The precoder is carried implicitly: V^t = c_t V^0 + H^H S X^t with
  // X^t of the shape of G (U N x U d), so that G^t = S H V^t = c_t G^0 + Q X^t
  // follows from G^{t-1}, G^{t-2} and one product with Q per iteration
  // (G^t = s (G^ - 2 gamma Q Z'), X^t = s (X^ - 2 gamma Z'), Z' = D G^ - Y, s
  // the projection factor); V^T is rebuilt with one product by H^H at the end.
  // Register state: element [i][j][r] is row 16 (wave + 4 i) + 4 lk + r,
  // column 16 j + li.  X^{t-2} and G^0 live in LDS per lane (entry e of this
  // lane at [e * 256 + tid]); G^0 reuses the area of H, which the loop does
  // not read.
  float2* XqS = (float2*)(smem + S::oVq);
  float2* G0S = Hs;
  static_assert(sizeof(float2) * 256 * S::GRB * S::UDB * 4 <= sizeof(float2) * UN * S::HLD,
                "G0 area");
  float2 Xp[S::GRB][S::UDB][4];
  float2 Gp[S::GRB][S::UDB][4], Gq[S::GRB][S::UDB][4];

  // Q = S H H^H S for the step-size operator, once per solve
  {
    floatx4 P[S::GRB][S::UNB][3];
    wave_cgemm<S::GRB, S::UNB, M, false, true>(Hs, S::HLD, Hs, S::HLD, wave, P);
#pragma unroll
    for (int i = 0; i < S::GRB; ++i)
#pragma unroll
      for (int j = 0; j < S::UNB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
          const float s = (float)(invsig[row] * invsig[col]);
          const float2 v = cplx_at(P[i][j], r);
          Qs[row * S::QLD + col] = c2(s * v.x, s * v.y);
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

  // The projection factor is applied lazily: the registers Gp and Xp and the
  // copies Gq and X^{t-2} hold their matrices divided by these scales.
  float sgp = 1.f, sgq = 1.f, sxp = 1.f, sxq = 1.f;

  // G = S H V (V in Bs) into Gp (previous Gp to Gq); own blocks into Fs
  auto product_G = [&]() {
    floatx4 P[S::GRB][S::UDB][3];
    wave_cgemm<S::GRB, S::UDB, M, false>(Hs, S::HLD, Bs, S::BLD, wave, P);
#pragma unroll
    for (int i = 0; i < S::GRB; ++i)
#pragma unroll
      for (int j = 0; j < S::UDB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
          const float s = (float)invsig[row];
          const float2 v = cplx_at(P[i][j], r);
          const float2 g = c2(s * v.x, s * v.y);
          Gq[i][j][r] = Gp[i][j][r];
          Gp[i][j][r] = g;
          const int u = row >> lgN, c = col - (u << lgd);
          if (c >= 0 && c < d) {
            const int g4 = row >> 2, u0 = (g4 * 4) >> lgN;
            Fs[g4 * 16 + r * 4 + ((u - u0) << lgN) + c] = g;
          }
        }
    sgq = sgp;
    sgp = 1.f;
  };

  // Per block user (i = row block of this wave, group lk): J-, Cholesky,
  // rate, UW = J-^{-1} G_own and E = (I + G_own^H J-^{-1} G_own)^{-1}.
  // Returns the weighted rate contribution of this lane (diagonal lanes).
  zd UWr[S::GRB], Lir[S::GRB];
  auto receivers = [&](bool with_rate) {
    double rsum = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < S::GRB; ++i) {
      const int row0 = 16 * (wave + 4 * i) + 4 * lk;
      // partial J over this lane's columns in float (Hermitian: the upper
      // triangle is accumulated, the lower one mirrored)
      float2 s[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) s[e] = c2(0.f, 0.f);
      // own columns (block jo, N = d) are left out by zeroing them; rows a and
      // c pair only within one user (row0 is a multiple of 4)
      const int jo = wave + 4 * i;
      bool ownr[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) ownr[r] = own_entry(row0 + r, 16 * jo + li, lgN, lgd) >= 0;
#pragma unroll
      for (int j = 0; j < S::UDB; ++j) {
        float2 gz[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) gz[r] = (j == jo && ownr[r]) ? c2(0.f, 0.f) : Gp[i][j][r];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = a; c < 4; ++c) {
            const bool same = (a >> lgN) == (c >> lgN);
            const float2 ga = gz[a], gc = gz[c];
            const float2 sn = c2(fmaf(ga.y, gc.y, fmaf(ga.x, gc.x, s[a * 4 + c].x)),
                                 fmaf(-ga.x, gc.y, fmaf(ga.y, gc.x, s[a * 4 + c].y)));
            if (same) s[a * 4 + c] = sn;
          }
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < a; ++c) s[a * 4 + c] = c2(s[c * 4 + a].x, -s[c * 4 + a].y);
      // reduce-scatter over the 16 lanes: lane li ends with entry li
      // (partner lane li ^ bit: DPP row_ror 8, swizzle xor 4, DPP quad_perm)
      rs_level<8>(s, li);
      rs_level<4>(s, li);
      rs_level<2>(s, li);
      rs_level<1>(s, li);
      const double sg2 = (double)sgp * (double)sgp;      // G = sgp Gp
      zd J = {sg2 * (double)s[0].x, sg2 * (double)s[0].y};
      if (L4.a == L4.b) J = {J.x + 1.0, 0.0};
      const float2 fo = Fs[(row0 >> 2) * 16 + li];
      zd F = {(double)fo.x, (double)fo.y};
      double io[4], iw[4];                        // reciprocal diagonals of the factors
      const zd Lo = chol16(L4, J, ok, io);
      F = trsm16(L4, Lo, io, F);                  // L^{-1} G_own
      zd X = mm_hn(L4, F, F);                     // I + F^H F
      if (L4.a == L4.b) X = {X.x + 1.0, 0.0};
      UWr[i] = trsm16h(L4, Lo, io, F);            // J-^{-1} G_own
      const zd Lw = chol16(L4, X, ok, iw);
      // rate term 2 log Lw_aa in float (the WSR enters only the stage and stop
      // tests and the reported value, all at FP32 accuracy here)
      if (with_rate && L4.a == L4.b)
        rsum += alpha[row0 + L4.a] * (double)(2.0f * __logf((float)Lw.x));
      const zd Li = trsm16(L4, Lw, iw, zd{(L4.a == L4.b) ? 1.0 : 0.0, 0.0});
      Lir[i] = Li;                                // E = Li^H Li (formed where needed)
    }
    if (!ok) atomicOr(&misc[0], AMMSE_INST_CHOLESKY);
    return rsum;
  };

  // D = alpha U W U^H and Y = alpha U W per block user, and C with D = C C^H,
  // into LDS
  auto weights = [&](bool stage2, bool for_step) {
#pragma unroll
    for (int i = 0; i < S::GRB; ++i) {
      const int row0 = 16 * (wave + 4 * i) + 4 * lk;
      // stage II (W = E^{-1}): U W = UW, D = alpha UW E UW^H = alpha C C^H with
      // C = UW Li^H; stage I (W = I): U = UW E, D = alpha U U^H, C = U
      zd Ur, Cv;
      if (stage2) {
        Cv = mm_nh(L4, UWr[i], Lir[i]);
        Ur = UWr[i];
      } else {
        Cv = mm_nn(L4, UWr[i], mm_hn(L4, Lir[i], Lir[i]));
        Ur = Cv;
      }
      zd Dv = mm_nh(L4, Cv, Cv);
      const zd Dt = L4.at(Dv, L4.b, L4.a);
      Dv = {0.5 * (Dv.x + Dt.x), 0.5 * (Dv.y - Dt.y)};   // exactly Hermitian
      const double al = alpha[row0 + L4.a];
      const int g4 = row0 >> 2;
      Ds[g4 * 16 + li] = c2((float)(al * Dv.x), (float)(al * Dv.y));
      Ys[g4 * 16 + li] = c2((float)(al * Ur.x), (float)(al * Ur.y));
      Cs[g4 * S::CST + li] = scal(sqrt(al), Cv);
    }
    // D and Y are read back by the same wave; C by all waves (step size only)
    if (for_step) __syncthreads();
  };

  // lambda_max(A), A = H^H S D S H.  With D = C C^H (C block diagonal) and
  // Q = S H H^H S (formed once per solve), lambda_max(A) = lambda_max(K) for
  // the U N x U N matrix K = C^H Q C.  K is formed in LDS (over the product
  // operand, free here; stored transposed so that lane r reads row r of K
  // from consecutive addresses), then plain Lanczos on K: every wave holds
  // the whole Lanczos vectors (lane r: entry r), multiplies its 16 columns of
  // K, and the four partial products meet in LDS (over C, no longer needed);
  // the recurrence scalars and the tridiagonal eigenvalue are computed by
  // every wave alike, the stop decision of wave 0 is shared through LDS.
  //   beta^2 = ||y||^2 - alpha^2 - 2 beta_prev Re(p^H y) + beta_prev^2.
  auto lanczos = [&]() {
    static_assert(UN == 64 && S::NG == 16, "one Lanczos entry per lane");
    static_assert(sizeof(float2) * UN * UN <= sizeof(float2) * S::BROWS * S::BLD, "K area");
    static_assert(sizeof(zd) * 4 * UN <= sizeof(zd) * S::NG * S::CST, "partial area");
    float2* Kt = Bs;                              // Kt[c * UN + r] = K[r][c]
    zd* part0 = (zd*)Cs;                          // [4 waves][UN], even steps
    zd* part1 = (zd*)(smem + S::oP2);             // odd steps
    float2* xs = Bs + UN * UN;                    // float copy of x; each wave writes and
                                                  // reads back only its own 16 columns
    double2* tp = (double2*)la;                   // tridiagonal pairs (wave 0)
    {
      // block (g, h): K_gh = C_g^H Q_gh C_h, one thread per block; Q_gh is
      // read as Q_hg^H (Q is exactly Hermitian) for conflict-light LDS reads
      const int g = tid & 15, h = tid >> 4;
      float2 q[4][4];
      float2 cg[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float2 qt = Qs[(4 * h + k) * S::QLD + 4 * g + a];
          q[a][k] = c2(qt.x, -qt.y);
          const zd c = Cs[g * S::CST + a * 4 + k];
          cg[a][k] = c2((float)c.x, (float)c.y);
        }
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        zd ch[4], w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) ch[k] = Cs[h * S::CST + k * 4 + bb];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          w[a] = {0.0, 0.0};
#pragma unroll
          for (int k = 0; k < 4; ++k) w[a] = w[a] + zd{(double)q[a][k].x, (double)q[a][k].y} * ch[k];
        }
        float4 kv2[2];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          zd kv = {0.0, 0.0};
#pragma unroll
          for (int k = 0; k < 4; ++k)
            kv = kv + cj(zd{(double)cg[k][a].x, (double)cg[k][a].y}) * w[k];
          if (a & 1) {
            kv2[a >> 1].z = (float)kv.x;
            kv2[a >> 1].w = (float)kv.y;
          } else {
            kv2[a >> 1].x = (float)kv.x;
            kv2[a >> 1].y = (float)kv.y;
          }
        }
        float4* dst = (float4*)(Kt + (4 * h + bb) * UN + 4 * g);
        dst[0] = kv2[0];
        dst[1] = kv2[1];
      }
    }
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    zd x = {1.0 + 0.5 * sin(0.731 * lane + 0.25), 0.3 * cos(1.37 * lane + 0.5)};
    x = scal(1.0 / sqrt(wave_sum_dpp(nrm2(x))), x);
    zd pp = {0.0, 0.0};
    double ta = 0.0, tb = 0.0;                    // T entries, lane j holds entry j
    const int m = max(1, min(p.lanczos_steps, UN));
    const double ltol = 1e-8;
    double beta_prev = 0.0, tmax = 0.0, theta = 0.0;
    bool stop = false;
    int jlast = 0;
    for (int j = 0;; ++j) {
      // partial product over this wave's 16 columns in float (K is stored in
      // float), two accumulator pairs, combined in double
      float2 ya = c2(0.f, 0.f), yb = c2(0.f, 0.f);
      {
        if ((lane >> 4) == wv) xs[lane] = c2((float)x.x, (float)x.y);   // read back broadcast
        float2 kv[16], xv[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          kv[k] = Kt[(16 * wv + k) * UN + lane];
          xv[k] = xs[16 * wv + k];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          float2& acc = (k & 1) ? yb : ya;
          acc.x = fmaf(-kv[k].y, xv[k].y, fmaf(kv[k].x, xv[k].x, acc.x));
          acc.y = fmaf(kv[k].y, xv[k].x, fmaf(kv[k].x, xv[k].y, acc.y));
        }
      }
      const zd yw = {(double)ya.x + (double)yb.x, (double)ya.y + (double)yb.y};
      // one barrier per step: partials, the stop flag and theta alternate
      // between two slots, so a slot is rewritten only after every wave has
      // passed the barrier that follows its last read
      zd* part = (j & 1) ? part1 : part0;
      if (tid == 0) {
        misc[1 + (j & 1)] = stop ? 1 : 0;
        red[12 + (j & 1)] = theta;
      }
      part[wave * UN + lane] = yw;
      __syncthreads();
      if (misc[1 + (j & 1)]) {
        jlast = j;
        break;
      }
      const zd y = (part[lane] + part[UN + lane]) + (part[2 * UN + lane] + part[3 * UN + lane]);
      double al = x.x * y.x + x.y * y.y, yy = nrm2(y), py = pp.x * y.x + pp.y * y.y;
      wave_sum3_dpp(al, yy, py);
      const double b2 = fmax(yy - al * al - 2.0 * beta_prev * py + beta_prev * beta_prev, 0.0);
      const double ib = rsqrt_nr(fmin(fmax(b2, 1e-300), __DBL_MAX__));   // 1 / beta
      const double bb = b2 * ib;
      if (lane == j) {
        ta = al;
        tb = bb;
      }
      const int msz = j + 1;
      tmax = fmax(tmax, fabs(al) + bb);
      const bool breakdown = !(bb > 1e-12 * tmax);
      // only wave 0's decision is used (shared through LDS above)
      if (wave == 0 && (breakdown || (msz >= 14 && (msz % 2) == 0) || msz == m)) {
        bool conv = false;
        theta = (tmax > 0.0) ? wave_tridiag_lmax(ta, tb, msz, tmax, theta, ltol, tp, &conv) : 0.0;
        stop = breakdown || conv || msz == m;
      }
      if (!stop) {
        const zd xn = scal(ib, y - scal(al, x) - scal(beta_prev, pp));
        pp = x;
        x = xn;
        beta_prev = bb;
      }
    }
    return red[12 + (jlast & 1)];
  };

  // G^0 = S H V^0 (V^0 in Bs) and nu = ||V^0||^2
  product_G();
  double nu = 0.0;
#pragma unroll
  for (int i = 0; i < S::VRB; ++i)
#pragma unroll
    for (int j = 0; j < S::UDB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float2 v = Bs[(16 * (wave + 4 * i) + 4 * lk + r) * S::BLD + 16 * j + li];
        nu += (double)v.x * v.x + (double)v.y * v.y;
      }
  nu = block_sum4(nu, red);                    // its barrier also ends the reads of H
#pragma unroll
  for (int i = 0; i < S::GRB; ++i)
#pragma unroll
    for (int j = 0; j < S::UDB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = ((i * S::UDB + j) * 4 + r) * 256 + tid;
        Gq[i][j][r] = Gp[i][j][r];
        G0S[e] = Gp[i][j][r];
        Xp[i][j][r] = c2(0.f, 0.f);
        XqS[e] = c2(0.f, 0.f);
      }
  double c1 = 1.0, c2s = 1.0;                  // c_{t-1}, c_{t-2}

  const int T = p.wsr_only ? 0 : p.max_iters;
  int fsw = p.force_switch_iter;
  if (p.force_switch && p.force_switch[b] > 0) fsw = p.force_switch[b];
  bool stage2 = (fsw >= 1) ? (fsw <= 1) : (p.warm_start == 0);
  int switch_iter = stage2 ? 1 : -1;
  bool prev_step_stage2 = false;
  double wsr_prev = 0.0, wsr_prev2 = 0.0, gamma = 0.0;
  // 1 / Lhat, the stage-II step of the bound rule, from ammse_fast_bound_kernel
  // (launched before this kernel on the same stream)
  const double gbound = p.gbound ? p.gbound[blockIdx.x] : 0.0;
  int iters_run = 0, status = 0;

  for (int t = 1; t <= T; ++t) {
    // WSR(V^{t-1}) is needed for the stage test (stage I), the eps2 stop and
    // the trace; otherwise the rate terms and their block reduction are skipped
    // (a factorisation failure is then caught after the next barrier)
    const bool need_wsr = !stage2 || p.eps2 > 0 || p.trace != nullptr;
    const double rs = receivers(need_wsr);
    wsr_prev2 = wsr_prev;
    if (need_wsr) {
      wsr_prev = block_sum4(rs, red + 4) * (1.0 / M_LN2);
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
    } else {
      wsr_prev = NAN;
    }
    if (!stage2) {
      const bool trig = (fsw >= 1) ? (t >= fsw)
                                   : (t >= 2 && rel_change(wsr_prev, wsr_prev2) <= p.eps1);
      if (trig) {
        stage2 = true;
        switch_iter = t;
      }
    }
    const bool adaptive = t <= p.T_c || (p.rearm && switch_iter >= 1 && t >= switch_iter &&
                                         t < switch_iter + p.T_c);
    const bool use_bound = stage2 && !adaptive && !(p.gamma_c > 0.0) &&
                           p.step_rule == AMMSE_STEP_BOUND;
    weights(stage2, adaptive);
    if (adaptive) {
      const double lm = lanczos();
      gamma = (lm > 0.0) ? 1.0 / (2.0 * lm) : 0.0;
    } else if (p.gamma_c > 0.0) {
      gamma = p.gamma_c;
    } else if (use_bound) {
      gamma = gbound;
    }

    // Z' = D G^ - Y from the registers, into Bs (the gradient is 2 H^H S Z')
    const float om = p.extrapolate ? (float)fmax((t - 2.0) / (t + 1.0), 0.0) : 0.f;
    const float cgp = (1.f + om) * sgp, cgq = om * sgq;
#pragma unroll
    for (int i = 0; i < S::GRB; ++i) {
      const int row0 = 16 * (wave + 4 * i) + 4 * lk, g4 = row0 >> 2;
      float2 dm[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) dm[r][k] = Ds[g4 * 16 + r * 4 + k];
      // Y is nonzero only on the own entries, which lie in column block jo
      // (N = d here); the lane's four candidates are loaded up front
      const int jo = wave + 4 * i;
      bool own[4];
      float2 yo[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = own_entry(row0 + r, 16 * jo + li, lgN, lgd);
        own[r] = e >= 0;
        yo[r] = Ys[g4 * 16 + max(e, 0)];
      }
#pragma unroll
      for (int j = 0; j < S::UDB; ++j) {
        // G^ = (1 + w) G^{t-1} - w G^{t-2}, kept over G^{t-2} (no longer needed)
        float2 gh[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          gh[r] = c2(cgp * Gp[i][j][r].x - cgq * Gq[i][j][r].x,
                     cgp * Gp[i][j][r].y - cgq * Gq[i][j][r].y);
          Gq[i][j][r] = gh[r];
        }
        const int col = 16 * j + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float zx = 0.f, zy = 0.f;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            zx = fmaf(-dm[r][k].y, gh[k].y, fmaf(dm[r][k].x, gh[k].x, zx));
            zy = fmaf(dm[r][k].y, gh[k].x, fmaf(dm[r][k].x, gh[k].y, zy));
          }
          const bool sub = (j == jo) && own[r];
          zx = sub ? zx - yo[r].x : zx;
          zy = sub ? zy - yo[r].y : zy;
          Bs[(row0 + r) * S::BLD + col] = c2(zx, zy);
        }
      }
    }
    __syncthreads();
    if (!need_wsr && misc[0]) {   // factorisation failure flagged by this iteration's receivers
      status |= misc[0];
      break;
    }

    // G~ = G^ - 2 gamma Q Z' (G^ in Gq), X~ = X^ - 2 gamma Z', and the projection:
    // ||V~||^2 = c^2 nu + c Re<G^0, X~> + Re<X~, G~>  (c = c^, exact algebra
    // of V~ = c V^0 + H^H S X~ with G~ = c G^0 + Q X~)
    {
      floatx4 P[S::GRB][S::UDB][3];
      wave_cgemm<S::GRB, S::UDB, UN, false>(Qs, S::QLD, Bs, S::BLD, wave, P);
      const float g2 = (float)(2.0 * gamma);
      const double ch = (1.0 + om) * c1 - om * c2s;
      const float chf = (float)ch;
      const float cxp = (1.f + om) * sxp, cxq = om * sxq;
      float acc = 0.f;
#pragma unroll
      for (int i = 0; i < S::GRB; ++i)
#pragma unroll
        for (int j = 0; j < S::UDB; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = ((i * S::UDB + j) * 4 + r) * 256 + tid;
            const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
            const float2 pq = cplx_at(P[i][j], r);
            const float2 gp = Gp[i][j][r], gh = Gq[i][j][r];
            const float2 gt = c2(fmaf(-g2, pq.x, gh.x), fmaf(-g2, pq.y, gh.y));
            const float2 xp = Xp[i][j][r], xq = XqS[e], z = Bs[row * S::BLD + col];
            const float2 xt = c2(cxp * xp.x - cxq * xq.x - g2 * z.x,
                                 cxp * xp.y - cxq * xq.y - g2 * z.y);
            const float2 g0 = G0S[e];
            acc = fmaf(xt.x, fmaf(chf, g0.x, gt.x), acc);   // Re<X~, c G^0 + G~>
            acc = fmaf(xt.y, fmaf(chf, g0.y, gt.y), acc);
            XqS[e] = xp;             // X^{t-1} becomes X^{t-2} (scale sxp)
            Xp[i][j][r] = xt;        // X~ (the projection factor becomes its scale)
            Gq[i][j][r] = gp;        // G^{t-1} becomes G^{t-2} (scale sgp)
            Gp[i][j][r] = gt;        // G~
          }
      const double pw = ch * ch * nu + block_sum4((double)acc, red + 8);
      // sqrt(Pc / pw) = 1 / sqrt(pw / Pc) by the refined reciprocal square root
      const double scd = (pw > Pc) ? ((Pc > 0.0) ? rsqrt_nr(fmin(pw * iPc, __DBL_MAX__)) : 0.0)
                                   : 1.0;
      const float sc = (float)scd;
      c2s = c1;
      c1 = scd * ch;
      sxq = sxp;
      sxp = sc;
      sgq = sgp;
      sgp = sc;
#pragma unroll
      for (int i = 0; i < S::GRB; ++i) {
        // own entries (column block jo, N = d), scaled, into Fs for the receivers
        const int row0 = 16 * (wave + 4 * i) + 4 * lk, jo = wave + 4 * i;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float2 g = Gp[i][0][r];
#pragma unroll
          for (int j = 1; j < S::UDB; ++j) g = (j == jo) ? Gp[i][j][r] : g;
          const int e = own_entry(row0 + r, 16 * jo + li, lgN, lgd);
          if (e >= 0) Fs[(row0 >> 2) * 16 + e] = c2(sc * g.x, sc * g.y);
        }
      }
    }
    prev_step_stage2 = stage2;
    iters_run = t;
  }

  // V = c V^0 + H^H S X (the precoder of the last state), projected onto the
  // power ball exactly, written out; then its WSR from G = S H V.
  double pw = 0.0;
  if (!p.wsr_only) {
    __syncthreads();                           // loop reads of Bs, G^0 and X done
    for (int e = tid; e < UN * M; e += 256) Hs[(e / M) * S::HLD + (e % M)] = Hg[e];
#pragma unroll
    for (int i = 0; i < S::GRB; ++i)
#pragma unroll
      for (int j = 0; j < S::UDB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
          const float s = (float)invsig[row] * sxp;   // X = sxp Xp
          Bs[row * S::BLD + col] = c2(s * Xp[i][j][r].x, s * Xp[i][j][r].y);
        }
    __syncthreads();
    floatx4 P[S::VRB][S::UDB][3];
    wave_cgemm<S::VRB, S::UDB, UN, true>(Hs, S::HLD, Bs, S::BLD, wave, P);
    const float cf = (float)c1;
    float2 vf[S::VRB][S::UDB][4];
#pragma unroll
    for (int i = 0; i < S::VRB; ++i)
#pragma unroll
      for (int j = 0; j < S::UDB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
          const float2 v0 = Vg[row * UD + col];
          const float2 hx = cplx_at(P[i][j], r);
          const float2 v = c2(cf * v0.x + hx.x, cf * v0.y + hx.y);
          vf[i][j][r] = v;
          pw += (double)v.x * v.x + (double)v.y * v.y;
        }
    pw = block_sum4(pw, red);                  // its barrier also ends the reads of Bs
    const float sc = (pw > Pc) ? (float)sqrt(Pc / pw) : 1.f;
    if (pw > Pc) pw = Pc;
#pragma unroll
    for (int i = 0; i < S::VRB; ++i)
#pragma unroll
      for (int j = 0; j < S::UDB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (wave + 4 * i) + 4 * lk + r, col = 16 * j + li;
          const float2 v = c2(sc * vf[i][j][r].x, sc * vf[i][j][r].y);
          Bs[row * S::BLD + col] = v;
          Vg[row * UD + col] = v;
        }
    __syncthreads();
    product_G();
  } else {
    pw = nu;
  }
  double wsr_final;
  if (!status) {
    const double rs = receivers(true);
    wsr_final = block_sum4(rs, red + 4) * (1.0 / M_LN2);
    if (misc[0]) status |= misc[0];
    if (!isfinite(wsr_final)) status |= AMMSE_INST_NONFINITE;
    if (p.trace && tid == 0 && iters_run == T) p.trace[(long)b * p.trace_len + T] = wsr_final;
  } else {
    wsr_final = wsr_prev;
  }
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

// Stage-II step of the bound rule for the instances of the LDS-resident
// kernel: gb[k] = 1 / (2 lambda_max(H^H S_a^2 H)) for the instance at launch
// position k, S_a = diag(sqrt(alpha_u) / sigma_u) over the rows of H
// (M = U N = 64).  One wave per instance, H staged in LDS; plain three-term
// Lanczos on the antenna-side operator x -> H^H S_a^2 H x with lane i holding
// entry i of the vectors (double), start vector, step limit and stopping rule
// as the step-size Lanczos of the solve kernels (relative 1e-8 between checks
// from step 12 on every second step).  The operator depends only on the
// channel, so the value is computed once per solve, at an occupancy of
// several instances per CU, instead of serially inside the solve.
__global__ __launch_bounds__(64) void ammse_fast_bound_kernel(ammse_kparams_t p, double* gb) {
  constexpr int M = Shape64::M, UN = Shape64::UN, LD = M + 1;
  __shared__ float2 Hs[UN * LD];
  __shared__ float2 xs[M];        // broadcast of the vector being multiplied
  __shared__ double2 tp[64];      // tridiagonal pairs of the Ritz-value search
  const ammse_desc_t D = p.desc[blockIdx.x];
  const int lane = threadIdx.x;
  const float2* Hg = (const float2*)p.H + D.h_off;
  for (int e = lane; e < UN * M; e += 64) Hs[(e / M) * LD + (e % M)] = Hg[e];
  const int u = lane / D.N;
  const double sa = sqrt(p.alpha[D.user_off + u] / p.sigma2[D.user_off + u]);
  const double s2 = sa * sa;
  zd x = {1.0 + 0.5 * sin(0.731 * lane + 0.25), 0.3 * cos(1.37 * lane + 0.5)};
  x = scal(1.0 / sqrt(wave_sum(nrm2(x))), x);
  zd pp = {0.0, 0.0};
  const int m = max(1, min(p.lanczos_steps, M));
  const double ltol = 1e-8;
  double ta = 0.0, tb = 0.0, beta_prev = 0.0, tmax = 0.0, theta = 0.0;
  for (int j = 0;; ++j) {
    // y_r = s_r^2 (H x)_r  (lane r), then w_i = (H^H y)_i  (lane i); the
    // products in float (H is stored in float) on two accumulator pairs,
    // combined in double
    __syncthreads();
    xs[lane] = make_float2((float)x.x, (float)x.y);
    __syncthreads();
    float2 ya = make_float2(0.f, 0.f), yb = make_float2(0.f, 0.f);
#pragma unroll 16
    for (int k = 0; k < M; k += 2) {
      const float2 h0 = Hs[lane * LD + k], h1 = Hs[lane * LD + k + 1];
      const float2 x0 = xs[k], x1 = xs[k + 1];
      ya.x = fmaf(-h0.y, x0.y, fmaf(h0.x, x0.x, ya.x));
      ya.y = fmaf(h0.y, x0.x, fmaf(h0.x, x0.y, ya.y));
      yb.x = fmaf(-h1.y, x1.y, fmaf(h1.x, x1.x, yb.x));
      yb.y = fmaf(h1.y, x1.x, fmaf(h1.x, x1.y, yb.y));
    }
    const zd y = scal(s2, zd{(double)ya.x + (double)yb.x, (double)ya.y + (double)yb.y});
    __syncthreads();
    xs[lane] = make_float2((float)y.x, (float)y.y);
    __syncthreads();
    float2 wa = make_float2(0.f, 0.f), wb = make_float2(0.f, 0.f);
#pragma unroll 16
    for (int r = 0; r < UN; r += 2) {   // conj(H[r][i]) y_r
      const float2 h0 = Hs[r * LD + lane], h1 = Hs[(r + 1) * LD + lane];
      const float2 y0 = xs[r], y1 = xs[r + 1];
      wa.x = fmaf(h0.y, y0.y, fmaf(h0.x, y0.x, wa.x));
      wa.y = fmaf(-h0.y, y0.x, fmaf(h0.x, y0.y, wa.y));
      wb.x = fmaf(h1.y, y1.y, fmaf(h1.x, y1.x, wb.x));
      wb.y = fmaf(-h1.y, y1.x, fmaf(h1.x, y1.y, wb.y));
    }
    const zd w = {(double)wa.x + (double)wb.x, (double)wa.y + (double)wb.y};
    double al = x.x * w.x + x.y * w.y, yy = nrm2(w), py = pp.x * w.x + pp.y * w.y;
    wave_sum3_dpp(al, yy, py);
    const double bb = sqrt(fmax(yy - al * al - 2.0 * beta_prev * py + beta_prev * beta_prev, 0.0));
    if (lane == j) {
      ta = al;
      tb = bb;
    }
    const int msz = j + 1;
    tmax = fmax(tmax, fabs(al) + bb);
    const bool breakdown = !(bb > 1e-13 * tmax);
    bool stop = breakdown || msz == m;
    if (breakdown || (msz >= 12 && (msz % 2) == 0) || msz == m) {
      bool conv = false;
      theta = (tmax > 0.0) ? wave_tridiag_lmax(ta, tb, msz, tmax, theta, ltol, tp, &conv) : 0.0;
      stop = stop || conv;
    }
    if (stop) break;
    const zd xn = scal(1.0 / bb, w - scal(al, x) - scal(beta_prev, pp));
    pp = x;
    x = xn;
    beta_prev = bb;
  }
  if (lane == 0) gb[blockIdx.x] = (theta > 0.0) ? 1.0 / (2.0 * theta) : 0.0;
}

template <class S>
__global__ __launch_bounds__(256, 1) void ammse_fast_kernel(ammse_kparams_t p) {
  const int N = p.desc[blockIdx.x].N;   // uniform over the workgroup
  if (N == 4) fast_body<S, 2>(p);
  else if (N == 2) fast_body<S, 1>(p);
  else fast_body<S, 0>(p);
}


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
  ammse_kparams_t q = p;
  q.gbound = nullptr;
  if (!p.wsr_only && p.step_rule == AMMSE_STEP_BOUND && !(p.gamma_c > 0.0) &&
      p.max_iters > p.T_c) {
    // the stage-II step bound, one double per launch position in the workspace
    q.gbound = (double*)p.ws;
    hipLaunchKernelGGL(ammse_fast_bound_kernel, dim3(p.batch), dim3(64), 0, s, p, q.gbound);
  }
  hipLaunchKernelGGL(ammse_fast_kernel<Shape64>, dim3(p.batch), dim3(256), Shape64::bytes, s, q);
  return hipGetLastError();
}
