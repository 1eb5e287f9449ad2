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
//   step size 1/||2 A_c||_2 by Lanczos on A_c = H^H S D S H (adaptive window);
//                                     after it, in stage II, 1/Lhat_c with Lhat_c/2 =
//                                     lambda_max(H_c^H S diag(alpha) S H_c), once per solve
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

#include <mutex>
#include <type_traits>

#include "ammse_internal.h"

#include "ammse_device.h"
#include "ammse_gemm.h"

namespace {
using namespace ammse_dev;

template <class R>
struct Smem {
  alignas(16) char tiles[tile_bytes<R>()];
  double invsig[AMMSE_MAX_USERS];
  double alpha[AMMSE_MAX_USERS];
  int cellOf[AMMSE_MAX_USERS];
  int local[AMMSE_MAX_USERS];
  int cu[AMMSE_MAX_CELLS];
  int colOff[AMMSE_MAX_CELLS + 1];
  double Pc[AMMSE_MAX_CELLS];
  double gamma[AMMSE_MAX_CELLS];
  double gbound[AMMSE_MAX_CELLS];  // 1 / Lhat_c, the stage-II step of the bound rule
  double scur[AMMSE_MAX_CELLS];    // projection factor of the current iterate per BS
  double sprev[AMMSE_MAX_CELLS];   // and of the previous one
  double mu[AMMSE_MAX_CELLS];      // WMMSE: dual variable of each BS (warm start)
  double la[AMMSE_MAX_LANCZOS];
  double lb[AMMSE_MAX_LANCZOS];
  double2 tp[64];   // Sturm-count operands of the FP32 Lanczos checks (wave 0)
  double red[16];
  double gfix;   // the fixed step gamma_c of the options
  int fail;
  int imin;
};

// Largest eigenvalue of the Hermitian float matrix K of order n <=
// AMMSE_GRAM_WAVE_N (row-major; row r of K is read as column r, conj(K[c n + r])
// = K(r, c), coalesced over r) by the three-term Lanczos iteration inside one
// wave, with no block barriers: lane l holds entries l, l + 64, l + 128 of the
// vectors, q is broadcast through qs (n + 16 float pairs of wave-private LDS,
// zero past n) and the products run in float over 8 columns at a time,
// combined in double.  tp: 64 pairs of wave-private LDS for the Sturm counts.
// The start vector, the step limit and the convergence test are those of the
// block-wide iteration for float storage (beta from the norms; converged when
// the value moves by less than 1e-8 relative); a check here costs a fraction
// of a step (which reads K from memory), so checks run from step 12 on every
// 2 steps (block-wide: every 4) and at the last.
__device__ double wave_lanczos_lmax(const cx<float>* __restrict__ K, int n, int steps,
                                    float2* qs, double2* tp) {
  const int lane = threadIdx.x & 63;
  const int nk = (n + 63) >> 6;                  // row blocks (1..3), uniform
  zd x[3], pp[3];
  double nn = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = lane + 64 * k;
    x[k] = (i < n) ? zd{1.0 + 0.5 * sin(0.731 * i + 0.25), 0.3 * cos(1.37 * i + 0.5)}
                   : zd{0.0, 0.0};
    pp[k] = {0.0, 0.0};
    nn += nrm2(x[k]);
  }
  const double i0 = 1.0 / sqrt(wave_sum(nn));
#pragma unroll
  for (int k = 0; k < 3; ++k) x[k] = scal(i0, x[k]);
  if (lane < 16) qs[n + lane] = make_float2(0.f, 0.f);
  const int m = max(1, min(steps, n));
  const double ltol = 1e-8;
  double ta = 0.0, tb = 0.0;                     // T entries, lane j holds entry j
  double beta_prev = 0.0, tmax = 0.0, theta = 0.0;
  for (int j = 0;; ++j) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k < nk && lane + 64 * k < n) qs[lane + 64 * k] = make_float2((float)x[k].x, (float)x[k].y);
    __builtin_amdgcn_wave_barrier();
    zd w[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    // w = K x over chunks of 8 columns; the chunk's loads for NK row blocks from
    // block K0 on are issued together (rows past n read row n - 1 and are
    // discarded below)
    auto matvec = [&](auto k0c, auto nkc) __attribute__((always_inline)) {
      constexpr int K0 = decltype(k0c)::value, NK = decltype(nkc)::value;
      for (int c0 = 0; c0 < n; c0 += 8) {
        float2 qv[8];
        cx<float> kv[NK][8];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          const int r = min(lane + 64 * (K0 + k), n - 1);
#pragma unroll
          for (int u = 0; u < 8; ++u) kv[k][u] = K[(long)min(c0 + u, n - 1) * n + r];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) qv[u] = qs[c0 + u];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          float ax = 0.f, ay = 0.f, bx = 0.f, by = 0.f;
#pragma unroll
          for (int u = 0; u < 8; u += 2) {        // K(r, c) q_c, K(r, c) = conj(kv)
            ax = fmaf(kv[k][u].x, qv[u].x, fmaf(kv[k][u].y, qv[u].y, ax));
            ay = fmaf(kv[k][u].x, qv[u].y, fmaf(-kv[k][u].y, qv[u].x, ay));
            bx = fmaf(kv[k][u + 1].x, qv[u + 1].x, fmaf(kv[k][u + 1].y, qv[u + 1].y, bx));
            by = fmaf(kv[k][u + 1].x, qv[u + 1].y, fmaf(-kv[k][u + 1].y, qv[u + 1].x, by));
          }
          w[K0 + k].x += (double)ax + (double)bx;
          w[K0 + k].y += (double)ay + (double)by;
        }
      }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    if (nk == 1) {
      matvec(I0{}, I1{});
    } else {                                       // two row blocks at a time at most
      matvec(I0{}, I2{});
      if (nk == 3) matvec(I2{}, I1{});
    }
    double al = 0.0, yy = 0.0, py = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (lane + 64 * k >= n) w[k] = {0.0, 0.0};
      al += x[k].x * w[k].x + x[k].y * w[k].y;
      yy += nrm2(w[k]);
      py += pp[k].x * w[k].x + pp[k].y * w[k].y;
    }
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
    const double ib = 1.0 / bb;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const zd xn = scal(ib, w[k] - scal(al, x[k]) - scal(beta_prev, pp[k]));
      pp[k] = x[k];
      x[k] = xn;
    }
    beta_prev = bb;
  }
  return theta;
}
static_assert((AMMSE_BLOCK / 64) * ((AMMSE_GRAM_WAVE_N + 16) * sizeof(float2) + 64 * sizeof(double2)) <=
                  3 * AMMSE_LANCZOS_LDS_N * sizeof(zd),
              "the per-wave Gram Lanczos buffers fit the A-MMMSE dynamic LDS");

// K = C^H Q C ((U N) x (U N)) for the Q-path Lanczos, C block diagonal with an
// N x N block per user (Cm: 4 x 4 padded, double), Q exactly Hermitian.  One
// thread per entry, in row-major order so that the reads of Q and the writes
// of K are coalesced; an entry below the diagonal is the conjugate of its
// mirror computed with the same operations on the same values in the same
// order (Q's own block read and conjugated, Q being exactly Hermitian), so K
// is exactly Hermitian.  Compiled per N; two entries per trip with the loads
// of both issued first (the pointers are restrict-qualified, so they need not
// wait for the previous trip's stores).
template <class R, int NN>
__device__ __forceinline__ void kq_form_n(const cx<R>* __restrict__ Q, const zd* __restrict__ Cm,
                                          cx<R>* __restrict__ K, int U, int tid) {
  const int un = U * NN, ne = un * un;
  const float run = 1.f / (float)un;
  constexpr int QB = 2;
  for (int e0 = tid; e0 < ne; e0 += QB * AMMSE_BLOCK) {
    cx<R> qb[QB][NN][NN];
    zd co[QB][NN], ci[QB][NN];
    int ii[QB], jj[QB];
    bool up[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = min(e0 + q * AMMSE_BLOCK, ne - 1);
      const int i = quot(e, run), j = e - i * un;
      const int u = i / NN, a = i - u * NN, v = j / NN, b = j - v * NN;
      ii[q] = i;
      jj[q] = j;
      up[q] = i <= j;
      // outer side (conjugated C) and inner side: (u, a) and (v, b) on and
      // above the diagonal, swapped below it
      const int pu = up[q] ? u : v, pa = up[q] ? a : b, su = up[q] ? v : u, sb = up[q] ? b : a;
#pragma unroll
      for (int k = 0; k < NN; ++k) {
        co[q][k] = Cm[pu * 16 + k * 4 + pa];
        ci[q][k] = Cm[su * 16 + k * 4 + sb];
#pragma unroll
        for (int l = 0; l < NN; ++l) qb[q][k][l] = Q[(long)(u * NN + k) * un + v * NN + l];
      }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      zd acc = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < NN; ++k) {
        zd t = {0.0, 0.0};
#pragma unroll
        for (int l = 0; l < NN; ++l)
          t = t + (up[q] ? to_d(qb[q][k][l]) : cj(to_d(qb[q][l][k]))) * ci[q][l];
        acc = acc + cj(co[q][k]) * t;
      }
      if (ii[q] == jj[q]) acc.y = 0.0;
      if (e0 + q * AMMSE_BLOCK < ne) K[(long)ii[q] * un + jj[q]] = from_d<R>(up[q] ? acc : cj(acc));
    }
  }
}
template <class R>
__device__ __forceinline__ void kq_form(const cx<R>* Q, const zd* Cm, cx<R>* K, int U, int N,
                                        int tid) {
  switch (N) {
    case 1: kq_form_n<R, 1>(Q, Cm, K, U, tid); break;
    case 2: kq_form_n<R, 2>(Q, Cm, K, U, tid); break;
    case 3: kq_form_n<R, 3>(Q, Cm, K, U, tid); break;
    default: kq_form_n<R, 4>(Q, Cm, K, U, tid); break;
  }
}

// Epilogue of the single-cell Q-path product P = Q X~ (row-major, leading
// dimension ld): G~ = c~ G^0 + P written over G^{t-2}, and the thread's partial
// sum of 2 c~ Re<G^0, X~> + Re<X~, P> for the power of the extrapolated step.
// The reads of X~ and G^0 form the load phase (see has_pre).
template <class R>
struct QpathEpi {
  const cx<R>* X;
  const cx<R>* G0;
  cx<R>* G;
  long ld;
  double ch;
  double acc;
  struct L {
    cx<R> x, g0;
  };
  __device__ __forceinline__ L pre(int i, int j) const {
    const long e = (long)i * ld + j;
    return {X[e], G0[e]};
  }
  template <class V>
  __device__ __forceinline__ void operator()(int i, int j, V pq, const L& l) {
    acc += 2.0 * ch * ((double)l.g0.x * l.x.x + (double)l.g0.y * l.x.y) +
           ((double)l.x.x * pq.x + (double)l.x.y * pq.y);
    G[(long)i * ld + j] =
        from_d<R>(zd{ch * (double)l.g0.x + (double)pq.x, ch * (double)l.g0.y + (double)pq.y});
  }
  template <class V>
  __device__ __forceinline__ void operator()(int i, int j, V pq) {
    (*this)(i, j, pq, pre(i, j));
  }
};

// Stage-II step of the bound rule for the general kernel's instances that
// ammse_bound_gram selects (float storage, not the single-cell Q path,
// M <= AMMSE_GRAM_WAVE_N): for every BS c with users, 1 / (2 lambda_max(A_c)),
// A_c = R_c^H R_c, R_c = S_a H_{:,c}, S_a = diag(sqrt(alpha_u) / sigma_u).
// R_c is formed in one pass over H_{:,c}, A_c by one MFMA product (made
// exactly Hermitian), then one wave per BS runs the Lanczos iteration of the
// step size (wave_lanczos_lmax) on its A_c.  The bound depends only on the
// channel, the noise powers and the weights, so this kernel runs before the
// solve kernel (one workgroup per instance, same stream) and writes the
// values into the instance workspace, where the solve kernel reads them when
// its second stage first needs them.  Other instances return at once.
__global__ __launch_bounds__(AMMSE_BLOCK, 2) void ammse_bound_gram_kernel(ammse_kparams_t p) {
  __shared__ __align__(16) char tiles[tile_bytes<float>()];
  __shared__ float2 qsa[4 * (AMMSE_GRAM_WAVE_N + 16)];
  __shared__ double2 tpa[4 * 64];
  __shared__ double sa[AMMSE_MAX_USERS];
  const ammse_desc_t D = p.desc[blockIdx.x];
  const int C = D.C, U = D.U, M = D.M, N = D.N, d = D.d, un = D.un;
  const bool wm = p.algorithm == AMMSE_ALGO_WMMSE || p.algorithm == AMMSE_ALGO_MMMSE;
  const bool bc = p.algorithm == AMMSE_ALGO_BCGD;
  if (!ammse_bound_gram(4, C, U, M, N, wm, bc)) return;   // uniform over the workgroup
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = (p.tile_force > 0) ? p.tile_force - 1 : D.tile;
  const ammse_ws_layout_t L =
      ammse_ws_layout(4, C, U, M, N, d, p.lanczos_steps, wm, p.bf16_copies != 0, bc);
  char* ws = p.ws + D.ws_off;
  cx<float>* Rb = (cx<float>*)(ws + L.Rb);
  cx<float>* Ab = (cx<float>*)(ws + L.Ab);
  double* gb = (double*)(ws + L.Gb);
  const cx<float>* H = (const cx<float>*)p.H + D.h_off;
  for (int u = tid; u < U; u += AMMSE_BLOCK)
    sa[u] = sqrt(p.alpha[D.user_off + u] / p.sigma2[D.user_off + u]);
  __syncthreads();
  for (int c = 0; c < C; ++c) {
    if (p.cell_users[D.cell_off + c] == 0) continue;   // no precoder, no step
    const cx<float>* __restrict__ Hc = H + (long)c * un * M;
    cx<float>* __restrict__ Ac = Ab + (long)c * M * M;
    // four elements per trip, every load issued before the stores; the row's
    // user by quot (un M < 2^22)
    const float rM = 1.f / (float)M, rN = 1.f / (float)N;
    for (int e0 = tid; e0 < un * M; e0 += 4 * AMMSE_BLOCK) {
      cx<float> h[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) h[q] = Hc[min(e0 + q * AMMSE_BLOCK, un * M - 1)];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * AMMSE_BLOCK;
        if (e >= un * M) continue;
        const double f = sa[quot(quot(e, rM), rN)];
        Rb[e] = {(float)(f * (double)h[q].x), (float)(f * (double)h[q].y)};
      }
    }
    __syncthreads();
    // exactly Hermitian: the computed upper triangle, its conjugate transpose
    // below the diagonal and a real diagonal
    channel_gemm<float, true, false>(M, M, un, Rb, M, Rb, M, tiles, false, tile,
                                     [&](int i, int j, cx<float> v) {
                                       if (i < j) {
                                         Ac[(long)i * M + j] = v;
                                         Ac[(long)j * M + i] = {v.x, -v.y};
                                       } else if (i == j) {
                                         Ac[(long)i * M + j] = {v.x, 0.f};
                                       }
                                     });
    __syncthreads();
  }
  float2* qs = qsa + wave * (AMMSE_GRAM_WAVE_N + 16);
  double2* tp = tpa + wave * 64;
  for (int c = wave; c < C; c += AMMSE_BLOCK / 64) {
    const double lm = (p.cell_users[D.cell_off + c] == 0)
                          ? 0.0
                          : wave_lanczos_lmax(Ab + (long)c * M * M, M, p.lanczos_steps, qs, tp);
    if (lane == 0) gb[c] = (lm > 0.0) ? 1.0 / (2.0 * lm) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// The fused kernel
// ---------------------------------------------------------------------------
// QP = 1: the instances of the single-cell Q path (ammse_qpath_instance), QP =
// 0: all others; the plan puts the former first in launch order and each
// variant runs over its own range (block_base), so that neither carries the
// other's code.
template <class R, int QP>
__global__ __launch_bounds__(AMMSE_BLOCK, sizeof(R) == 4 ? 2 : 1) void ammse_solve_kernel(
    ammse_kparams_t p) {
  __shared__ Smem<R> sm;
  extern __shared__ __align__(16) char dyn_lds[];   // WMMSE / MMMSE: Cholesky factor
  const ammse_desc_t D = p.desc[p.block_base + blockIdx.x];
  if constexpr (QP != 0) {
    if (!ammse_qpath_instance(D.C, D.U, D.M, D.N, p.algorithm)) {
      // not an instance of this variant (the plan never launches one here)
      if (threadIdx.x == 0) {
        p.wsr[D.b] = NAN;
        if (p.status) p.status[D.b] = AMMSE_INST_NONFINITE;
      }
      return;
    }
  }
  // output tile shape of the channel products: forced by the options, else
  // the plan's (autotuned) choice for this instance's shape class
  const int tile = (p.tile_force > 0) ? p.tile_force - 1 : D.tile;
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

  // exact V step (Algorithm 2 / MMMSE); BCGD-WMMSE (explicit steps for U, W, V)
  const bool wm = p.algorithm == AMMSE_ALGO_WMMSE || p.algorithm == AMMSE_ALGO_MMMSE;
  const bool bc = p.algorithm == AMMSE_ALGO_BCGD;
  // stream-space Lanczos with Q = S H H^H S, one product with Q per iteration
  const bool qpath = QP != 0;
  const bool gpath = ammse_gram_path((int)sizeof(R), C, U, M, N, d, wm || bc);   // ... K = R R^H
  // float storage on the Q path: one product with Q per iteration, the
  // precoder carried implicitly as V = c V^0 + H^H S X (see the update below);
  // in bfloat16 iterations that product takes bfloat16 operands, and the
  // refinement pass starts from G^{t-1}, G^{t-2} recomputed with float products.
  const bool rpath = qpath && sizeof(R) == 4;
  // stage-II bound from the antenna-side Gram matrices (see ammse_bound_gram)
  const bool bgram = ammse_bound_gram((int)sizeof(R), C, U, M, N, wm, bc);
  const ammse_ws_layout_t L =
      ammse_ws_layout((int)sizeof(R), C, U, M, N, d, p.lanczos_steps, wm, p.bf16_copies != 0, bc);
  char* ws = p.ws + D.ws_off;
  cx<R>* Gp = (cx<R>*)(ws + L.Gp);
  cx<R>* Gq = (cx<R>*)(ws + L.Gq);
  cx<R>* Z = (cx<R>*)(ws + L.Z);
  cx<R>* Vq = (cx<R>*)(ws + L.Vq);
  zd* UWm = (zd*)(ws + L.UWm);
  zd* Em = (zd*)(ws + L.Em);
  zd* Dm = (zd*)(ws + L.Dm);
  zd* Ym = (zd*)(ws + L.Ym);
  cx<float>* Dmf = (cx<float>*)(ws + L.Dmf);   // float copies (float storage)
  cx<float>* Ymf = (cx<float>*)(ws + L.Ymf);
  zd* Lq = (zd*)(ws + L.Lq);
  zd* Lw = (zd*)(ws + L.Lw);
  zd* Ly1 = (zd*)(ws + L.Ly1);
  zd* Ly2 = (zd*)(ws + L.Ly2);
  zd* Am = (zd*)(ws + L.Am);
  zd* Lm = (zd*)(ws + L.Lm);
  zd* Bm = (zd*)(ws + L.Bm);
  zd* Xm = (zd*)(ws + L.Xm);
  zd* Tm = (zd*)(ws + L.Tm);
  cx<R>* Qm = (cx<R>*)(ws + L.Qm);
  cx<R>* Kq = (cx<R>*)(ws + L.Kq);
  bfc* Hb = (bfc*)(ws + L.Hb);     // bfloat16 operand copies (mixed precision)
  bfc* Xb = (bfc*)(ws + L.Xb);
  bfc* Zb = (bfc*)(ws + L.Zb);
  // bfloat16 copies of H, the precoder and Z for the two-product form (the Q
  // path converts its operands while staging them)
  const bool copies = sizeof(R) == 4 && p.bf16_copies && p.lowp_iters >= 1 && !p.wsr_only &&
                      !rpath;
  zd* Lwm = (zd*)(ws + L.Lwm);
  zd* Lim = (zd*)(ws + L.Lim);
  zd* Cm = (zd*)(ws + L.Cm);
  cx<R>* Rg = (cx<R>*)(ws + L.Rg);
  cx<R>* Kg = (cx<R>*)(ws + L.Kg);
  const double* Gbw = (const double*)(ws + L.Gb);   // stage-II bound (bgram below)
  zd* Ubm = (zd*)(ws + L.Ubm);       // BCGD-WMMSE: U, W iterates, J and G_own of V^{t-1}
  zd* Wbm = (zd*)(ws + L.Wbm);
  zd* Jbm = (zd*)(ws + L.Jbm);
  zd* Fbm = (zd*)(ws + L.Fbm);
  cx<R>* X1 = (cx<R>*)(ws + L.X1);   // Q recursion: X^{t-1}, X^{t-2}, G^0
  cx<R>* X2 = (cx<R>*)(ws + L.X2);
  cx<R>* G0 = (cx<R>*)(ws + L.G0);
  const cx<R>* H = (const cx<R>*)p.H + D.h_off;
  cx<R>* V = (cx<R>*)p.V + D.v_off;
  const long Vtot = (long)M * D.ud;

  // G_c = S H_{:,c} (scale_c X_c) for every BS c: X holds the precoders up
  // to the per-BS factor of the sum-power projection, which is applied here
  // (by linearity) instead of rewriting X.
  const float rN = 1.f / (float)N;   // row i of G belongs to user quot(i, rN)
  auto channel_product = [&](cx<R>* G, const cx<R>* X, const double* scale, bool lowp) {
    for (int c = 0; c < C; ++c) {
      const int nc = sm.cu[c] * d;
      if (nc == 0) continue;
      cx<R>* __restrict__ Gc = G + (long)un * sm.colOff[c];
      const double sc = scale[c];
      auto epi = [&](int i, int j, cx<R> v) {
        const R f = (R)(sc * sm.invsig[quot(i, rN)]);
        Gc[(long)i * nc + j] = {f * v.x, f * v.y};
      };
      if constexpr (sizeof(R) == 4) {
        if (lowp && copies) {   // bfloat16 copies of H and of X (the current precoder)
          channel_gemm_bf16<false>(un, nc, M, Hb + (long)c * un * M, M,
                                   Xb + (long)M * sm.colOff[c], nc, sm.tiles, tile, epi);
          continue;
        }
      }
      channel_gemm<R, false>(un, nc, M, H + (long)c * un * M, M, X + (long)M * sm.colOff[c], nc,
                             sm.tiles, lowp, tile, epi);
    }
  };

  // Per-user receiver algebra on G (normalised products of the current V):
  // one user per 16-lane group, lane 4a + b holding entry (a, b) of the
  // user's N x N and d x d matrices zero/identity-padded to 4 x 4.
  //   J- = I + sum of G G^H over the columns of the other streams
  //   F = L^{-1} G_own (J- = L L^H), W = E^{-1} = I + F^H F, R = log det W,
  //   UW = J-^{-1} G_own, E = Lw^{-H} Lw^{-1}
  // UW and E go to the workspace; returns the sum of alpha_u R_u (nats) over
  // the block.
  // BCGD-WMMSE: the full J and G_own go to the workspace as well, and with
  // bc_init the MMSE weights W = I + F^H F (zero outside d x d).
  auto receivers = [&](const cx<R>* G, double gscale, bool bc_init = false) -> double {
    const int tid = phase_tid();
    const int lane = tid & 63, li = lane & 15;
    const Lane4 L4{lane & ~15, li >> 2, li & 3};
    const int ea = L4.a, eb = L4.b;
    double rsum = 0.0;
    bool ok = true;
    for (int u0 = 0; u0 < U; u0 += AMMSE_BLOCK / 16) {
      const int u = u0 + (tid >> 4);
      const bool act = u < U;
      const int uu = act ? u : U - 1;
      const int cown = sm.cellOf[uu], j0 = sm.local[uu] * d;
      // J-: lane li accumulates all N x N entries over the stream columns
      // t = li (mod 16) of the other streams (t runs over the per-BS blocks
      // one after the other), then a reduce-scatter over the 16 lanes leaves
      // entry (a, b) on lane 4a + b.  The sums are in the storage precision's
      // working type (float with float storage, as in the LDS-resident
      // kernel), scaled by gscale^2 at the end.  Compiled per N; the lane's
      // columns go in chunks of CH with the loads of a whole chunk issued
      // before its arithmetic (CH N = 16 loads in flight with float storage,
      // 8 with double).
      using TJ = typename std::conditional<sizeof(R) == 4, float, double>::type;
      cx<TJ> sj[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) sj[q] = {TJ(0), TJ(0)};
      auto cov = [&](auto nn) __attribute__((always_inline)) {
        constexpr int NN = decltype(nn)::value;
        constexpr int CH = (sizeof(R) == 4 ? 16 : 8) / (NN == 3 ? 4 : NN);
        const int nstr = sm.colOff[C];
        int c = 0;
        for (int t0 = li; t0 < nstr; t0 += 16 * CH) {
          cx<R> g[CH][NN];
          bool use[CH];
#pragma unroll
          for (int q = 0; q < CH; ++q) {
            const int t = min(t0 + 16 * q, nstr - 1);
            while (c < C - 1 && t >= sm.colOff[c + 1]) ++c;   // BS of column t
            const int nc = sm.cu[c] * d, col = t - sm.colOff[c];
            const cx<R>* r0 = G + (long)un * sm.colOff[c] + (long)(uu * NN) * nc + col;
#pragma unroll
            for (int k = 0; k < NN; ++k) g[q][k] = r0[(long)k * nc];
            use[q] = t0 + 16 * q < nstr && !(c == cown && col >= j0 && col < j0 + d);
          }
#pragma unroll
          for (int q = 0; q < CH; ++q) {
            if (!use[q]) continue;
            cx<TJ> gt[NN];
#pragma unroll
            for (int k = 0; k < NN; ++k) gt[k] = {(TJ)g[q][k].x, (TJ)g[q][k].y};
#pragma unroll
            for (int x = 0; x < NN; ++x)
#pragma unroll
              for (int y = 0; y < NN; ++y) sj[x * 4 + y] = sj[x * 4 + y] + mulc(gt[x], gt[y]);
          }
        }
      };
      switch (N) {
        case 1: cov(std::integral_constant<int, 1>{}); break;
        case 2: cov(std::integral_constant<int, 2>{}); break;
        case 3: cov(std::integral_constant<int, 3>{}); break;
        default: cov(std::integral_constant<int, 4>{}); break;
      }
#pragma unroll
      for (int step = 0; step < 4; ++step) {
        const int bit = 8 >> step;                 // 8, 4, 2, 1 entries exchanged
        const bool hi = (li & bit) != 0;
#pragma unroll
        for (int q = 0; q < bit; ++q) {
          const cx<TJ> send = hi ? sj[q] : sj[q + bit];
          const cx<TJ> keep = hi ? sj[q + bit] : sj[q];
          sj[q] = keep + cx<TJ>{__shfl_xor(send.x, bit, 64), __shfl_xor(send.y, bit, 64)};
        }
      }
      zd J = {(ea == eb) ? 1.0 : 0.0, 0.0}, F = {0.0, 0.0};
      if (ea < N && eb < N) J = J + scal(gscale * gscale, to_d(sj[0]));
      if (ea < N && eb < d) {
        const int c = cown, nc = sm.cu[c] * d;
        F = scal(gscale, to_d(G[(long)un * sm.colOff[c] + (long)(uu * N + ea) * nc + j0 + eb]));
      }
      if (bc && act) {                            // J = J- + G_own G_own^H
        Jbm[u * 16 + li] = J + mm_nh(L4, F, F);
        Fbm[u * 16 + li] = F;
      }
      bool oku = true;
      double io[4], iw[4];                        // reciprocal diagonals of the factors
      const zd Lo = chol16(L4, J, oku, io);
      F = trsm16(L4, Lo, io, F);                  // L^{-1} G_own
      zd X = mm_hn(L4, F, F);                     // I + F^H F
      if (bc_init && act)
        Wbm[u * 16 + li] = (ea == eb && ea < d) ? zd{X.x + 1.0, 0.0} : X;
      if (ea == eb) X = {X.x + 1.0, 0.0};
      const zd UWv = trsm16h(L4, Lo, io, F);      // J-^{-1} G_own
      const zd Lw = chol16(L4, X, oku, iw);
      const zd Li = trsm16(L4, Lw, iw, zd{(ea == eb) ? 1.0 : 0.0, 0.0});
      const zd Ev = mm_hn(L4, Li, Li);            // E = Lw^{-H} Lw^{-1}
      if (act) {
        if (ea == eb) rsum += sm.alpha[u] * 2.0 * log(Lw.x);
        UWm[u * 16 + li] = UWv;
        Em[u * 16 + li] = Ev;
        if (wm) Lwm[u * 16 + li] = Lw;
        if (wm || qpath || gpath) Lim[u * 16 + li] = Li;
        ok = ok && oku;
      }
    }
    if (!ok) atomicOr(&sm.fail, AMMSE_INST_CHOLESKY);
    return rsum;
  };

  // WSR in bits from the per-thread rate sums (all threads get the value).
  auto wsr_sum = [&](double rs) { return block_sum(rs, sm.red) * (1.0 / M_LN2); };

  // D_u = alpha U W U^H and Y_u = alpha U W into the workspace (padded 4 x 4):
  // stage I uses W = I (U = UW E), stage II W = E^{-1} (U W = UW).
  auto weights = [&](bool stage2) {
    const int tid = phase_tid();
    const int lane = tid & 63, li = lane & 15;
    const Lane4 L4{lane & ~15, li >> 2, li & 3};
    for (int u0 = 0; u0 < U; u0 += AMMSE_BLOCK / 16) {
      const int u = u0 + (tid >> 4);
      const bool act = u < U;
      const int uu = act ? u : U - 1;
      const zd UWv = UWm[uu * 16 + li], Ev = Em[uu * 16 + li];
      const zd T = mm_nn(L4, UWv, Ev);            // U
      const zd Ur = stage2 ? UWv : T;
      zd Dv = mm_nh(L4, T, Ur);
      const zd Dt = L4.at(Dv, L4.b, L4.a);
      Dv = {0.5 * (Dv.x + Dt.x), 0.5 * (Dv.y - Dt.y)};   // exactly Hermitian
      const double al = sm.alpha[uu];
      if (act) {
        Dm[u * 16 + li] = scal(al, Dv);
        Ym[u * 16 + li] = scal(al, Ur);
        if constexpr (sizeof(R) == 4) {
          Dmf[u * 16 + li] = from_d<float>(scal(al, Dv));
          Ymf[u * 16 + li] = from_d<float>(scal(al, Ur));
        }
      }
      if (wm || qpath || gpath) {   // D = C C^H: C = sqrt(alpha) UW Lw^{-H} (stage II) or sqrt(alpha) U (stage I)
        const zd Cv = scal(sqrt(al), stage2 ? mm_nh(L4, UWv, Lim[uu * 16 + li]) : T);
        if (act) Cm[u * 16 + li] = Cv;
      }
    }
    __syncthreads();
  };

  // BCGD-WMMSE (Section VII-F ablation), per user on the normalised channel
  // (unit noise): U <- U - (J U W - G_own W) / (||J||_F ||W||_F) (one gradient
  // step of f in U, the step bounding the block Lipschitz constant), then
  // E = I - U^H G_own - G_own^H U + U^H J U at the new U and the Schulz step
  // W <- W (2I - E W); D = alpha U W U^H and Y = alpha U W for the V step.
  // init: U and W start as the MMSE receivers (U W E, U W from the receivers)
  // and W = E^{-1}.  Blocks are zero outside N x d and d x d.
  auto bcgd_update = [&](bool init) {
    const int tid = phase_tid();
    const int lane = tid & 63, li = lane & 15;
    const Lane4 L4{lane & ~15, li >> 2, li & 3};
    const int ea = L4.a, eb = L4.b;
    const bool inN = ea < N && eb < N, inD = ea < d && eb < d;
    for (int u0 = 0; u0 < U; u0 += AMMSE_BLOCK / 16) {
      const int u = u0 + (tid >> 4);
      const bool act = u < U;
      const int uu = act ? u : U - 1;
      const zd J = Jbm[uu * 16 + li], G = Fbm[uu * 16 + li];
      const zd Ub = init ? mm_nn(L4, UWm[uu * 16 + li], Em[uu * 16 + li]) : Ubm[uu * 16 + li];
      const zd Wb = Wbm[uu * 16 + li];
      const zd Rg = mm_nn(L4, mm_nn(L4, J, Ub), Wb) - mm_nn(L4, G, Wb);
      const double nj = row16_sum(inN ? nrm2(J) : 0.0), nw = row16_sum(inD ? nrm2(Wb) : 0.0);
      const double al = sm.alpha[uu];
      const double st = (al > 0.0 && nj * nw > 0.0) ? 1.0 / sqrt(nj * nw) : 0.0;
      const zd Un = Ub - scal(st, Rg);
      const zd UhG = mm_hn(L4, Un, G);
      zd Eb = mm_hn(L4, Un, mm_nn(L4, J, Un)) - UhG - cj(L4.at(UhG, eb, ea));
      if (ea == eb && ea < d) Eb.x += 1.0;
      zd T2 = scal(-1.0, mm_nn(L4, Eb, Wb));
      if (ea == eb && ea < d) T2.x += 2.0;
      zd Wn = mm_nn(L4, Wb, T2);
      const zd Wt = L4.at(Wn, eb, ea);
      Wn = {0.5 * (Wn.x + Wt.x), 0.5 * (Wn.y - Wt.y)};   // Hermitian part
      const zd UWn = mm_nn(L4, Un, Wn);
      zd Dv = mm_nh(L4, UWn, Un);
      const zd Dt = L4.at(Dv, eb, ea);
      Dv = {0.5 * (Dv.x + Dt.x), 0.5 * (Dv.y - Dt.y)};
      if (act) {
        Ubm[u * 16 + li] = Un;
        Wbm[u * 16 + li] = Wn;
        Dm[u * 16 + li] = scal(al, Dv);
        Ym[u * 16 + li] = scal(al, UWn);
        if constexpr (sizeof(R) == 4) {
          Dmf[u * 16 + li] = from_d<float>(scal(al, Dv));
          Ymf[u * 16 + li] = from_d<float>(scal(al, UWn));
        }
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
  // Plain three-term Lanczos for the largest eigenvalue of a Hermitian PSD
  // operator of order nl (the largest Ritz value converges without
  // re-orthogonalisation).  apply(q, w) writes w = Op q (vectors in the
  // workspace).  FP64 forms ||w - alpha q - beta p|| explicitly, FP32 uses
  // beta^2 = ||w||^2 - alpha^2 - 2 beta_prev Re(p^H w) + beta_prev^2.
  // The three vectors live in the dynamic LDS area when they fit (order <=
  // AMMSE_LANCZOS_LDS_N), else in the workspace.
  auto lanczos_core = [&](int nl, auto&& apply) __attribute__((always_inline)) {
   auto run = [&](zd* qv, zd* pv, zd* wv) __attribute__((always_inline)) {
    const int tid = phase_tid();
    for (int i = tid; i < nl; i += AMMSE_BLOCK) {
      qv[i] = {1.0 + 0.5 * sin(0.731 * i + 0.25), 0.3 * cos(1.37 * i + 0.5)};
      pv[i] = {0.0, 0.0};
    }
    double nn = 0.0;
    for (int i = tid; i < nl; i += AMMSE_BLOCK) nn += nrm2(qv[i]);
    nn = block_sum(nn, sm.red);
    for (int i = tid; i < nl; i += AMMSE_BLOCK) qv[i] = scal(1.0 / sqrt(nn), qv[i]);
    __syncthreads();
    const int m = min(p.lanczos_steps, nl);
    constexpr bool exact_beta = sizeof(R) == 8;
    const double ltol = exact_beta ? 1e-14 : 1e-8;
    const double rtol = 1e-16;   // FP64 checks (the FP32 multisection stops at 1e-10)
    const int first = exact_beta ? 8 : 12, every = exact_beta ? 8 : 4;
    double beta_prev = 0.0, tmax = 0.0, theta = 0.0;
    // apply() writes w[i] from thread i mod AMMSE_BLOCK (or ends with a
    // barrier), so each thread reads back only its own entries below; the
    // barrier after the partial sums also ends every read of q, p and w
    // before the update writes them.
    for (int j = 0; j < m; ++j) {
      apply(qv, wv);
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int i = tid; i < nl; i += AMMSE_BLOCK) {
        const zd w = wv[i], q = qv[i], pp = pv[i];
        s0 += nrm2(w);
        s1 += q.x * w.x + q.y * w.y;
        s2 += pp.x * w.x + pp.y * w.y;
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
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
        for (int i = tid; i < nl; i += AMMSE_BLOCK) {
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
        bool conv = false;
        double th;
        if constexpr (exact_beta) {   // FP64: the full value at every check (block multisection)
          th = (tmax > 0.0) ? tridiag_lmax(sm.la, sm.lb, msz, &sm.imin, rtol) : 0.0;
        } else {
          // FP32: wave 0 runs the multisection, whose first round tests the
          // ltol criterion above the previous value (wave_tridiag_lmax); the
          // other waves wait at the barrier
          if (tid < 64) {
            bool cv = false;
            const double v = (tmax > 0.0) ? wave_tridiag_lmax(sm.la[tid], sm.lb[tid], msz, tmax,
                                                              theta, ltol, sm.tp, &cv)
                                          : 0.0;
            if (tid == 0) {
              sm.red[12] = v;
              sm.imin = cv ? 1 : 0;
            }
          }
          __syncthreads();
          th = sm.red[12];
          conv = sm.imin != 0;
        }
        stop = stop || conv || (exact_beta && fabs(th - theta) <= ltol * fabs(th));
        theta = th;
      }
      if (stop) break;
      const double ib = 1.0 / bb;
      for (int i = tid; i < nl; i += AMMSE_BLOCK) {
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
    if (nl <= AMMSE_LANCZOS_LDS_N) {
      zd* v = (zd*)dyn_lds;
      return run(v, v + nl, v + 2 * nl);
    }
    return run(Lq, Lq + nl, Lq + 2 * nl);
  };

  // lambda_max(A_c), A_c = H_c^H S D S H_c, on the M-dimensional operator:
  // products with H use several threads per row / column (a power of two
  // within one wave, combined by shuffles).
  auto lanczos_lmax = [&](int c) {
    const int tid = phase_tid();
    const cx<R>* __restrict__ Hc = H + (long)c * un * M;
    int tpr = 1;
    while (tpr < 64 && tpr * 2 * un <= AMMSE_BLOCK) tpr *= 2;
    int tpc = 1;
    while (tpc < 64 && tpc * 2 * M <= AMMSE_BLOCK) tpc *= 2;
    return lanczos_core(M, [&](const zd* qv, zd* wv) {
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
      {  // w = H^H y2
        const int part = tid & (tpc - 1);
        for (int i = tid / tpc; i < M; i += AMMSE_BLOCK / tpc) {
          zd acc = {0.0, 0.0};
#pragma unroll 4
          for (int r = part; r < un; r += tpc) acc = acc + cj(to_d(Hc[(long)r * M + i])) * Ly2[r];
          for (int o = 1; o < tpc; o <<= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
          }
          if (part == 0) wv[i] = acc;
        }
      }
      __syncthreads();   // w written by other threads than those that read it
    });
  };

  // lambda_max(A_c) from a Gram matrix: with D = C C^H (C block diagonal,
  // N x d per user), A_c = R_c^H R_c for R_c = C^H S H_{:,c} ((U d) x M), so
  // lambda_max(A_c) = lambda_max(K_c) for K_c = R_c R_c^H ((U d) x (U d)) or
  // K_c = A_c itself, whichever is smaller (ammse_gram_order).  R_c is formed
  // in one pass over H_{:,c}, K_c by one MFMA product (made exactly
  // Hermitian), and each Lanczos step reads K_c once instead of H_{:,c} twice.
  auto gram_form = [&](int c, cx<R>* __restrict__ Kc) {
    const int tid = phase_tid();
    const cx<R>* __restrict__ Hc = H + (long)c * un * M;
    const int ud = U * d;
    // two elements per trip, all loads of both issued before their arithmetic
    // (the stores to R would otherwise order each trip's loads after the
    // previous trip's store)
    const float rM = 1.f / (float)M, rd = 1.f / (float)d;   // quot: ud M <= 2^22
    for (int e0 = tid; e0 < ud * M; e0 += 2 * AMMSE_BLOCK) {
      cx<R> hv[2][4];
      zd cv[2][4];
      int uu[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int e = min(e0 + q * AMMSE_BLOCK, ud * M - 1);
        const int i = quot(e, rM), m = e - i * M;
        const int u = quot(i, rd), s = i - u * d;
        uu[q] = u;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int nn = min(n, N - 1);
          hv[q][n] = Hc[(long)(u * N + nn) * M + m];
          cv[q][n] = Cm[u * 16 + nn * 4 + s];
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int e = e0 + q * AMMSE_BLOCK;
        zd acc = {0.0, 0.0};
#pragma unroll
        for (int n = 0; n < 4; ++n)
          if (n < N) acc = acc + cj(cv[q][n]) * to_d(hv[q][n]);
        const double f = sm.invsig[uu[q]];
        if (e < ud * M) Rg[e] = {(R)(f * acc.x), (R)(f * acc.y)};
      }
    }
    __syncthreads();
    // square output: the 64 x 64 tile shape whatever the channel products
    // use; K made exactly Hermitian by taking the computed upper triangle
    // (its conjugate transpose below the diagonal, a real diagonal)
    const int ng = (int)ammse_gram_order(U, M, d);
    auto epi = [&](int i, int j, cx<R> v) {
      if (i < j) {
        Kc[(long)i * ng + j] = v;
        Kc[(long)j * ng + i] = {v.x, -v.y};
      } else if (i == j) {
        Kc[(long)i * ng + j] = {v.x, (R)0};
      }
    };
    if (ng < ud)   // antenna side: R^H R
      channel_gemm<R, true, false>(M, M, ud, Rg, M, Rg, M, sm.tiles, false, 0, epi);
    else           // stream side: R R^H
      channel_gemm<R, false, true>(ud, ud, M, Rg, M, Rg, M, sm.tiles, false, 0, epi);
    __syncthreads();
  };
  // Lanczos on a formed Hermitian matrix of order ud (storage precision,
  // row-major; column r read for row r, coalesced over r).  Per step w = K q:
  // q staged in LDS in the storage precision (zero past ud), nparts threads
  // per row, each over every nparts-th column, the loads of a chunk of
  // kDenseChunk columns issued together and the chunk's products in the
  // storage precision summed in double; partial sums combined through LDS
  // (the product tiles, free here).
  constexpr int kDenseChunk = 8;
  auto lanczos_dense = [&](const cx<R>* Kd, int ud) __attribute__((always_inline)) {
    const int tid = phase_tid();
    const int nparts = (ud >= AMMSE_BLOCK) ? 1 : AMMSE_BLOCK / ud;
    zd* partial = (zd*)sm.tiles;
    cx<R>* qs = (cx<R>*)(partial + (nparts > 1 ? nparts * ud : 0));
    const int nq = ud + kDenseChunk * nparts;
    return lanczos_core(ud, [&](const zd* qv, zd* wv) {
      for (int i = tid; i < nq; i += AMMSE_BLOCK)
        qs[i] = (i < ud) ? from_d<R>(qv[i]) : cx<R>{R(0), R(0)};
      __syncthreads();
      auto row = [&](int r, int part) __attribute__((always_inline)) {
        zd acc = {0.0, 0.0};
        for (int c0 = part; c0 < ud; c0 += kDenseChunk * nparts) {
          cx<R> kv[kDenseChunk];
#pragma unroll
          for (int u = 0; u < kDenseChunk; ++u)
            kv[u] = Kd[(long)min(c0 + u * nparts, ud - 1) * ud + r];
          if constexpr (sizeof(R) == 4) {
            float ax = 0.f, ay = 0.f, bx = 0.f, by = 0.f;
#pragma unroll
            for (int u = 0; u < kDenseChunk; u += 2) {   // conj(K(c, r)) q_c
              const cx<float> q0 = qs[c0 + u * nparts], q1 = qs[c0 + (u + 1) * nparts];
              ax = fmaf(kv[u].x, q0.x, fmaf(kv[u].y, q0.y, ax));
              ay = fmaf(kv[u].x, q0.y, fmaf(-kv[u].y, q0.x, ay));
              bx = fmaf(kv[u + 1].x, q1.x, fmaf(kv[u + 1].y, q1.y, bx));
              by = fmaf(kv[u + 1].x, q1.y, fmaf(-kv[u + 1].y, q1.x, by));
            }
            acc.x += (double)ax + (double)bx;
            acc.y += (double)ay + (double)by;
          } else {
#pragma unroll
            for (int u = 0; u < kDenseChunk; ++u) acc = acc + cj(kv[u]) * qs[c0 + u * nparts];
          }
        }
        return acc;
      };
      if (nparts == 1) {
        for (int r = tid; r < ud; r += AMMSE_BLOCK) wv[r] = row(r, 0);
        return;
      }
      const int r = tid % ud, part = tid / ud;
      if (part < nparts) partial[part * ud + r] = row(r, part);
      __syncthreads();
      for (int rr = tid; rr < ud; rr += AMMSE_BLOCK) {
        zd acc = {0.0, 0.0};
        for (int q = 0; q < nparts; ++q) acc = acc + partial[q * ud + rr];
        wv[rr] = acc;
      }
    });
  };

  // Single cell with U N <= M: the same lambda_max on the (U N)-dimensional
  // matrix K = C^H Q C (D = C C^H per user, Q = S H H^H S formed once per
  // solve), formed per call; each Lanczos step reads it once.
  auto lanczos_q = [&]() __attribute__((always_inline)) {
    kq_form<R>(Qm, Cm, Kq, U, N, phase_tid());
    __syncthreads();
    return lanczos_dense(Kq, un);
  };

  // The iterate V^t is kept as scur_c * Xc (per BS c) and V^{t-1} as
  // sprev_c * Xp; Xc and Xp rotate between the caller's V and the workspace
  // copy Vq.
  cx<R>* Xc = V;
  cx<R>* Xp = Vq;

  // ---- WMMSE V step (Algorithm 2, Section IV): per BS c,
  //   A_c = H_c^H S D S H_c over all users, B_c = H_c^H S Y on the columns of
  //   the BS's own users (D, Y of the second stage: W = E^{-1}),
  //   V_c = (A_c + mu I)^{-1} B_c with mu = 0 if the minimum-norm minimiser
  //   meets the budget, else the root of ||V_c(mu)||^2 = P_c.
  // With D = C C^H per user, A_c = R^H R and B_c = R^H Z for R = C^H S H_c
  // ((U d) x M) and Z = sqrt(alpha) Lw^H on the own users' blocks, so
  //   V_c(mu) = R^H (K + mu I)^{-1} Z,  K = R R^H  ((U d) x (U d)).
  // When U d <= M this stream-space form is used: K is then generically
  // nonsingular, mu = 0 gives the minimum-norm (pseudo-inverse) minimiser
  // even though A_c is singular, and the factorised matrix is the smaller
  // one.  Otherwise A_c (M x M, generically nonsingular) is factorised.
  // The root is found by safeguarded Newton steps on 1/||V_c(mu)|| inside a
  // bisection bracket; the factorisations and solves are in double.
  // Lm = Cholesky factor (lower) of Am + mu I (n x n); false when not positive
  // definite.  Lm and the solution block Y below live in LDS or in global
  // memory; the helpers are inlined into one copy of the solve per case, so
  // each access uses its own address space.
  auto wm_chol = [&](int n, double mu_, auto* Lm) __attribute__((always_inline)) -> bool {
    const int tid = phase_tid();
    const int tx = tid & 15, ty = tid >> 4;
    for (int i = ty; i < n; i += 16)
      for (int j = tx; j <= i; j += 16) {
        zd a = Am[i * n + j];
        if (i == j) a = {a.x + mu_, 0.0};
        Lm[i * n + j] = a;
      }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      const double dkk = Lm[k * n + k].x;
      if (!(dkk > 0.0) || !isfinite(dkk)) {
        __syncthreads();
        return false;
      }
      const double lkk = sqrt(dkk), il = 1.0 / lkk;
      for (int i = k + 1 + tid; i < n; i += AMMSE_BLOCK) Lm[i * n + k] = scal(il, Lm[i * n + k]);
      __syncthreads();
      if (tid == 0) Lm[k * n + k] = {lkk, 0.0};
      for (int i = k + 1 + ty; i < n; i += 16) {
        const zd lik = Lm[i * n + k];
        for (int j = k + 1 + tx; j <= i; j += 16)
          Lm[i * n + j] = Lm[i * n + j] - mulc(lik, Lm[j * n + k]);
      }
      __syncthreads();
    }
    return true;
  };
  // Triangular solves on the nc columns of a row-major n x nc block: four
  // threads per column, thread q of a column owning the rows i = q (mod 4);
  // the partial sums meet by shuffles, so no barrier is needed inside.
  // Y <- L^{-1} Y (conjT = false) or L^{-H} Y (conjT = true), in place.
  auto wm_trsm = [&](auto* Y, int n, int nc, bool conjT, const auto* Lm)
      __attribute__((always_inline)) {
    const int tid = phase_tid();
    const int q = tid & 3;
    for (int j0 = 0; j0 < nc; j0 += AMMSE_BLOCK / 4) {
      const int j = j0 + (tid >> 2);
      const bool act = j < nc;
      const int jj = act ? j : nc - 1;
      for (int s = 0; s < n; ++s) {
        const int k = conjT ? n - 1 - s : s;
        zd part = {0.0, 0.0};
        if (!conjT) {
#pragma unroll 4
          for (int i = q; i < k; i += 4) part = part + Lm[k * n + i] * Y[i * nc + jj];
        } else {
#pragma unroll 4
          for (int i = k + 1 + ((q - (k + 1)) & 3); i < n; i += 4)
            part = part + cj(Lm[i * n + k]) * Y[i * nc + jj];
        }
        part.x += __shfl_xor(part.x, 1, 64);
        part.y += __shfl_xor(part.y, 1, 64);
        part.x += __shfl_xor(part.x, 2, 64);
        part.y += __shfl_xor(part.y, 2, 64);
        const zd yk = scal(1.0 / Lm[k * n + k].x, Y[k * nc + jj] - part);
        if (act && q == (k & 3)) Y[k * nc + jj] = yk;
      }
    }
    __syncthreads();
  };
  auto wm_norm2 = [&](const auto* Y, int n) __attribute__((always_inline)) {
    const int tid = phase_tid();
    double v = 0.0;
    for (int e = tid; e < n; e += AMMSE_BLOCK) v += nrm2(Y[e]);
    return block_sum(v, sm.red);
  };
  // Probe mu: X = (Am + mu I)^{-1} Bm (n x nc) and q = ||V(mu)||^2 with V = X
  // (antenna space) or V = R^H X (stream space).  In stream space
  // ||V||^2 = ||L^{-1} Z||^2 - mu ||X||^2 is used when its rounding error
  // (about 1e-16 of the two terms) is below 1e-11 of the result; otherwise
  // (a switched-off stream makes K singular and mu tiny) V is formed.
  // Returns false if Am + mu I is not positive definite.
  auto wm_probe = [&](int n, int nc, bool sspace, double mu_, double& q, auto* Lf, auto* Xf)
      __attribute__((always_inline)) -> bool {
    const int tid = phase_tid();
    if (!wm_chol(n, mu_, Lf)) return false;
    for (int e = tid; e < n * nc; e += AMMSE_BLOCK) Xf[e] = Bm[e];
    __syncthreads();
    wm_trsm(Xf, n, nc, false, Lf);
    const double yy = sspace ? wm_norm2(Xf, n * nc) : 0.0;
    wm_trsm(Xf, n, nc, true, Lf);
    const double xx = wm_norm2(Xf, n * nc);
    if (!sspace) {
      q = xx;
    } else if (yy - mu_ * xx > 1e-5 * (yy + mu_ * xx)) {
      q = yy - mu_ * xx;
    } else {
      double v = 0.0;
      for (int e = tid; e < M * nc; e += AMMSE_BLOCK) {
        const int m = e / nc, j = e - m * nc;
        zd acc = {0.0, 0.0};
#pragma unroll 4
        for (int k = 0; k < n; ++k) acc = acc + cj(Tm[(long)k * M + m]) * Xf[k * nc + j];
        v += nrm2(acc);
      }
      q = block_sum(v, sm.red);
    }
    return true;
  };
  auto wmmse_step = [&](bool stage2) {
    const int tid = phase_tid();
    const int nsd = U * d;
    const bool sspace = nsd <= M;
    const int n = sspace ? nsd : M;
    for (int c = 0; c < C; ++c) {
      const int nc = sm.cu[c] * d;
      if (nc == 0) continue;
      const cx<R>* Hc = H + (long)c * un * M;
      int u0 = 0;
      while (u0 < U && sm.cellOf[u0] != c) ++u0;
      if (sspace) {
        // R = C^H S H_c, one thread per (user, antenna)
        for (int e = tid; e < U * M; e += AMMSE_BLOCK) {
          const int u = e / M, m = e - u * M;
          zd h[AMMSE_MAX_RX];
#pragma unroll
          for (int k = 0; k < AMMSE_MAX_RX; ++k)
            h[k] = (k < N) ? scal(sm.invsig[u], to_d(Hc[(long)(u * N + k) * M + m]))
                           : zd{0.0, 0.0};
          for (int s_ = 0; s_ < d; ++s_) {
            zd r = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < AMMSE_MAX_RX; ++k)
              if (k < N) r = r + cj(Cm[u * 16 + k * 4 + s_]) * h[k];
            Tm[(long)(u * d + s_) * M + m] = r;
          }
        }
        // Z: sqrt(alpha_u) Lw_u^H (stage II) or sqrt(alpha_u) I (stage I) on the
        // own users' diagonal blocks
        for (int e = tid; e < nsd * nc; e += AMMSE_BLOCK) {
          const int i = e / nc, j = e - (e / nc) * nc;
          const int u = i / d, s_ = i - u * d, ul = u - u0, t_ = j - (j / d) * d;
          zd z = {0.0, 0.0};
          if (ul >= 0 && ul < sm.cu[c] && j / d == ul)
            z = stage2 ? scal(sqrt(sm.alpha[u]), cj(Lwm[u * 16 + t_ * 4 + s_]))
                       : zd{(s_ == t_) ? sqrt(sm.alpha[u]) : 0.0, 0.0};
          Bm[e] = z;
        }
        __syncthreads();
        // K = R R^H
        for (int e = tid; e < nsd * nsd; e += AMMSE_BLOCK) {
          const int i = e / nsd, j = e - i * nsd;
          const zd* ri = Tm + (long)i * M;
          const zd* rj = Tm + (long)j * M;
          zd acc = {0.0, 0.0};
          for (int m = 0; m < M; ++m) acc = acc + mulc(ri[m], rj[m]);
          Am[e] = acc;
        }
      } else {
        // T = S D S H_c: one thread per (user, antenna), N rows each
        for (int e = tid; e < U * M; e += AMMSE_BLOCK) {
          const int u = e / M, m = e - u * M;
          const double s2 = sm.invsig[u] * sm.invsig[u];
          zd h[AMMSE_MAX_RX];
#pragma unroll
          for (int k = 0; k < AMMSE_MAX_RX; ++k)
            h[k] = (k < N) ? to_d(Hc[(long)(u * N + k) * M + m]) : zd{0.0, 0.0};
#pragma unroll
          for (int nn = 0; nn < AMMSE_MAX_RX; ++nn) {
            if (nn < N) {
              zd acc = {0.0, 0.0};
#pragma unroll
              for (int k = 0; k < AMMSE_MAX_RX; ++k)
                if (k < N) acc = acc + Dm[u * 16 + nn * 4 + k] * h[k];
              Tm[(long)(u * N + nn) * M + m] = scal(s2, acc);
            }
          }
        }
        // B_c[m][j] = sum_n conj(H[uN+n][m]) (1/sigma_u) Y_u[n][s], j = local user * d + s
        for (int e = tid; e < M * nc; e += AMMSE_BLOCK) {
          const int m = e / nc, j = e - m * nc;
          const int u = u0 + j / d, s_ = j - (j / d) * d;
          zd acc = {0.0, 0.0};
          for (int nn = 0; nn < N; ++nn)
            acc = acc + cj(to_d(Hc[(long)(u * N + nn) * M + m])) * Ym[u * 16 + nn * 4 + s_];
          Bm[e] = scal(sm.invsig[u], acc);
        }
        __syncthreads();
        // A_c = H_c^H T
        for (int e = tid; e < M * M; e += AMMSE_BLOCK) {
          const int i = e / M, j = e - i * M;
          zd acc = {0.0, 0.0};
          for (int r = 0; r < un; ++r)
            acc = acc + cj(to_d(Hc[(long)r * M + i])) * Tm[(long)r * M + j];
          Am[e] = acc;
        }
      }
      __syncthreads();
      // where=0: factor and solution in LDS, 1: factor in LDS, 2: both global
      auto solve_with = [&](auto where) __attribute__((always_inline)) {
        zd* Lf;
        zd* Xf;
        if constexpr (decltype(where)::value == 0) {
          Lf = (zd*)dyn_lds;
          Xf = (zd*)dyn_lds + 64 * 64;
        } else if constexpr (decltype(where)::value == 1) {
          Lf = (zd*)dyn_lds;
          Xf = Xm;
        } else {
          Lf = Lm;
          Xf = Xm;
        }
        const double Pc = sm.Pc[c];
        double q = 0.0;
        if (!(Pc > 0.0)) {
          for (int e = tid; e < n * nc; e += AMMSE_BLOCK) Xf[e] = {0.0, 0.0};
          __syncthreads();
        } else {
          // Root of phi(mu) = 1/||V(mu)|| - 1/sqrt(P) (increasing, nearly linear
          // in mu) by secant steps through the last two probes, kept inside the
          // bracket [lo, hi]; bisection (geometric once lo > 0) when a step
          // leaves the bracket or the bracket stops halving.
          const double sP = sqrt(Pc);
          bool ok = wm_probe(n, nc, sspace, 0.0, q, Lf, Xf);
          double mu_ = 0.0;
          if (!ok || q > Pc) {
            double lo = 0.0, hi;
            if (sspace) {
              // ||B_c||^2 = ||R^H Z||^2 <= ||K||_F ||Z||_F^2 and ||V(mu)|| <= ||B_c|| / mu
              hi = sqrt(sqrt(wm_norm2(Am, n * n)) * wm_norm2(Bm, n * nc) / Pc);
            } else {
              hi = sqrt(wm_norm2(Bm, n * nc) / Pc);
            }
            bool have_a = ok && q > 0.0;
            double mu_a = 0.0, ph_a = have_a ? 1.0 / sqrt(q) - 1.0 / sP : 0.0;
            double next = (sm.mu[c] > 0.0 && sm.mu[c] < hi) ? sm.mu[c] : 0.5 * hi;
            double wref = hi - lo;
            int since = 0;
            for (int probe = 0; probe < 100; ++probe) {
              double mid = (lo > 0.0) ? sqrt(lo * hi) : 0.5 * (lo + hi);
              if (!(next > lo && next < hi)) next = mid;
              mu_ = next;
              ok = wm_probe(n, nc, sspace, mu_, q, Lf, Xf);
              if (!ok) {
                lo = mu_;
                next = sqrt(lo * hi);
                have_a = false;
                continue;
              }
              if (q > Pc) lo = mu_;
              else hi = mu_;
              if (fabs(sqrt(q) - sP) <= 1e-13 * sP || hi - lo <= 1e-13 * hi) break;
              const double ph = (q > 0.0) ? 1.0 / sqrt(q) - 1.0 / sP : 1e300;
              mid = (lo > 0.0) ? sqrt(lo * hi) : 0.5 * (lo + hi);
              next = (have_a && ph != ph_a) ? mu_ - ph * (mu_ - mu_a) / (ph - ph_a) : mid;
              have_a = true;
              mu_a = mu_;
              ph_a = ph;
              if (++since >= 3) {
                if (hi - lo > 0.5 * wref) next = mid;
                wref = hi - lo;
                since = 0;
              }
            }
            if (!ok) atomicOr(&sm.fail, AMMSE_INST_CHOLESKY);
          }
          if (tid == 0) sm.mu[c] = mu_;
        }
        cx<R>* Vc = Xc + (long)M * sm.colOff[c];
        if (sspace) {   // V_c = R^H X
          for (int e = tid; e < M * nc; e += AMMSE_BLOCK) {
            const int m = e / nc, j = e - m * nc;
            zd acc = {0.0, 0.0};
  #pragma unroll 4
            for (int k = 0; k < nsd; ++k) acc = acc + cj(Tm[(long)k * M + m]) * Xf[k * nc + j];
            Vc[e] = from_d<R>(acc);
          }
        } else {
          for (int e = tid; e < M * nc; e += AMMSE_BLOCK) Vc[e] = from_d<R>(Xf[e]);
        }
      };
      if (p.lds_factor >= 2 && n <= 64 && nc <= 64) solve_with(std::integral_constant<int, 0>{});
      else if (p.lds_factor >= 1 && n <= 64) solve_with(std::integral_constant<int, 1>{});
      else solve_with(std::integral_constant<int, 2>{});
      __syncthreads();
    }
  };

  // ---- initial state.
  for (int c = tid; c < C; c += AMMSE_BLOCK) {
    sm.scur[c] = 1.0;
    sm.sprev[c] = 1.0;
    sm.mu[c] = 0.0;
  }
  __syncthreads();
  if (qpath && !p.wsr_only) {   // Q = S H H^H S (float products), made exactly Hermitian
    channel_gemm<R, false, true>(un, un, M, H, M, H, M, sm.tiles, false, tile,
                                 [&](int i, int j, cx<R> v) {
                                   const R f = (R)(sm.invsig[i / N] * sm.invsig[j / N]);
                                   Qm[(long)i * un + j] = {f * v.x, f * v.y};
                                 });
    __syncthreads();
    for (int e = tid; e < un * un; e += AMMSE_BLOCK) {
      const int i = e / un, j = e - i * un;
      if (i < j) {
        const cx<R> x = Qm[e], y = Qm[(long)j * un + i];
        const cx<R> mm = {R(0.5) * (x.x + y.x), R(0.5) * (x.y - y.y)};
        Qm[e] = mm;
        Qm[(long)j * un + i] = {mm.x, -mm.y};
      } else if (i == j) {
        Qm[e].y = R(0);
      }
    }
    __syncthreads();
  }
  if constexpr (sizeof(R) == 4) {
    if (copies) {   // bfloat16 copies of H and V^0 (rounded as the products would round them)
      const long nh = (long)C * un * M;
      for (long e = tid; e < nh; e += AMMSE_BLOCK) Hb[e] = to_bfc(H[e]);
      for (long e = tid; e < Vtot; e += AMMSE_BLOCK) Xb[e] = to_bfc(Xc[e]);
      __syncthreads();
    }
  }
  // G^0 (on the Q path it enters every iteration's G and projection norm, so it
  // is formed with float products there)
  channel_product(Gp, Xc, sm.scur, p.lowp_iters >= 1 && !rpath);
  __syncthreads();
  const int T = p.wsr_only ? 0 : p.max_iters;
  // Q recursion state: V^t = c_t V^0 + H^H S (xs_t X_t), G buffers carry
  // scales gsp (G^{t-1}) and gsq (G^{t-2}) applied where they are read
  double c1 = 1.0, c2 = 1.0, xs1 = 1.0, xs2 = 1.0, gsp = 1.0, gsq = 1.0, nu = 0.0;
  if (!p.wsr_only) {
    const int nv = (int)Vtot, ng = un * D.ud;
    if (rpath) {
      for (int e = tid; e < nv; e += AMMSE_BLOCK) nu += nrm2(to_d(Xc[e]));
#pragma unroll 4
      for (int e = tid; e < ng; e += AMMSE_BLOCK) {
        const cx<R> g = Gp[e];
        Gq[e] = g;
        G0[e] = g;
        X1[e] = cx<R>{(R)0, (R)0};
        X2[e] = cx<R>{(R)0, (R)0};
      }
      nu = block_sum(nu, sm.red);
    } else {
#pragma unroll 4
      for (int e = tid; e < nv; e += AMMSE_BLOCK) Xp[e] = Xc[e];
#pragma unroll 4
      for (int e = tid; e < ng; e += AMMSE_BLOCK) Gq[e] = Gp[e];
    }
  }
  __syncthreads();

  int fsw = p.force_switch_iter;
  if (p.force_switch && p.force_switch[b] > 0) fsw = p.force_switch[b];
  bool stage2 = p.algorithm == AMMSE_ALGO_WMMSE || bc ||
                ((fsw >= 1) ? (fsw <= 1) : (p.warm_start == 0));
  int switch_iter = stage2 ? 1 : -1;
  bool prev_step_stage2 = false;
  double wsr_prev = 0.0, wsr_prev2 = 0.0;   // WSR(V^{t-1}), WSR(V^{t-2})
  int iters_run = 0;
  int status = 0;
  bool have_bound = false;   // sm.gbound computed (once per solve, when first needed)
  // a given fixed step (gamma_c > 0): its value waits in LDS, so that no
  // register of the iteration loop holds it
  const bool fixed_gamma = p.gamma_c > 0.0;
  if (tid == 0) sm.gfix = p.gamma_c;
  __syncthreads();

  for (int t = 1; t <= T; ++t) {
    const bool lowp = t <= p.lowp_iters;   // bfloat16 products in this iteration
    if (p.lowp_iters >= 1 && t == p.lowp_iters + 1) {
      // refinement pass: G^{t-1} and G^{t-2} again with float products
      if (rpath) {   // G^{t-k} = c_{t-k} G^0 + Q (xs_k X_k), k = 1, 2 (scales folded in)
        const int ud = D.ud;
        channel_gemm<R, false>(un, ud, un, Qm, un, X1, ud, sm.tiles, false, tile,
                               [&](int i, int j, cx<R> pq) {
                                 const long e = (long)i * ud + j;
                                 const cx<R> g0 = G0[e];
                                 Gp[e] = from_d<R>(zd{c1 * (double)g0.x + xs1 * (double)pq.x,
                                                      c1 * (double)g0.y + xs1 * (double)pq.y});
                               });
        channel_gemm<R, false>(un, ud, un, Qm, un, X2, ud, sm.tiles, false, tile,
                               [&](int i, int j, cx<R> pq) {
                                 const long e = (long)i * ud + j;
                                 const cx<R> g0 = G0[e];
                                 Gq[e] = from_d<R>(zd{c2 * (double)g0.x + xs2 * (double)pq.x,
                                                      c2 * (double)g0.y + xs2 * (double)pq.y});
                               });
        gsp = 1.0;
        gsq = 1.0;
      } else {
        channel_product(Gp, Xc, sm.scur, false);
        channel_product(Gq, Xp, sm.sprev, false);
      }
      __syncthreads();
    }
    // receivers and rate of V^{t-1}
    const double rs = receivers(Gp, gsp, bc && t == 1);
    wsr_prev2 = wsr_prev;
    wsr_prev = wsr_sum(rs);
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
    // step size of this iteration: adaptive in the windows, otherwise fixed
    const bool adaptive = t <= p.T_c || (p.rearm && switch_iter >= 1 && t >= switch_iter &&
                                         t < switch_iter + p.T_c);
    const bool use_bound = !wm && stage2 && !adaptive && !fixed_gamma &&
                           p.step_rule == AMMSE_STEP_BOUND;
    if (use_bound && !have_bound && bgram && p.bound_pre) {
      // written by ammse_bound_gram_kernel (launched before this kernel)
      if (tid < C) sm.gbound[tid] = Gbw[tid];
      __syncthreads();
      have_bound = true;
    }
    if (use_bound && !have_bound) {
      // Lhat_c / 2 = lambda_max(H_c^H S diag(alpha) S H_c) by the step-size
      // Lanczos: on the Q path on K = C^H Q C with C = diag(sqrt(alpha)) (one
      // read of Q per step instead of two passes over H), otherwise on the
      // operator with D = alpha_u I (C and D are rewritten by the weights below)
      for (int e = tid; e < U * 16; e += AMMSE_BLOCK) {
        const int u = e >> 4, a = (e >> 2) & 3, bb = e & 3;
        const bool dg = a == bb && a < N;
        if (qpath) Cm[e] = dg ? zd{sqrt(sm.alpha[u]), 0.0} : zd{0.0, 0.0};
        else Dm[e] = dg ? zd{sm.alpha[u], 0.0} : zd{0.0, 0.0};
      }
      __syncthreads();
      for (int c = 0; c < C; ++c) {
        const double lm = (sm.cu[c] == 0) ? 0.0 : qpath ? lanczos_q() : lanczos_lmax(c);
        if (tid == 0) sm.gbound[c] = (lm > 0.0) ? 1.0 / (2.0 * lm) : 0.0;
        __syncthreads();
      }
      have_bound = true;
    }
    if (bc) bcgd_update(t == 1);
    else weights(stage2);

    if (wm) {   // Algorithm 2 / MMMSE: exact V minimiser, then G^t
      wmmse_step(stage2);
      {
        cx<R>* tmp = Gq;
        Gq = Gp;
        Gp = tmp;
      }
      channel_product(Gp, Xc, sm.scur, false);
      __syncthreads();
      prev_step_stage2 = stage2;
      iters_run = t;
      continue;
    }

    // step size
    if (adaptive) {
      // Gram path with order <= AMMSE_GRAM_WAVE_N: every K_c first (the whole
      // block on each), then one wave per BS runs its Lanczos iteration
      const int ng = (int)ammse_gram_order(U, M, d);
      const bool gw = gpath && ng <= AMMSE_GRAM_WAVE_N;
      for (int c = 0; c < C; ++c) {
        if (sm.cu[c] != 0 && gpath) gram_form(c, gw ? Kg + (long)c * ng * ng : Kg);
        if (gw) continue;
        const double lm = (sm.cu[c] == 0) ? 0.0
                          : qpath ? lanczos_q()
                          : gpath ? lanczos_dense(Kg, (int)ammse_gram_order(U, M, d))
                                  : lanczos_lmax(c);
        if (tid == 0) sm.gamma[c] = (lm > 0.0) ? 1.0 / (2.0 * lm) : 0.0;
        __syncthreads();
      }
      if constexpr (sizeof(R) == 4) {
        if (gw) {
          const int lane = tid & 63, wave = tid >> 6;
          float2* qs = (float2*)dyn_lds + wave * (AMMSE_GRAM_WAVE_N + 16);
          double2* tp = (double2*)((float2*)dyn_lds + 4 * (AMMSE_GRAM_WAVE_N + 16)) + wave * 64;
          for (int c = wave; c < C; c += AMMSE_BLOCK / 64) {
            const double lm = (sm.cu[c] == 0) ? 0.0
                              : wave_lanczos_lmax(Kg + (long)c * ng * ng, ng, p.lanczos_steps, qs, tp);
            if (lane == 0) sm.gamma[c] = (lm > 0.0) ? 1.0 / (2.0 * lm) : 0.0;
          }
          __syncthreads();
        }
      }
    } else if (fixed_gamma) {
      if (tid < C) sm.gamma[tid] = sm.gfix;
      __syncthreads();
    } else if (use_bound) {
      if (tid < C) sm.gamma[tid] = sm.gbound[tid];
      __syncthreads();
    }

    // Z = S (D G^ - Y), G^ = (1+w) G^{t-1} - w G^{t-2}: one thread per
    // (user, column), consecutive threads along the columns; the N rows of
    // the user's block of G^ are read once and give the N rows of Z.
    // Arithmetic in the storage precision's working type: float with float
    // storage (D and Y from their float copies), double otherwise.
    using T = typename std::conditional<sizeof(R) == 4, float, double>::type;
    const cx<T>* DmT;
    const cx<T>* YmT;
    if constexpr (sizeof(R) == 4) {
      DmT = Dmf;
      YmT = Ymf;
    } else {
      DmT = Dm;
      YmT = Ym;
    }
    const double om = p.extrapolate ? fmax((t - 2.0) / (t + 1.0), 0.0) : 0.0;
    const T ga1 = (T)((1.0 + om) * gsp), ga2 = (T)(om * gsq);
    const T xa1 = (T)((1.0 + om) * xs1), xa2 = (T)(om * xs2), gz = (T)(2.0 * sm.gamma[0]);
    // Compiled per N (the loop bounds fold); with float storage each thread
    // takes four (N <= 2) or two (user, column) elements per trip and issues
    // every load of them before the arithmetic, so that their latencies
    // overlap (one element with double storage, whose registers are the
    // tighter budget).
    auto zbuild = [&](auto nn) __attribute__((always_inline)) {
      constexpr int NN = decltype(nn)::value;
      // float storage with N <= 2: the users' D and Y blocks staged in LDS
      // (the product tiles, free here), read there in the arithmetic, so the
      // registers of their loads go to more elements per trip
      constexpr bool DL = sizeof(R) == 4 && NN <= 2 && QP != 0;
      cx<T>* Dl = (cx<T>*)sm.tiles;
      cx<T>* Yl = Dl + U * NN * NN;
      if constexpr (DL) {
        static_assert(!DL || 2 * AMMSE_MAX_USERS * 4 * sizeof(cx<float>) <= tile_bytes<R>(),
                      "the D and Y blocks fit the tile area");
        for (int e = tid; e < U * NN * NN; e += AMMSE_BLOCK) {
          const int u = e / (NN * NN), r = e - u * (NN * NN), n = r / NN, k = r - n * NN;
          Dl[e] = DmT[u * 16 + n * 4 + k];
          Yl[e] = YmT[u * 16 + n * 4 + k];
        }
        __syncthreads();
      }
      for (int c = 0; c < C; ++c) {
        const int nc = sm.cu[c] * d;
        const long base = (long)un * sm.colOff[c];
        const int ne = U * nc;
        const float rnc = 1.f / (float)max(nc, 1);
        constexpr int QB = sizeof(R) == 4 ? (NN <= 2 ? (DL ? 6 : 4) : 2) : 1;
        for (int e0 = tid; e0 < ne; e0 += QB * AMMSE_BLOCK) {
          int uq[QB], jq[QB];
          long gq0[QB];
          bool live[QB];
          cx<R> ga[QB][NN], gb[QB][NN], x1[QB][NN], x2[QB][NN];
          cx<T> dm[DL ? 1 : QB][NN][NN];
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            const int e = min(e0 + q * AMMSE_BLOCK, ne - 1);
            live[q] = e0 + q * AMMSE_BLOCK < ne;
            const int u = quot(e, rnc), j = e - u * nc;
            uq[q] = u;
            jq[q] = j;
            gq0[q] = base + (long)(u * NN) * nc + j;
            if (!live[q]) continue;   // (no loads for the trip's slots past the end)
#pragma unroll
            for (int k = 0; k < NN; ++k) {
              ga[q][k] = Gp[gq0[q] + (long)k * nc];
              gb[q][k] = Gq[gq0[q] + (long)k * nc];
              if (rpath) {
                x1[q][k] = X1[gq0[q] + (long)k * nc];
                x2[q][k] = X2[gq0[q] + (long)k * nc];
              }
            }
            if constexpr (!DL) {
#pragma unroll
              for (int n = 0; n < NN; ++n)
#pragma unroll
                for (int k = 0; k < NN; ++k) dm[q][n][k] = DmT[u * 16 + n * 4 + k];
            }
          }
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            const int u = uq[q], j = jq[q];
            cx<T> gh[NN];
#pragma unroll
            for (int k = 0; k < NN; ++k)
              gh[k] = {ga1 * (T)ga[q][k].x - ga2 * (T)gb[q][k].x,
                       ga1 * (T)ga[q][k].y - ga2 * (T)gb[q][k].y};
            const int j0 = sm.local[u] * d;
            const bool own = sm.cellOf[u] == c && j >= j0 && j < j0 + d;
            const T is = (T)sm.invsig[u];
            const int qd = DL ? 0 : q;
            if constexpr (DL) {
#pragma unroll
              for (int n = 0; n < NN; ++n)
#pragma unroll
                for (int k = 0; k < NN; ++k) dm[0][n][k] = Dl[(u * NN + n) * NN + k];
            }
#pragma unroll
            for (int n = 0; n < NN; ++n) {
              cx<T> acc = {T(0), T(0)};
#pragma unroll
              for (int k = 0; k < NN; ++k) acc = acc + dm[qd][n][k] * gh[k];
              if (own) acc = acc - (DL ? Yl[(u * NN + n) * NN + (j - j0)] : YmT[u * 16 + n * 4 + (j - j0)]);
              const long e = gq0[q] + (long)n * nc;
              if (!live[q]) continue;
              if (rpath) {
                // implicit precoder: Z' = D G^ - Y (the gradient is 2 H^H S Z'),
                // X~ = X^ - 2 gamma Z' over X^{t-2}
                X2[e] = cx<R>{(R)(xa1 * (T)x1[q][n].x - xa2 * (T)x2[q][n].x - gz * acc.x),
                              (R)(xa1 * (T)x1[q][n].y - xa2 * (T)x2[q][n].y - gz * acc.y)};
                continue;
              }
              const cx<R> zv = {(R)(is * acc.x), (R)(is * acc.y)};
              if constexpr (sizeof(R) == 4) {
                if (lowp && copies) {
                  Zb[e] = to_bfc(zv);
                  continue;
                }
              }
              Z[e] = zv;
            }
          }
        }
      }
    };
    switch (N) {
      case 1: zbuild(std::integral_constant<int, 1>{}); break;
      case 2: zbuild(std::integral_constant<int, 2>{}); break;
      case 3: zbuild(std::integral_constant<int, 3>{}); break;
      default: zbuild(std::integral_constant<int, 4>{}); break;
    }
    __syncthreads();

    if (rpath) {
      // One product P = Q X~ (single cell).  With V^t = c_t V^0 + H^H S X^t,
      // G^t = S H V^t = c_t G^0 + Q X^t, and X~ = X^ - 2 gamma Z' formed above:
      //   G~ = c~ G^0 + P,  ||V~||^2 = c~^2 ||V^0||^2 + 2 c~ Re<G^0, X~> + Re<X~, P>
      // (c~ = c^, the extrapolated coefficient); G~ goes over G^{t-2} and the
      // projection factor becomes the scale of G~ and X~.
      const int ud = D.ud;
      const double ch = (1.0 + om) * c1 - om * c2;
      QpathEpi<R> epi{X2, G0, Gq, ud, ch, 0.0};
      channel_gemm<R, false>(un, ud, un, Qm, un, X2, ud, sm.tiles, lowp, tile, epi);
      const double pw = ch * ch * nu + block_sum(epi.acc, sm.red);
      const double sc = (pw > sm.Pc[0]) ? sqrt(sm.Pc[0] / pw) : 1.0;
      cx<R>* tg = Gq;
      Gq = Gp;
      Gp = tg;
      gsq = gsp;
      gsp = sc;
      cx<R>* tx = X2;
      X2 = X1;
      X1 = tx;
      xs2 = xs1;
      xs1 = sc;
      c2 = c1;
      c1 = sc * ch;
      __syncthreads();
      prev_step_stage2 = stage2;
      iters_run = t;
      continue;
    }

    // gradient 2 H_c^H Z_c and, in the product's epilogue, the extrapolated
    // step X~ = (1+w) V^{t-1} - w V^{t-2} - gamma Grad written over V^{t-2};
    // then the projection factor of each BS from ||X~||^2.
    for (int c = 0; c < C; ++c) {
      const int nc = sm.cu[c] * d;
      if (nc == 0) continue;
      const long base = (long)M * sm.colOff[c];
      const cx<R>* __restrict__ xc = Xc + base;
      cx<R>* __restrict__ xp = Xp + base;
      const double a1 = (1.0 + om) * sm.scur[c], a2 = om * sm.sprev[c], g2 = 2.0 * sm.gamma[c];
      double pw = 0.0;
      bfc* __restrict__ xb = Xb + base;
      const bool bcopy = lowp && copies;
      auto epi = [&](int i, int j, cx<R> g) {
        const long e = (long)i * nc + j;
        const zd v = to_d(xc[e]), q = to_d(xp[e]);
        const cx<R> xs = from_d<R>(zd{a1 * v.x - a2 * q.x - g2 * (double)g.x,
                                      a1 * v.y - a2 * q.y - g2 * (double)g.y});
        xp[e] = xs;
        if constexpr (sizeof(R) == 4) {
          if (bcopy) xb[e] = to_bfc(xs);
        }
        pw += nrm2(to_d(xs));
      };
      bool done = false;
      if constexpr (sizeof(R) == 4) {
        if (bcopy) {
          channel_gemm_bf16<true>(M, nc, un, Hb + (long)c * un * M, M,
                                  Zb + (long)un * sm.colOff[c], nc, sm.tiles, tile, epi);
          done = true;
        }
      }
      if (!done)
        channel_gemm<R, true>(M, nc, un, H + (long)c * un * M, M, Z + (long)un * sm.colOff[c], nc,
                              sm.tiles, lowp, tile, epi);
      pw = block_sum(pw, sm.red);
      if (tid == 0) {
        sm.sprev[c] = sm.scur[c];
        sm.scur[c] = (pw > sm.Pc[c]) ? sqrt(sm.Pc[c] / pw) : 1.0;
      }
    }
    {
      cx<R>* tmp = Xc;
      Xc = Xp;
      Xp = tmp;
    }
    __syncthreads();

    // G^{t} = S H V^t ; keep G^{t-1}
    {
      cx<R>* tmp = Gq;
      Gq = Gp;
      Gp = tmp;
    }
    channel_product(Gp, Xc, sm.scur, lowp);
    __syncthreads();
    prev_step_stage2 = stage2;
    iters_run = t;
  }

  // ---- recursion path: V = c V^0 + H^H S (xs X) into the caller's buffer,
  // projected onto the power ball exactly, and G = S H V for its WSR
  if (rpath && !p.wsr_only) {
    const int ud = D.ud;
    __syncthreads();
    for (int e = tid; e < un * ud; e += AMMSE_BLOCK) {
      const int i = e / ud;
      const double f = xs1 * sm.invsig[i / N];
      const cx<R> x = X1[e];
      Z[e] = {(R)(f * x.x), (R)(f * x.y)};
    }
    __syncthreads();
    double pw = 0.0;
    channel_gemm<R, true>(M, ud, un, H, M, Z, ud, sm.tiles, false, tile,
                          [&](int i, int j, cx<R> v) {
                            const long e = (long)i * ud + j;
                            const cx<R> v0 = V[e];
                            const zd w = {c1 * (double)v0.x + (double)v.x,
                                          c1 * (double)v0.y + (double)v.y};
                            V[e] = from_d<R>(w);
                            pw += nrm2(w);
                          });
    pw = block_sum(pw, sm.red);
    if (pw > sm.Pc[0]) {
      const double sc = sqrt(sm.Pc[0] / pw);
      for (long e = tid; e < Vtot; e += AMMSE_BLOCK) {
        const cx<R> v = V[e];
        V[e] = {(R)(sc * v.x), (R)(sc * v.y)};
      }
    }
    __syncthreads();
    channel_product(Gp, V, sm.scur, false);
    gsp = 1.0;
    __syncthreads();
  }
  // ---- WSR of the returned precoders
  double wsr_final;
  if ((iters_run == T || rpath) && !status) {
    const double rs = receivers(Gp, gsp);
    wsr_final = wsr_sum(rs);
    if (sm.fail) status |= sm.fail;
    if (!isfinite(wsr_final)) status |= AMMSE_INST_NONFINITE;
    if (p.trace && tid == 0 && iters_run == T) p.trace[(long)b * p.trace_len + T] = wsr_final;
  } else {
    wsr_final = wsr_prev;   // stopped early: V^{iters_run} is the iterate, WSR already known
  }
  // V = scur X into the caller's buffer; zero-power check
  for (int c = 0; c < C; ++c) {
    const long base = (long)M * sm.colOff[c];
    const int n = M * sm.cu[c] * d;
    const double sc = sm.scur[c];
    double pw = 0.0;
    for (int e = tid; e < n; e += AMMSE_BLOCK) {
      const cx<R> v = Xc[base + e];
      if (!p.wsr_only) {
        const cx<R> o = from_d<R>(scal(sc, to_d(v)));
        V[base + e] = o;
        pw += nrm2(to_d(o));
      } else {
        pw += nrm2(to_d(v));
      }
    }
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

// Static plus dynamic LDS of one workgroup, as launched below.
size_t ammse_general_lds_bytes(int precision, int algorithm) {
  const bool f64 = precision == AMMSE_PREC_FP64;
  const size_t st = f64 ? sizeof(Smem<double>) : sizeof(Smem<float>);
  const bool exact_v = algorithm == AMMSE_ALGO_WMMSE || algorithm == AMMSE_ALGO_MMMSE;
  const size_t dyn = exact_v ? sizeof(zd) * 64 * 64 * (f64 ? 1 : 2)
                             : sizeof(zd) * 3 * AMMSE_LANCZOS_LDS_N;
  return st + dyn;
}

// Exact-V-step algorithms get 64 KiB of dynamic LDS for a factor of order <= 64
// (128 KiB with FP32 storage: factor and solution); A-MMMSE gets the area of
// the Lanczos vectors.
template <class R>
hipError_t launch_general(const ammse_kparams_t& p0, hipStream_t s) {
  ammse_kparams_t p = p0;
  // A-MMMSE: the Lanczos vectors (order <= AMMSE_LANCZOS_LDS_N)
  size_t dyn = sizeof(zd) * 3 * AMMSE_LANCZOS_LDS_N;
  if (p.algorithm == AMMSE_ALGO_WMMSE || p.algorithm == AMMSE_ALGO_MMMSE) {
    static bool attr_set = false;
    // FP32: factor and solution block (128 KiB); FP64 (larger static tiles): factor only
    dyn = sizeof(zd) * 64 * 64 * (sizeof(R) == 4 ? 2 : 1);
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute((const void*)ammse_solve_kernel<R, 0>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)ammse_solve_kernel<R, 1>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    p.lds_factor = sizeof(R) == 4 ? 2 : 1;
  } else {
    p.lds_factor = 0;
  }
  p.bound_pre = 0;
  p.block_base = 0;
  if constexpr (sizeof(R) == 4) {
    // the stage-II bound of the instances that ammse_bound_gram selects
    // (the kernel returns at once for the others)
    if ((p.algorithm == AMMSE_ALGO_AMMMSE || p.algorithm == AMMSE_ALGO_BCGD) && !p.wsr_only &&
        p.step_rule == AMMSE_STEP_BOUND && !(p.gamma_c > 0.0) && p.max_iters > p.T_c) {
      hipLaunchKernelGGL(ammse_bound_gram_kernel, dim3(p.batch), dim3(AMMSE_BLOCK), 0, s, p);
      p.bound_pre = 1;
    }
  }
  // the Q-path instances (launch positions [0, n_qp)), then the others
  if (p.n_qp > 0)
    hipLaunchKernelGGL((ammse_solve_kernel<R, 1>), dim3(p.n_qp), dim3(AMMSE_BLOCK), dyn, s, p);
  if (p.batch > p.n_qp) {
    p.block_base = p.n_qp;
    hipLaunchKernelGGL((ammse_solve_kernel<R, 0>), dim3(p.batch - p.n_qp), dim3(AMMSE_BLOCK), dyn,
                       s, p);
  }
  return hipGetLastError();
}

hipError_t ammse_launch_fp64(const ammse_kparams_t& p, hipStream_t s) {
  return launch_general<double>(p, s);
}

hipError_t ammse_launch_fp32(const ammse_kparams_t& p, hipStream_t s) {
  return launch_general<float>(p, s);
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free solve: a static device array (one copy per
// device), whose device address is looked up once per device with that device
// current.  Host code never passes the array's name to a kernel (in host code
// it is a host-side stand-in); it passes the looked-up address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[AMMSE_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t ammse_scratch_resolve(int device, void** ptr) {
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}
