// Unrolled A-MMMSE and its adjoint (reverse-mode derivative) for gfx950.
//
// The unrolled solver runs T iterations of Algorithm 3 on single-cell
// instances with the step size of each iteration given from outside
// (gamma_t, the learnable step sizes of an unrolled network), the stage
// switch by the eps1 rule (or forced), the extrapolation weight omega^t and
// the projection onto the sum-power ball; its output is V^T and WSR(V^T).
// The adjoint kernel returns dWSR/dgamma_t and dWSR/dH for an upstream
// weight per instance, with the switch iteration and the projection branch
// held fixed (they are piecewise constant).
//
// Memory: the forward writes (V^t, V^{t-1}) every K iterations to a
// checkpoint buffer.  The adjoint walks the segments backwards: it recomputes
// a segment's K iterations from its checkpoint with the same forward step
// (same code, same arithmetic) while keeping every intermediate in the
// workspace, then propagates the adjoints through them in reverse.
//
// Per iteration (single cell, S = diag(1/sigma_u), G = S H V):
//   receivers of G^{t-1} (J-, Cholesky, UW = J-^{-1} F, E = (I + F^H UW)^{-1})
//   D = alpha U W U^H, Y = alpha U W (stage I: W = I, stage II: W = E^{-1})
//   Z = S (D G^ - Y),  G^ = (1+w) G^{t-1} - w G^{t-2}
//   Grad = 2 H^H Z,  V~ = V^ - gamma_t Grad,  V^t = s V~ (s = min(1, sqrt(P/||V~||^2)))
// Adjoints use the convention dL = Re sum(conj(Xbar) dX) for complex X.
// The per-user derivative relations (all matrices N x N or N x d):
//   WSR = sum alpha_u (log det(I + G_u G_u^H) - log det J-_u) / ln 2, so
//     dWSR/dG_u = -(2 alpha_u / ln 2) (UW E UW^H G_u - UW on the own columns);
//   stage II: UWbar = alpha (Dbar + Dbar^H) UW E + alpha Ybar, Ebar = alpha UW^H Dbar UW;
//   stage I (T = UW E): Tbar = alpha (Dbar + Dbar^H) T + alpha Ybar,
//     UWbar = Tbar E, Ebar = UW^H Tbar;
//   Xbar = -E Ebar E (E = X^{-1}, X = I + F^H UW);
//   Fbar = UW Xbar^H + J-^{-1} (UWbar + F Xbar),
//   J-bar = -J-^{-1} (UWbar + F Xbar) UW^H;
//   Gbar_u on the other streams' columns += (J-bar + J-bar^H) G_u, on the own columns += Fbar.

#include <math.h>

#include "ammse_internal.h"

#include "ammse_device.h"
#include "ammse_gemm.h"

namespace {
using namespace ammse_dev;

__device__ __forceinline__ int utid() {
  int x = threadIdx.x;
  asm volatile("" : "+v"(x));
  return x;
}

// Elementwise pass over n entries: each thread takes entries e = tid + 256 q
// in trips of QB, with ld(e) (loads only) for every entry of a trip before
// st(e, loaded) (arithmetic and stores), so that a trip's loads are in flight
// together instead of each waiting for the previous entry's stores.  An
// entry's st touches only that entry's own locations.
template <int QB, class Ld, class St>
__device__ __forceinline__ void u_batched(int n, Ld&& ld, St&& st) {
  const int tid = utid();
  using L = decltype(ld(0));
  for (int e0 = tid; e0 < n; e0 += QB * AMMSE_BLOCK) {
    L v[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) v[q] = ld(min(e0 + q * AMMSE_BLOCK, n - 1));
#pragma unroll
    for (int q = 0; q < QB; ++q)
      if (e0 + q * AMMSE_BLOCK < n) st(e0 + q * AMMSE_BLOCK, v[q]);
  }
}

template <class R>
struct USmem {
  alignas(16) char tiles[tile_bytes<R>()];
  double invsig[AMMSE_MAX_USERS];
  double alpha[AMMSE_MAX_USERS];
  double red[16];
  double sp[2];
  int fail;
};

// Views of one instance's workspace (see ammse_unroll_layout).
template <class R>
struct UView {
  int U, M, N, d, un, ud, K;
  double P;
  const cx<R>* H;
  cx<R>* Vs;    // (K+2) x M x ud: V^{t0-1}, V^{t0}, ..., V^{t0+K}
  cx<R>* Gs;    // (K+2) x un x ud
  cx<R>* Zs;    // K x un x ud
  cx<R>* Grs;   // K x M x ud  (Grad_t)
  cx<R>* Vts;   // K x M x ud  (V~_t)
  double* sp;   // K x 2       (s_t, ||V~_t||^2)
  zd* UWs;      // K x U x 16
  zd* Es;
  zd* Los;      // Cholesky factor of J-
  zd* Ds;
  zd* Ys;
  cx<R>* Vb;    // 3 x M x ud  adjoint ring, slot t mod 3
  cx<R>* Gb;    // 3 x un x ud
  cx<R>* Zb;    // un x ud
  cx<R>* Tb;    // M x ud
  zd* Pa;       // U x 16 per-user adjoint blocks (Dbar, then Jbar + Jbar^H)
  zd* Pb;       // U x 16 (Ybar, then Fbar)
  size_t v, g;  // elements of one V / G matrix
  float rud, rN;  // 1 / (U d) and 1 / N (quotients by quot)
};

template <class R>
__device__ UView<R> make_view(const ammse_desc_t& D, const ammse_kparams_t& p,
                              const ammse_unroll_params_t& q) {
  const int K = q.ckpt_every;
  UView<R> w;
  w.U = D.U;
  w.M = D.M;
  w.N = D.N;
  w.d = D.d;
  w.un = D.un;
  w.ud = D.ud;
  w.K = K;
  w.P = p.P[D.bs_off];
  w.H = (const cx<R>*)p.H + D.h_off;
  const ammse_unroll_layout_t L = ammse_unroll_layout((int)sizeof(R), D.U, D.M, D.N, D.d, K);
  char* ws = p.ws + (size_t)blockIdx.x * q.ws_stride;
  w.Vs = (cx<R>*)(ws + L.Vs);
  w.Gs = (cx<R>*)(ws + L.Gs);
  w.Zs = (cx<R>*)(ws + L.Zs);
  w.Grs = (cx<R>*)(ws + L.Grs);
  w.Vts = (cx<R>*)(ws + L.Vts);
  w.sp = (double*)(ws + L.sp);
  w.UWs = (zd*)(ws + L.UWs);
  w.Es = (zd*)(ws + L.Es);
  w.Los = (zd*)(ws + L.Los);
  w.Ds = (zd*)(ws + L.Ds);
  w.Ys = (zd*)(ws + L.Ys);
  w.Vb = (cx<R>*)(ws + L.Vb);
  w.Gb = (cx<R>*)(ws + L.Gb);
  w.Zb = (cx<R>*)(ws + L.Zb);
  w.Tb = (cx<R>*)(ws + L.Tb);
  w.Pa = (zd*)(ws + L.Pa);
  w.Pb = (zd*)(ws + L.Pb);
  w.v = (size_t)D.M * D.ud;
  w.g = (size_t)D.un * D.ud;
  w.rud = 1.f / (float)D.ud;
  w.rN = 1.f / (float)D.N;
  return w;
}

// G = S H V
template <class R>
__device__ void u_product(const UView<R>& w, USmem<R>& sm, cx<R>* G, const cx<R>* V) {
  const int N = w.N, ud = w.ud;
  channel_gemm64<R, false>(w.un, ud, w.M, w.H, w.M, V, ud, sm.tiles,
                         [&](int i, int j, cx<R> v) {
                           const R f = (R)sm.invsig[quot(i, w.rN)];
                           G[(long)i * ud + j] = {f * v.x, f * v.y};
                         });
}

// J- of user u on the 16 lanes of a group (lane 4a + b ends with entry (a, b)),
// from the columns of the other users' streams of G.
template <class R>
__device__ zd u_interference(const UView<R>& w, const cx<R>* G, int uu, int li) {
  const int N = w.N, d = w.d, ud = w.ud, j0 = uu * d;
  zd sj[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) sj[q] = {0.0, 0.0};
  const cx<R>* __restrict__ r0 = G + (long)(uu * N) * ud;
  // the lane's columns j = li (mod 16) in chunks of CH, the loads of a chunk
  // issued together
  constexpr int CH = 4;
  for (int jc = li; jc < ud; jc += 16 * CH) {
    cx<R> gl[CH][AMMSE_MAX_RX];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int j = min(jc + 16 * c, ud - 1);
#pragma unroll
      for (int k = 0; k < AMMSE_MAX_RX; ++k) gl[c][k] = r0[(long)min(k, N - 1) * ud + j];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int j = jc + 16 * c;
      if (j >= ud || (j >= j0 && j < j0 + d)) continue;
      zd g[AMMSE_MAX_RX];
#pragma unroll
      for (int k = 0; k < AMMSE_MAX_RX; ++k) g[k] = (k < N) ? to_d(gl[c][k]) : zd{0.0, 0.0};
#pragma unroll
      for (int x = 0; x < AMMSE_MAX_RX; ++x)
#pragma unroll
        for (int y = 0; y < AMMSE_MAX_RX; ++y)
          if (x < N && y < N) sj[x * 4 + y] = sj[x * 4 + y] + mulc(g[x], g[y]);
    }
  }
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    const int bit = 8 >> step;
    const bool hi = (li & bit) != 0;
#pragma unroll
    for (int q = 0; q < bit; ++q) {
      const zd send = hi ? sj[q] : sj[q + bit];
      const zd keep = hi ? sj[q + bit] : sj[q];
      sj[q] = keep + zd{__shfl_xor(send.x, bit, 64), __shfl_xor(send.y, bit, 64)};
    }
  }
  const int a = li >> 2, b = li & 3;
  zd J = {(a == b) ? 1.0 : 0.0, 0.0};
  if (a < N && b < N) J = J + sj[0];
  return J;
}

// Receivers of all users from G: UW, E and the Cholesky factor of J- per user;
// returns this thread's share of sum alpha_u R_u (nats).
template <class R>
__device__ double u_receivers(const UView<R>& w, USmem<R>& sm, const cx<R>* G, zd* UWo, zd* Eo,
                              zd* Loo) {
  const int tid = utid();
  const int lane = tid & 63, li = lane & 15;
  const Lane4 L4{lane & ~15, li >> 2, li & 3};
  const int N = w.N, d = w.d, ud = w.ud, U = w.U;
  double rsum = 0.0;
  bool ok = true;
  for (int u0 = 0; u0 < U; u0 += AMMSE_BLOCK / 16) {
    const int u = u0 + (tid >> 4);
    const bool act = u < U;
    const int uu = act ? u : U - 1;
    const zd J = u_interference(w, G, uu, li);
    zd F = {0.0, 0.0};
    if (L4.a < N && L4.b < d) F = to_d(G[(long)(uu * N + L4.a) * ud + uu * d + L4.b]);
    bool oku = true;
    double io[4], iw[4];                        // reciprocal diagonals of the factors
    const zd Lo = chol16(L4, J, oku, io);
    F = trsm16(L4, Lo, io, F);
    zd X = mm_hn(L4, F, F);
    if (L4.a == L4.b) X = {X.x + 1.0, 0.0};
    const zd UWv = trsm16h(L4, Lo, io, F);
    const zd Lw = chol16(L4, X, oku, iw);
    const zd Li = trsm16(L4, Lw, iw, zd{(L4.a == L4.b) ? 1.0 : 0.0, 0.0});
    const zd Ev = mm_hn(L4, Li, Li);
    if (act) {
      if (L4.a == L4.b) rsum += sm.alpha[u] * 2.0 * log(Lw.x);
      UWo[u * 16 + li] = UWv;
      Eo[u * 16 + li] = Ev;
      Loo[u * 16 + li] = Lo;
      ok = ok && oku;
    }
  }
  if (!ok) atomicOr(&sm.fail, AMMSE_INST_CHOLESKY);
  return rsum;
}

// D = alpha U W U^H, Y = alpha U W per user (stage I: W = I, U = UW E).
template <class R>
__device__ void u_weights(const UView<R>& w, USmem<R>& sm, const zd* UWi, const zd* Ei, bool stage2,
                          zd* Do, zd* Yo) {
  const int tid = utid();
  const int lane = tid & 63, li = lane & 15;
  const Lane4 L4{lane & ~15, li >> 2, li & 3};
  for (int u0 = 0; u0 < w.U; u0 += AMMSE_BLOCK / 16) {
    const int u = u0 + (tid >> 4);
    const bool act = u < w.U;
    const int uu = act ? u : w.U - 1;
    const zd UWv = UWi[uu * 16 + li], Ev = Ei[uu * 16 + li];
    const zd T = mm_nn(L4, UWv, Ev);
    const zd Ur = stage2 ? UWv : T;
    zd Dv = mm_nh(L4, T, Ur);
    const zd Dt = L4.at(Dv, L4.b, L4.a);
    Dv = {0.5 * (Dv.x + Dt.x), 0.5 * (Dv.y - Dt.y)};
    const double al = sm.alpha[uu];
    if (act) {
      Do[u * 16 + li] = scal(al, Dv);
      Yo[u * 16 + li] = scal(al, Ur);
    }
  }
  __syncthreads();
}

// One forward iteration t from V^{t-1} (Vp), V^{t-2} (Vq), G^{t-1} (Gp),
// G^{t-2} (Gq) and the receivers' UW, E of G^{t-1}: Z, Grad, V~, (s, p),
// V^t (Vn) and G^t (Gn).
template <class R>
__device__ void u_step(const UView<R>& w, USmem<R>& sm, int t, double gamma, bool stage2,
                       bool extrapolate, const cx<R>* Vp, const cx<R>* Vq, const cx<R>* Gp,
                       const cx<R>* Gq, const zd* UWi, const zd* Ei, zd* Do, zd* Yo, cx<R>* Z,
                       cx<R>* Gr, cx<R>* Vt, double* spo, cx<R>* Vn, cx<R>* Gn) {
  const int tid = utid();
  const int N = w.N, d = w.d, ud = w.ud, U = w.U, M = w.M;
  u_weights(w, sm, UWi, Ei, stage2, Do, Yo);
  const double om = extrapolate ? fmax((t - 2.0) / (t + 1.0), 0.0) : 0.0;
  {
    struct LZ {
      cx<R> a[AMMSE_MAX_RX], q[AMMSE_MAX_RX];
    };
    auto ld = [&](int e) {
      const int u = quot(e, w.rud), j = e - u * ud;
      const long g0 = (long)(u * N) * ud + j;
      LZ l;
#pragma unroll
      for (int k = 0; k < AMMSE_MAX_RX; ++k) {
        const long o = g0 + (long)min(k, N - 1) * ud;
        l.a[k] = Gp[o];
        l.q[k] = Gq[o];
      }
      return l;
    };
    u_batched<2>(U * ud, ld, [&](int e, const LZ& l) {
      const int u = quot(e, w.rud), j = e - u * ud;
      const long g0 = (long)(u * N) * ud + j;
      zd gh[AMMSE_MAX_RX];
#pragma unroll
      for (int k = 0; k < AMMSE_MAX_RX; ++k)
        gh[k] = (k < N) ? zd{(1.0 + om) * (double)l.a[k].x - om * (double)l.q[k].x,
                             (1.0 + om) * (double)l.a[k].y - om * (double)l.q[k].y}
                        : zd{0.0, 0.0};
      const int j0 = u * d;
      const bool own = j >= j0 && j < j0 + d;
      const double is = sm.invsig[u];
#pragma unroll
      for (int n = 0; n < AMMSE_MAX_RX; ++n) {
        if (n < N) {
          zd acc = {0.0, 0.0};
#pragma unroll
          for (int k = 0; k < AMMSE_MAX_RX; ++k)
            if (k < N) acc = acc + Do[u * 16 + n * 4 + k] * gh[k];
          if (own) acc = acc - Yo[u * 16 + n * 4 + (j - j0)];
          Z[g0 + (long)n * ud] = from_d<R>(scal(is, acc));
        }
      }
    });
  }
  __syncthreads();
  channel_gemm64<R, true>(M, ud, w.un, w.H, M, Z, ud, sm.tiles,
                        [&](int i, int j, cx<R> v) {
                          Gr[(long)i * ud + j] = {R(2) * v.x, R(2) * v.y};
                        });
  __syncthreads();
  double pw = 0.0;
  const int nv = (int)w.v;
  struct LV {
    cx<R> v, q, g;
  };
  u_batched<4>(
      nv, [&](int e) { return LV{Vp[e], Vq[e], Gr[e]}; },
      [&](int e, const LV& l) {
        const zd v = to_d(l.v), q = to_d(l.q), g = to_d(l.g);
        const cx<R> x = from_d<R>(zd{(1.0 + om) * v.x - om * q.x - gamma * g.x,
                                     (1.0 + om) * v.y - om * q.y - gamma * g.y});
        Vt[e] = x;
        pw += nrm2(to_d(x));
      });
  pw = block_sum(pw, sm.red);
  const double s = (pw > w.P) ? sqrt(w.P / pw) : 1.0;
  if (tid == 0) {
    spo[0] = s;
    spo[1] = pw;
  }
  u_batched<4>(
      nv, [&](int e) { return Vt[e]; },
      [&](int e, const cx<R>& x) { Vn[e] = from_d<R>(scal(s, to_d(x))); });
  __syncthreads();
  u_product(w, sm, Gn, Vn);
  __syncthreads();
}

template <class R>
__device__ void u_load_tables(const ammse_desc_t& D, const ammse_kparams_t& p, USmem<R>& sm) {
  for (int u = threadIdx.x; u < D.U; u += AMMSE_BLOCK) {
    sm.invsig[u] = 1.0 / sqrt(p.sigma2[D.user_off + u]);
    sm.alpha[u] = p.alpha[D.user_off + u];
  }
  if (threadIdx.x == 0) sm.fail = 0;
  __syncthreads();
}

template <class R>
__device__ void u_copy(cx<R>* dst, const cx<R>* src, size_t n) {
  for (size_t e = threadIdx.x; e < n; e += AMMSE_BLOCK) dst[e] = src[e];
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(AMMSE_BLOCK, sizeof(R) == 4 ? 2 : 1) void unroll_forward_kernel(
    ammse_kparams_t p, ammse_unroll_params_t q) {
  __shared__ USmem<R> sm;
  const ammse_desc_t D = p.desc[blockIdx.x];
  const int b = D.b, T = p.max_iters, K = q.ckpt_every;
  u_load_tables(D, p, sm);
  const UView<R> w = make_view<R>(D, p, q);
  cx<R>* V = (cx<R>*)p.V + D.v_off;            // in: V^0, out: V^T
  cx<R>* ck = (cx<R>*)q.ckpt + (long)D.v_off * 2 * q.nck;
  // rotating slots: V^{t-2}, V^{t-1}, V^t in Vs[0..2], G likewise
  cx<R>* Vslot[3] = {w.Vs, w.Vs + w.v, w.Vs + 2 * w.v};
  cx<R>* Gslot[3] = {w.Gs, w.Gs + w.g, w.Gs + 2 * w.g};
  u_copy(Vslot[0], V, w.v);
  u_copy(Vslot[1], V, w.v);
  u_copy(ck, V, w.v);
  u_copy(ck + w.v, V, w.v);
  __syncthreads();
  u_product(w, sm, Gslot[1], Vslot[1]);
  __syncthreads();
  u_copy(Gslot[0], Gslot[1], w.g);
  __syncthreads();
  int fsw = p.force_switch_iter;
  if (p.force_switch && p.force_switch[b] > 0) fsw = p.force_switch[b];
  bool stage2 = (fsw >= 1) ? (fsw <= 1) : (p.warm_start == 0);
  int switch_iter = stage2 ? 1 : -1;
  double wsr_prev = 0.0, wsr_prev2 = 0.0;
  int status = 0;
  int a = 0, c = 1;   // slots of V^{t-2}, V^{t-1}
  for (int t = 1; t <= T; ++t) {
    const double rs = u_receivers(w, sm, Gslot[c], w.UWs, w.Es, w.Los);
    wsr_prev2 = wsr_prev;
    wsr_prev = block_sum(rs, sm.red) * (1.0 / M_LN2);
    if (p.trace && threadIdx.x == 0) p.trace[(long)b * p.trace_len + (t - 1)] = wsr_prev;
    if (sm.fail) status |= sm.fail;
    if (!isfinite(wsr_prev)) status |= AMMSE_INST_NONFINITE;
    if (!stage2) {
      const bool trig = (fsw >= 1) ? (t >= fsw)
                                   : (t >= 2 && rel_change(wsr_prev, wsr_prev2) <= p.eps1);
      if (trig) {
        stage2 = true;
        switch_iter = t;
      }
    }
    const int n = 3 - a - c;   // the free slot receives V^t
    u_step(w, sm, t, q.gamma[(long)b * T + (t - 1)], stage2, p.extrapolate != 0, Vslot[c],
           Vslot[a], Gslot[c], Gslot[a], w.UWs, w.Es, w.Ds, w.Ys, w.Zs, w.Grs, w.Vts, w.sp,
           Vslot[n], Gslot[n]);
    a = c;
    c = n;
    if (t % K == 0 && t < T) {
      cx<R>* dst = ck + (long)(t / K) * 2 * w.v;
      u_copy(dst, Vslot[c], w.v);
      u_copy(dst + w.v, Vslot[a], w.v);
      __syncthreads();
    }
  }
  const double rs = u_receivers(w, sm, Gslot[c], w.UWs, w.Es, w.Los);
  const double wsr_final = block_sum(rs, sm.red) * (1.0 / M_LN2);
  if (sm.fail) status |= sm.fail;
  if (!isfinite(wsr_final)) status |= AMMSE_INST_NONFINITE;
  u_copy(V, Vslot[c], w.v);
  if (threadIdx.x == 0) {
    p.wsr[b] = wsr_final;
    if (p.trace) p.trace[(long)b * p.trace_len + T] = wsr_final;
    if (p.switch_iter) p.switch_iter[b] = switch_iter;
    if (p.status) p.status[b] = status;
    if (p.iters) p.iters[b] = T;
  }
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------

// Dbar_u = (S Zbar)_u G^_u^H and Ybar_u = -(S Zbar)_u on the own columns, into
// Pa / Pb (16 lanes per user: column split and reduce-scatter).
template <class R>
__device__ void u_zbar_blocks(const UView<R>& w, USmem<R>& sm, const cx<R>* Gp, const cx<R>* Gq,
                              double om) {
  const int tid = utid();
  const int lane = tid & 63, li = lane & 15;
  const int N = w.N, d = w.d, ud = w.ud, U = w.U;
  for (int u0 = 0; u0 < U; u0 += AMMSE_BLOCK / 16) {
    const int u = u0 + (tid >> 4);
    const bool act = u < U;
    const int uu = act ? u : U - 1;
    const double is = sm.invsig[uu];
    zd sj[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) sj[q] = {0.0, 0.0};
    const long r0 = (long)(uu * N) * ud;
    // the lane's columns in chunks of CH, the loads of a chunk issued together
    // (one column at a time: two more keep the adjoint kernel above 256 registers)
    constexpr int CH = 1;
    for (int jc = li; jc < ud; jc += 16 * CH) {
      cx<R> zl[CH][AMMSE_MAX_RX], al[CH][AMMSE_MAX_RX], ql[CH][AMMSE_MAX_RX];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int j = min(jc + 16 * c, ud - 1);
#pragma unroll
        for (int k = 0; k < AMMSE_MAX_RX; ++k) {
          const long o = r0 + (long)min(k, N - 1) * ud + j;
          zl[c][k] = w.Zb[o];
          al[c][k] = Gp[o];
          ql[c][k] = Gq[o];
        }
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        if (jc + 16 * c >= ud) continue;
        zd zb[AMMSE_MAX_RX], gh[AMMSE_MAX_RX];
#pragma unroll
        for (int k = 0; k < AMMSE_MAX_RX; ++k) {
          zb[k] = {0.0, 0.0};
          gh[k] = {0.0, 0.0};
          if (k < N) {
            zb[k] = scal(is, to_d(zl[c][k]));
            gh[k] = {(1.0 + om) * (double)al[c][k].x - om * (double)ql[c][k].x,
                     (1.0 + om) * (double)al[c][k].y - om * (double)ql[c][k].y};
          }
        }
#pragma unroll
        for (int x = 0; x < AMMSE_MAX_RX; ++x)
#pragma unroll
          for (int y = 0; y < AMMSE_MAX_RX; ++y)
            if (x < N && y < N) sj[x * 4 + y] = sj[x * 4 + y] + mulc(zb[x], gh[y]);
      }
    }
#pragma unroll
    for (int step = 0; step < 4; ++step) {
      const int bit = 8 >> step;
      const bool hi = (li & bit) != 0;
#pragma unroll
      for (int q = 0; q < bit; ++q) {
        const zd send = hi ? sj[q] : sj[q + bit];
        const zd keep = hi ? sj[q + bit] : sj[q];
        sj[q] = keep + zd{__shfl_xor(send.x, bit, 64), __shfl_xor(send.y, bit, 64)};
      }
    }
    const int a = li >> 2, b = li & 3;
    if (act) {
      w.Pa[u * 16 + li] = (a < N && b < N) ? sj[0] : zd{0.0, 0.0};
      zd yb = {0.0, 0.0};
      if (a < N && b < d) yb = scal(-is, to_d(w.Zb[r0 + (long)a * ud + uu * d + b]));
      w.Pb[u * 16 + li] = yb;
    }
  }
  __syncthreads();
}

// Adjoint of the receivers and weights of one user group: from Dbar (Pa),
// Ybar (Pb), UW, E, Lo and G^{t-1} (own block F) to Jsym = Jbar + Jbar^H (Pa)
// and Fbar (Pb).
template <class R>
__device__ void u_receiver_adjoint(const UView<R>& w, USmem<R>& sm, const cx<R>* Gp, const zd* UWi,
                                   const zd* Ei, const zd* Loi, bool stage2) {
  const int tid = utid();
  const int lane = tid & 63, li = lane & 15;
  const Lane4 L4{lane & ~15, li >> 2, li & 3};
  const int N = w.N, d = w.d, ud = w.ud;
  for (int u0 = 0; u0 < w.U; u0 += AMMSE_BLOCK / 16) {
    const int u = u0 + (tid >> 4);
    const bool act = u < w.U;
    const int uu = act ? u : w.U - 1;
    const double al = sm.alpha[uu];
    const zd UWv = UWi[uu * 16 + li], Ev = Ei[uu * 16 + li], Lo = Loi[uu * 16 + li];
    const zd Db = w.Pa[uu * 16 + li], Yb = w.Pb[uu * 16 + li];
    const zd Dbt = L4.at(Db, L4.b, L4.a);
    const zd Sd = Db + cj(Dbt);                       // Dbar + Dbar^H
    zd UWb, Eb;
    if (stage2) {
      UWb = scal(al, mm_nn(L4, Sd, mm_nn(L4, UWv, Ev)) + Yb);
      Eb = scal(al, mm_hn(L4, UWv, mm_nn(L4, Db, UWv)));
    } else {
      const zd Tm = mm_nn(L4, UWv, Ev);
      const zd Tb = scal(al, mm_nn(L4, Sd, Tm) + Yb);
      UWb = mm_nn(L4, Tb, Ev);
      Eb = mm_hn(L4, UWv, Tb);
    }
    const zd Xb = scal(-1.0, mm_nn(L4, Ev, mm_nn(L4, Eb, Ev)));
    zd F = {0.0, 0.0};
    if (L4.a < N && L4.b < d) F = to_d(Gp[(long)(uu * N + L4.a) * ud + uu * d + L4.b]);
    const zd Wb = UWb + mm_nn(L4, F, Xb);            // total adjoint of UW = J^{-1} F
    const zd JW = trsm16h(L4, Lo, trsm16(L4, Lo, Wb));   // J-^{-1} Wb
    const zd Fb = mm_nh(L4, UWv, Xb) + JW;
    const zd Jb = scal(-1.0, mm_nh(L4, JW, UWv));
    const zd Jbt = L4.at(Jb, L4.b, L4.a);
    if (act) {
      w.Pa[u * 16 + li] = (L4.a < N && L4.b < N) ? Jb + cj(Jbt) : zd{0.0, 0.0};
      w.Pb[u * 16 + li] = (L4.a < N && L4.b < d) ? Fb : zd{0.0, 0.0};
    }
  }
  __syncthreads();
}

template <class R>
__global__ __launch_bounds__(AMMSE_BLOCK, 1) void unroll_backward_kernel(ammse_kparams_t p,
                                                                        ammse_unroll_params_t q) {
  __shared__ USmem<R> sm;
  const ammse_desc_t D = p.desc[blockIdx.x];
  const int b = D.b, T = p.max_iters, K = q.ckpt_every;
  u_load_tables(D, p, sm);
  const UView<R> w = make_view<R>(D, p, q);
  const int N = w.N, d = w.d, ud = w.ud, un = w.un, U = w.U, M = w.M;
  const int nv = (int)w.v, ng = (int)w.g;
  const cx<R>* ck = (const cx<R>*)q.ckpt + (long)D.v_off * 2 * q.nck;
  cx<R>* dH = (cx<R>*)q.dH + D.h_off;
  const int sw = q.switch_iter[b];
  const double gw = q.dwsr[b];
  int tid = utid();
  for (long e = tid; e < (long)un * M; e += AMMSE_BLOCK) dH[e] = {R(0), R(0)};
  for (int e = tid; e < 3 * nv; e += AMMSE_BLOCK) w.Vb[e] = {R(0), R(0)};
  for (int e = tid; e < 3 * ng; e += AMMSE_BLOCK) w.Gb[e] = {R(0), R(0)};
  __syncthreads();
  const int nseg = (T + K - 1) / K;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int t0 = seg * K, t1 = min(T, t0 + K);
    // recompute the segment from its checkpoint
    const cx<R>* src = ck + (long)seg * 2 * w.v;
    u_copy(w.Vs + w.v, src, w.v);          // V^{t0}
    u_copy(w.Vs, src + w.v, w.v);          // V^{t0-1}
    __syncthreads();
    u_product(w, sm, w.Gs + w.g, w.Vs + w.v);
    u_product(w, sm, w.Gs, w.Vs);
    __syncthreads();
    for (int t = t0 + 1; t <= t1; ++t) {
      const int k = t - t0;
      const long uo = (long)(k - 1) * U * 16;
      (void)u_receivers(w, sm, w.Gs + k * w.g, w.UWs + uo, w.Es + uo, w.Los + uo);
      __syncthreads();
      const bool st2 = sw >= 1 && t >= sw;
      u_step(w, sm, t, q.gamma[(long)b * T + (t - 1)], st2, p.extrapolate != 0,
             w.Vs + k * w.v, w.Vs + (k - 1) * w.v, w.Gs + k * w.g, w.Gs + (k - 1) * w.g,
             w.UWs + uo, w.Es + uo, w.Ds + uo, w.Ys + uo, w.Zs + (k - 1) * w.g,
             w.Grs + (k - 1) * w.v, w.Vts + (k - 1) * w.v, w.sp + 2 * (k - 1),
             w.Vs + (k + 1) * w.v, w.Gs + (k + 1) * w.g);
    }
    if (t1 == T) {
      // dWSR(V^T)/dG^T = -(2 alpha_u / ln 2) (UW E UW^H G - UW on own columns)
      const int kT = T - t0 + 1;
      const cx<R>* GT = w.Gs + kT * w.g;
      (void)u_receivers(w, sm, GT, w.Pa, w.Pb, w.UWs + (long)K * U * 16);
      __syncthreads();
      {
        const int lane = tid & 63, li = lane & 15;
        const Lane4 L4{lane & ~15, li >> 2, li & 3};
        for (int u0 = 0; u0 < U; u0 += AMMSE_BLOCK / 16) {
          const int u = u0 + (tid >> 4);
          const int uu = u < U ? u : U - 1;
          const zd UWv = w.Pa[uu * 16 + li], Ev = w.Pb[uu * 16 + li];
          const zd Dp = mm_nh(L4, mm_nn(L4, UWv, Ev), UWv);
          __syncthreads();
          if (u < U) {
            w.Pa[u * 16 + li] = Dp;
            w.Pb[u * 16 + li] = UWv;
          }
          __syncthreads();
        }
      }
      cx<R>* GbT = w.Gb + (long)(T % 3) * ng;
      for (int e = tid; e < U * ud; e += AMMSE_BLOCK) {
        const int u = quot(e, w.rud), j = e - u * ud;
        const double f = -2.0 * gw * sm.alpha[u] / M_LN2;
        const long g0 = (long)(u * N) * ud + j;
        const bool own = j >= u * d && j < u * d + d;
        for (int n = 0; n < N; ++n) {
          zd acc = {0.0, 0.0};
          for (int kk = 0; kk < N; ++kk) acc = acc + w.Pa[u * 16 + n * 4 + kk] * to_d(GT[g0 + (long)kk * ud]);
          if (own) acc = acc - w.Pb[u * 16 + n * 4 + (j - u * d)];
          const zd cur = to_d(GbT[g0 + (long)n * ud]);
          GbT[g0 + (long)n * ud] = from_d<R>(cur + scal(f, acc));
        }
      }
      __syncthreads();
    }
    for (int t = t1; t > t0; --t) {
      const int k = t - t0;
      const long uo = (long)(k - 1) * U * 16;
      const double om = p.extrapolate ? fmax((t - 2.0) / (t + 1.0), 0.0) : 0.0;
      const double gamma = q.gamma[(long)b * T + (t - 1)];
      const bool st2 = sw >= 1 && t >= sw;
      cx<R>* Vbt = w.Vb + (long)(t % 3) * nv;
      cx<R>* Vb1 = w.Vb + (long)((t + 2) % 3) * nv;   // V^{t-1}
      cx<R>* Vb2 = w.Vb + (long)((t + 1) % 3) * nv;   // V^{t-2}
      cx<R>* Gbt = w.Gb + (long)(t % 3) * ng;
      cx<R>* Gb1 = w.Gb + (long)((t + 2) % 3) * ng;
      cx<R>* Gb2 = w.Gb + (long)((t + 1) % 3) * ng;
      const cx<R>* Vt_ = w.Vs + (k + 1) * w.v;
      const cx<R>* Gp = w.Gs + k * w.g;
      const cx<R>* Gq = w.Gs + (k - 1) * w.g;
      // (a) G^t = S H V^t: dH += (S Gbar) V^H, Vbar^t += H^H (S Gbar)
      tid = utid();
      for (int e = tid; e < ng; e += AMMSE_BLOCK) {
        const double f = sm.invsig[quot(quot(e, w.rud), w.rN)];
        const cx<R> x = Gbt[e];
        Gbt[e] = {(R)f * x.x, (R)f * x.y};
      }
      __syncthreads();
      channel_gemm64<R, false, true>(un, M, ud, Gbt, ud, Vt_, ud, sm.tiles,
                                   [&](int i, int j, cx<R> v) {
                                     cx<R>& o = dH[(long)i * M + j];
                                     o = {o.x + v.x, o.y + v.y};
                                   });
      channel_gemm64<R, true>(M, ud, un, w.H, M, Gbt, ud, sm.tiles,
                            [&](int i, int j, cx<R> v) {
                              cx<R>& o = Vbt[(long)i * ud + j];
                              o = {o.x + v.x, o.y + v.y};
                            });
      __syncthreads();
      tid = utid();
      for (int e = tid; e < ng; e += AMMSE_BLOCK) Gbt[e] = {R(0), R(0)};
      // (b) projection: V~bar = s Vbar - (s / p) Re<Vbar, V~> V~ when active
      const double s = w.sp[2 * (k - 1)], pw = w.sp[2 * (k - 1) + 1];
      const cx<R>* Vtil = w.Vts + (k - 1) * w.v;
      const cx<R>* Gr = w.Grs + (k - 1) * w.v;
      double dot = 0.0;
      struct LB {
        cx<R> a, x;
      };
      u_batched<4>(
          nv, [&](int e) { return LB{Vbt[e], Vtil[e]}; },
          [&](int, const LB& l) {
            const zd a = to_d(l.a), x = to_d(l.x);
            dot += a.x * x.x + a.y * x.y;
          });
      dot = block_sum(dot, sm.red);
      const bool active = pw > w.P;
      const double c2 = active ? s / pw * dot : 0.0;
      // (c) gamma: gbar = -Re<V~bar, Grad>; V^bar = V~bar; Gradbar = -gamma V~bar
      double gd = 0.0;
      struct LC {
        cx<R> a, x, g, v1, v2;
      };
      u_batched<4>(
          nv, [&](int e) { return LC{Vbt[e], Vtil[e], Gr[e], Vb1[e], Vb2[e]}; },
          [&](int e, const LC& l) {
            const zd a = to_d(l.a), x = to_d(l.x);
            const zd vb = active ? zd{s * a.x - c2 * x.x, s * a.y - c2 * x.y} : a;
            const zd g = to_d(l.g);
            gd += vb.x * g.x + vb.y * g.y;
            Vb1[e] = from_d<R>(to_d(l.v1) + scal(1.0 + om, vb));
            Vb2[e] = from_d<R>(to_d(l.v2) - scal(om, vb));
            w.Tb[e] = from_d<R>(scal(-gamma, vb));
            Vbt[e] = {R(0), R(0)};
          });
      gd = block_sum(gd, sm.red);
      if (tid == 0) q.dgamma[(long)b * T + (t - 1)] = -gd;
      // (d) Grad = 2 H^H Z: Zbar = 2 H Gradbar, dH += 2 Z Gradbar^H
      channel_gemm64<R, false>(un, ud, M, w.H, M, w.Tb, ud, sm.tiles,
                             [&](int i, int j, cx<R> v) {
                               w.Zb[(long)i * ud + j] = {R(2) * v.x, R(2) * v.y};
                             });
      channel_gemm64<R, false, true>(un, M, ud, w.Zs + (k - 1) * w.g, ud, w.Tb, ud, sm.tiles,
                                   [&](int i, int j, cx<R> v) {
                                     cx<R>& o = dH[(long)i * M + j];
                                     o = {o.x + R(2) * v.x, o.y + R(2) * v.y};
                                   });
      __syncthreads();
      // (e) Z = S (D G^ - Y): G^bar = D (S Zbar) into Gbar^{t-1}, Gbar^{t-2};
      //     Dbar, Ybar per user
      u_zbar_blocks(w, sm, Gp, Gq, om);
      tid = utid();
      const zd* Dt = w.Ds + uo;
      {
        struct LE {
          cx<R> zb[AMMSE_MAX_RX], b1[AMMSE_MAX_RX], b2[AMMSE_MAX_RX];
        };
        auto ld = [&](int e) {
          const int u = quot(e, w.rud), j = e - u * ud;
          const long g0 = (long)(u * N) * ud + j;
          LE l;
#pragma unroll
          for (int kk = 0; kk < AMMSE_MAX_RX; ++kk) {
            const long o = g0 + (long)min(kk, N - 1) * ud;
            l.zb[kk] = w.Zb[o];
            l.b1[kk] = Gb1[o];
            l.b2[kk] = Gb2[o];
          }
          return l;
        };
        u_batched<2>(U * ud, ld, [&](int e, const LE& l) {
          const int u = quot(e, w.rud), j = e - u * ud;
          const long g0 = (long)(u * N) * ud + j;
          const double is = sm.invsig[u];
          zd zb[AMMSE_MAX_RX];
#pragma unroll
          for (int kk = 0; kk < AMMSE_MAX_RX; ++kk)
            zb[kk] = (kk < N) ? scal(is, to_d(l.zb[kk])) : zd{0.0, 0.0};
#pragma unroll
          for (int n = 0; n < AMMSE_MAX_RX; ++n) {
            if (n >= N) continue;
            zd acc = {0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < AMMSE_MAX_RX; ++kk)
              if (kk < N) acc = acc + Dt[u * 16 + n * 4 + kk] * zb[kk];
            const long o = g0 + (long)n * ud;
            Gb1[o] = from_d<R>(to_d(l.b1[n]) + scal(1.0 + om, acc));
            Gb2[o] = from_d<R>(to_d(l.b2[n]) - scal(om, acc));
          }
        });
      }
      __syncthreads();
      // (f) receivers and weights of G^{t-1}
      u_receiver_adjoint(w, sm, Gp, w.UWs + uo, w.Es + uo, w.Los + uo, st2);
      tid = utid();
      {
        struct LF {
          cx<R> g[AMMSE_MAX_RX], b1[AMMSE_MAX_RX];
        };
        auto ld = [&](int e) {
          const int u = quot(e, w.rud), j = e - u * ud;
          const long g0 = (long)(u * N) * ud + j;
          LF l;
#pragma unroll
          for (int kk = 0; kk < AMMSE_MAX_RX; ++kk) {
            const long o = g0 + (long)min(kk, N - 1) * ud;
            l.g[kk] = Gp[o];
            l.b1[kk] = Gb1[o];
          }
          return l;
        };
        u_batched<2>(U * ud, ld, [&](int e, const LF& l) {
          const int u = quot(e, w.rud), j = e - u * ud;
          const long g0 = (long)(u * N) * ud + j;
          const bool own = j >= u * d && j < u * d + d;
          zd g[AMMSE_MAX_RX];
#pragma unroll
          for (int kk = 0; kk < AMMSE_MAX_RX; ++kk)
            g[kk] = (kk < N && !own) ? to_d(l.g[kk]) : zd{0.0, 0.0};
#pragma unroll
          for (int n = 0; n < AMMSE_MAX_RX; ++n) {
            if (n >= N) continue;
            zd acc = {0.0, 0.0};
            if (own) {
              acc = w.Pb[u * 16 + n * 4 + (j - u * d)];
            } else {
#pragma unroll
              for (int kk = 0; kk < AMMSE_MAX_RX; ++kk)
                if (kk < N) acc = acc + w.Pa[u * 16 + n * 4 + kk] * g[kk];
            }
            Gb1[g0 + (long)n * ud] = from_d<R>(to_d(l.b1[n]) + acc);
          }
        });
      }
      __syncthreads();
    }
  }
  // G^0 = S H V^0 (also standing in for G^{-1}, whose adjoint is zero)
  {
    cx<R>* Gb0 = w.Gb;   // slot 0 mod 3
    tid = utid();
    for (int e = tid; e < ng; e += AMMSE_BLOCK) {
      const double f = sm.invsig[quot(quot(e, w.rud), w.rN)];
      const cx<R> x = Gb0[e];
      Gb0[e] = {(R)f * x.x, (R)f * x.y};
    }
    __syncthreads();
    channel_gemm64<R, false, true>(un, M, ud, Gb0, ud, ck, ud, sm.tiles,
                                 [&](int i, int j, cx<R> v) {
                                   cx<R>& o = dH[(long)i * M + j];
                                   o = {o.x + v.x, o.y + v.y};
                                 });
    __syncthreads();
  }
}

}  // namespace

hipError_t ammse_launch_unroll(const ammse_kparams_t& p, const ammse_unroll_params_t& q,
                               bool backward, hipStream_t s) {
  if (p.batch == 0) return hipSuccess;
  if (backward) {
    if (q.fp64)
      hipLaunchKernelGGL(unroll_backward_kernel<double>, dim3(p.batch), dim3(AMMSE_BLOCK), 0, s,
                         p, q);
    else
      hipLaunchKernelGGL(unroll_backward_kernel<float>, dim3(p.batch), dim3(AMMSE_BLOCK), 0, s,
                         p, q);
  } else {
    if (q.fp64)
      hipLaunchKernelGGL(unroll_forward_kernel<double>, dim3(p.batch), dim3(AMMSE_BLOCK), 0, s,
                         p, q);
    else
      hipLaunchKernelGGL(unroll_forward_kernel<float>, dim3(p.batch), dim3(AMMSE_BLOCK), 0, s, p,
                         q);
  }
  return hipGetLastError();
}
