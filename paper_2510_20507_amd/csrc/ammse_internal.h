// Internal declarations shared by the host side and the kernels of libammse.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ammse.h"

// Per-instance descriptor in launch order (device copy built by the plan).
struct ammse_desc_t {
  int32_t C, U, M, N, d, cell_off;
  int32_t un;   // U*N: rows of a stacked channel H_{:,c}
  int32_t ud;   // U*d: columns of all precoders together
  int32_t b;    // index of the instance in the caller's table
  int32_t tile; // output tile shape of the MFMA channel products (0, 1, 2)
  int64_t h_off, v_off, user_off, bs_off;
  int64_t ws_off;  // byte offset of the instance workspace
};

// Byte offsets of the sub-buffers inside one instance workspace.
struct ammse_ws_layout_t {
  size_t Gp, Gq, Z, Vq;       // storage-precision complex matrices
  size_t UWm, Em, Dm, Ym;     // double complex per-user 4 x 4 blocks
  size_t Lq, Lw, Ly1, Ly2;    // Lanczos basis and work vectors (double complex)
  size_t Am, Lm, Bm, Xm;      // WMMSE: matrix and its Cholesky factor (M x M at most),
                              // right-hand sides and solution (M x (U d) at most),
                              // double complex; empty for Algorithm 3
  size_t Tm;                  // WMMSE: S D S H_{:,c} or R = C^H S H_{:,c} ((U N) x M,
                              // double complex)
  size_t Qm;                  // S H H^H S ((U N) x (U N), storage precision), see below
  size_t Kq;                  // Q path: K = C^H Q C of the step-size Lanczos ((U N) x (U N))
  size_t Hb, Xb, Zb;          // bfloat16 copies of H, X and Z (mixed precision only)
  size_t Dmf, Ymf;            // float copies of Dm, Ym (float storage only)
  size_t Lwm, Lim, Cm;        // per-user Lw, Lw^{-1}, C (double complex 4 x 4): WMMSE,
                              // and Lw^{-1}, C for the Q- and Gram-based Lanczos
  size_t Rg, Kg;              // Gram-based Lanczos: R = C^H S H_{:,c} ((U d) x M) and
                              // R R^H or R^H R (ammse_gram_order), storage precision
  size_t X1, X2, G0;          // Q recursion (single cell, U N <= M, float products): the
                              // implicit precoder's X^{t-1}, X^{t-2} and G^0 ((U N) x (U d),
                              // storage precision)
  size_t Ubm, Wbm, Jbm, Fbm;  // BCGD-WMMSE: per-user U and W iterates, receive covariance J
                              // and own-stream image G_own of the current V (double complex
                              // 4 x 4 blocks)
  size_t Rb, Ab, Gb;          // stage-II step bound on the antenna side (ammse_bound_gram):
                              // S_a H_{:,c} ((U N) x M, one BS at a time),
                              // A_c = H_{:,c}^H S_a^2 H_{:,c} (M x M per BS), storage
                              // precision, and the resulting steps 1 / Lhat_c (C doubles)
  size_t total;
};

// Launch parameters of the fused solve kernel.
struct ammse_kparams_t {
  const ammse_desc_t* desc;
  const int32_t* cell_users;
  const void* H;
  const double* sigma2;
  const double* alpha;
  const double* P;
  void* V;
  double* wsr;
  int32_t* iters;
  int32_t* switch_iter;
  int32_t* status;
  double* trace;
  const int32_t* force_switch;
  char* ws;
  int32_t batch;
  int32_t max_iters;
  int32_t T_c;
  int32_t warm_start;
  int32_t extrapolate;
  int32_t rearm;
  int32_t force_switch_iter;
  int32_t lanczos_steps;
  int32_t wsr_only;      // 1: evaluate WSR(V) and return (no iteration, V not written)
  int32_t trace_len;     // max_iters + 1
  int32_t algorithm;     // AMMSE_ALGO_*
  int32_t lds_factor;    // exact V step: dynamic LDS holds a <= 64 x 64 Cholesky factor
                         // (1) and also the solution block (2)
  int32_t bf16_copies;   // BF16 mode: the workspace holds bfloat16 operand copies
  int32_t lowp_iters;    // BF16 mode: iterations 1..lowp_iters use bfloat16 products
                         // (and G^0 when lowp_iters >= 1); -1: float products only
  int32_t tile_force;    // 0: per-instance tile shape from the descriptor; v + 1: shape v
  int32_t step_rule;     // AMMSE_STEP_BOUND / AMMSE_STEP_FROZEN
  int32_t n_qp;          // general kernel: launch positions [0, n_qp) hold the instances
                         // of the single-cell Q path (ammse_qpath_instance)
  int32_t block_base;    // launch position of workgroup 0 of a general-kernel launch
  int32_t bound_pre;     // general kernel: the stage-II bound of the instances that
                         // ammse_bound_gram selects was written to their workspace by
                         // ammse_bound_gram_kernel before this launch
  double eps1, eps2, gamma_c;
  double* gbound;        // LDS-resident kernel: 1 / Lhat per launch position (bound rule)
};

#define AMMSE_BLOCK 256
#define AMMSE_TILE_SHAPES 3   // output tile shapes of the MFMA channel products
#define AMMSE_MAX_LANCZOS 64
#define AMMSE_LANCZOS_LDS_N 512   // Lanczos vectors of up to this order in LDS (general kernel)
#define AMMSE_GRAM_WAVE_N 192     // Gram-matrix Lanczos of up to this order: one wave per BS

// Workspace layout of one instance (bytes), for complex storage of
// `real_bytes` per component (8 for FP64, 4 for FP32).  Every sub-buffer
// starts on a 256-byte boundary.
__host__ __device__ inline size_t ammse_align256(size_t x) { return (x + 255) & ~size_t(255); }

// Algorithm 3 on a single cell with U N <= M: the one-product Q path of the
// general kernel (its own kernel variant, its instances first in launch order).
__host__ __device__ inline bool ammse_qpath_instance(int C, int U, int M, int N, int algorithm) {
  return algorithm == AMMSE_ALGO_AMMMSE && C == 1 && (long)U * N <= M;
}

// Order of the Gram matrix of the step-size Lanczos: with D = C C^H and
// R_c = C^H S H_{:,c} ((U d) x M), lambda_max(H_{:,c}^H S D S H_{:,c}) is the
// largest eigenvalue of both R_c R_c^H ((U d) x (U d), stream side) and
// R_c^H R_c (M x M, antenna side); the smaller one is used.
__host__ __device__ inline long ammse_gram_order(int U, int M, int d) {
  const long ud = (long)U * d;
  return ud < M ? ud : (long)M;
}

// Step-size Lanczos of Algorithm 3 on that Gram matrix instead of the operator
// x -> H_{:,c}^H S D S H_{:,c} x: float storage, not the single-cell Q path,
// and fewer matrix entries per step (order^2 < 2 U N M).
__host__ __device__ inline bool ammse_gram_path(int real_bytes, int C, int U, int M, int N, int d,
                                                bool wmmse) {
  const long un = (long)U * N, ng = ammse_gram_order(U, M, d);
  const bool qp = !wmmse && C == 1 && un <= M;
  return real_bytes == 4 && !wmmse && !qp && ng * ng < 2 * un * (long)M;
}

// Stage-II step bound of Algorithm 3 (and of BCGD-WMMSE), lambda_max(A_c) with
// A_c = H_{:,c}^H S_a^2 H_{:,c}, S_a = diag(sqrt(alpha_u) / sigma_u): with
// float storage off the single-cell Q path and M <= AMMSE_GRAM_WAVE_N, A_c is
// formed by an MFMA product and its largest eigenvalue found by one wave per
// BS (each Lanczos step then reads A_c once instead of passing over H_{:,c}
// twice), in a kernel of its own launched before the solve kernel.
__host__ __device__ inline bool ammse_bound_gram(int real_bytes, int C, int U, int M, int N,
                                                 bool wmmse, bool bcgd) {
  const bool qp = !wmmse && !bcgd && C == 1 && (long)U * N <= M;
  return real_bytes == 4 && !wmmse && !qp && M <= AMMSE_GRAM_WAVE_N;
}

__host__ __device__ inline ammse_ws_layout_t ammse_ws_layout(int real_bytes, int C, int U, int M,
                                                             int N, int d, int lanczos_steps,
                                                             bool wmmse, bool bf16 = false,
                                                             bool bcgd = false) {
  const size_t cs = 2 * (size_t)real_bytes;      // storage complex
  const size_t zs = 16;                          // double complex
  const size_t un = (size_t)U * N, ud = (size_t)U * d;
  ammse_ws_layout_t L;
  size_t o = 0;
  L.Gp = o;  o += ammse_align256(un * ud * cs);
  L.Gq = o;  o += ammse_align256(un * ud * cs);
  L.Z = o;   o += ammse_align256(un * ud * cs);
  L.Vq = o;  o += ammse_align256((size_t)M * ud * cs);
  L.UWm = o; o += ammse_align256((size_t)U * 16 * zs);
  L.Em = o;  o += ammse_align256((size_t)U * 16 * zs);
  L.Dm = o;  o += ammse_align256((size_t)U * 16 * zs);
  L.Ym = o;  o += ammse_align256((size_t)U * 16 * zs);
  const size_t gp = ammse_gram_path(real_bytes, C, U, M, N, d, wmmse || bcgd) ? 1 : 0;
  const size_t ng = (size_t)ammse_gram_order(U, M, d);   // <= M
  const size_t nl = (size_t)M;                           // Lanczos order (at most)
  L.Lq = o;  o += ammse_align256((size_t)3 * nl * zs);   // three Lanczos vectors
  L.Lw = o;  o += ammse_align256((size_t)M * zs);
  L.Ly1 = o; o += ammse_align256(un * zs);
  L.Ly2 = o; o += ammse_align256(un * zs);
  const size_t w = wmmse ? 1 : 0;
  L.Am = o;  o += ammse_align256(w * (size_t)M * M * zs);
  L.Lm = o;  o += ammse_align256(w * (size_t)M * M * zs);
  L.Bm = o;  o += ammse_align256(w * (size_t)M * ud * zs);
  L.Xm = o;  o += ammse_align256(w * (size_t)M * ud * zs);
  L.Tm = o;  o += ammse_align256(w * un * (size_t)M * zs);
  // Algorithm 3, single cell with U N <= M: Lanczos on Q = S H H^H S
  const size_t qp = (!wmmse && !bcgd && C == 1 && un <= (size_t)M) ? 1 : 0;
  L.Qm = o;  o += ammse_align256(qp * un * un * cs);
  L.Kq = o;  o += ammse_align256(qp * un * un * cs);
  // Algorithm 3 otherwise, float storage, when the (U d) x (U d) Gram matrix
  // is smaller than two passes over H_{:,c}: Lanczos on K = R R^H (gp above)
  L.Lwm = o; o += ammse_align256(w * (size_t)U * 16 * zs);
  L.Lim = o; o += ammse_align256((w | qp | gp) * (size_t)U * 16 * zs);
  L.Cm = o;  o += ammse_align256((w | qp | gp) * (size_t)U * 16 * zs);
  L.Rg = o;  o += ammse_align256(gp * ud * (size_t)M * cs);
  // one Gram matrix per BS when the per-BS iterations run one wave each
  // (order <= AMMSE_GRAM_WAVE_N), else one at a time
  const size_t gk = (ng <= (size_t)AMMSE_GRAM_WAVE_N) ? (size_t)C : 1;
  L.Kg = o;  o += ammse_align256(gp * gk * ng * ng * cs);
  const size_t rp = (qp && real_bytes == 4) ? 1 : 0;
  L.X1 = o;  o += ammse_align256(rp * un * ud * cs);
  L.X2 = o;  o += ammse_align256(rp * un * ud * cs);
  L.G0 = o;  o += ammse_align256(rp * un * ud * cs);
  // mixed precision: bfloat16 copies of H (all cells), of the precoder and of Z
  const size_t bb = bf16 ? 4 : 0;
  L.Hb = o;  o += ammse_align256(bb * (size_t)C * un * M);
  L.Xb = o;  o += ammse_align256(bb * (size_t)M * ud);
  L.Zb = o;  o += ammse_align256(bb * un * ud);
  // float storage: float copies of D and Y for the Z build
  const size_t fz = (real_bytes == 4) ? 8 : 0;
  L.Dmf = o; o += ammse_align256((size_t)U * 16 * fz);
  L.Ymf = o; o += ammse_align256((size_t)U * 16 * fz);
  const size_t bc = bcgd ? 1 : 0;
  L.Ubm = o; o += ammse_align256(bc * (size_t)U * 16 * zs);
  L.Wbm = o; o += ammse_align256(bc * (size_t)U * 16 * zs);
  L.Jbm = o; o += ammse_align256(bc * (size_t)U * 16 * zs);
  L.Fbm = o; o += ammse_align256(bc * (size_t)U * 16 * zs);
  const size_t ba = ammse_bound_gram(real_bytes, C, U, M, N, wmmse, bcgd) ? 1 : 0;
  L.Rb = o;  o += ammse_align256(ba * un * (size_t)M * cs);
  L.Ab = o;  o += ammse_align256(ba * (size_t)C * M * M * cs);
  L.Gb = o;  o += ammse_align256(ba * (size_t)C * sizeof(double));
  L.total = o;
  return L;
}

// Workspace of one instance of the unrolled solver (forward and adjoint), K
// iterations per checkpoint segment; every sub-buffer 256-byte aligned.
struct ammse_unroll_layout_t {
  size_t Vs, Gs, Zs, Grs, Vts, sp;           // segment storage
  size_t UWs, Es, Los, Ds, Ys;               // per-user blocks, K + 1 slots
  size_t Vb, Gb, Zb, Tb, Pa, Pb;             // adjoints
  size_t total;
};

__host__ __device__ inline ammse_unroll_layout_t ammse_unroll_layout(int real_bytes, int U, int M,
                                                                     int N, int d, int K) {
  const size_t cs = 2 * (size_t)real_bytes, zs = 16;
  const size_t v = (size_t)M * U * d * cs, g = (size_t)U * N * U * d * cs;
  const size_t ub = (size_t)U * 16 * zs;
  ammse_unroll_layout_t L;
  size_t o = 0;
  L.Vs = o;  o += ammse_align256((size_t)(K + 2) * v);
  L.Gs = o;  o += ammse_align256((size_t)(K + 2) * g);
  L.Zs = o;  o += ammse_align256((size_t)K * g);
  L.Grs = o; o += ammse_align256((size_t)K * v);
  L.Vts = o; o += ammse_align256((size_t)K * v);
  L.sp = o;  o += ammse_align256((size_t)K * 2 * sizeof(double));
  L.UWs = o; o += ammse_align256((size_t)(K + 1) * ub);
  L.Es = o;  o += ammse_align256((size_t)(K + 1) * ub);
  L.Los = o; o += ammse_align256((size_t)(K + 1) * ub);
  L.Ds = o;  o += ammse_align256((size_t)(K + 1) * ub);
  L.Ys = o;  o += ammse_align256((size_t)(K + 1) * ub);
  L.Vb = o;  o += ammse_align256(3 * v);
  L.Gb = o;  o += ammse_align256(3 * g);
  L.Zb = o;  o += ammse_align256(g);
  L.Tb = o;  o += ammse_align256(v);
  L.Pa = o;  o += ammse_align256(ub);
  L.Pb = o;  o += ammse_align256(ub);
  L.total = o;
  return L;
}

// Extra launch parameters of the unrolled solver.
struct ammse_unroll_params_t {
  const double* gamma;        // [batch][T] step sizes (caller's instance order)
  void* ckpt;                 // checkpoints: instance b at element 2 * nck * v_off
  void* dH;                   // adjoint only: dWSR/dH, layout of H
  double* dgamma;             // adjoint only: [batch][T]
  const int32_t* switch_iter; // adjoint only: stage-switch iteration of the forward
  const double* dwsr;         // adjoint only: upstream weight per instance
  size_t ws_stride;           // workspace bytes per launched workgroup
  int32_t ckpt_every;         // K
  int32_t nck;                // checkpoints per instance, ceil(T / K)
  int32_t fp64;
};

hipError_t ammse_launch_unroll(const ammse_kparams_t& p, const ammse_unroll_params_t& q,
                               bool backward, hipStream_t s);
hipError_t ammse_launch_fp64(const ammse_kparams_t& p, hipStream_t s);
size_t ammse_general_lds_bytes(int precision, int algorithm);
// LDS-resident MFMA kernel (FP32): shapes it serves, its LDS use, launch.
bool ammse_fast_eligible(int C, int U, int M, int N, int d);
size_t ammse_fast_lds_bytes();
hipError_t ammse_launch_fast_fp32(const ammse_kparams_t& p, hipStream_t s);
hipError_t ammse_launch_fp32(const ammse_kparams_t& p, hipStream_t s);
// Device address of the calling thread's current device's copy of the
// library's static workspace array (AMMSE_SCRATCH_BYTES), resolved once per
// device and cached; call with `device` current.
hipError_t ammse_scratch_resolve(int device, void** ptr);
