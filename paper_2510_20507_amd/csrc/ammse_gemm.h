// Channel products shared by the solve kernels (gfx950): complex GEMMs
// staged through LDS with an element-wise epilogue functor, FP64 on FMA and
// FP32 storage on MFMA (float or bfloat16 products, float accumulation).
#pragma once

#include <type_traits>

#include "ammse_device.h"
#include "ammse_internal.h"

namespace ammse_dev {

// Thread index hidden from loop-invariant code motion: each phase of the
// fused kernel re-derives its lane indices instead of the compiler keeping
// every phase's index arithmetic live across the whole iteration loop, which
// would cost occupancy.
__device__ __forceinline__ int phase_tid() {
  int x = threadIdx.x;
  asm volatile("" : "+v"(x));
  return x;
}

constexpr int KC = 16;   // k-chunk of the FP64 channel products
constexpr int TM = 64;   // FP64 output tile rows
constexpr int TN = 64;   // FP64 output tile columns

typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// Output tile shapes of the MFMA channel products (the autotuned choice):
//   0: 64 x 64  (each wave one 16-row block, four 16-column blocks)
//   1: 128 x 16 (each wave two 16-row blocks, one column block) for the
//      tall, narrow products of instances with few streams per cell
//   2: 64 x 32  (each wave one row block, two column blocks)
static_assert(AMMSE_TILE_SHAPES == 3, "tile shapes below");
template <int V> struct TileShape;
template <> struct TileShape<0> { static constexpr int TM = 64, TN = 64; };
template <> struct TileShape<1> { static constexpr int TM = 128, TN = 16; };
template <> struct TileShape<2> { static constexpr int TM = 64, TN = 32; };
// 3: 64 x 16 (each wave one row block, one column block): not an autotuner
//    choice; the products with 33-64 output rows and at most 16 columns take it
template <> struct TileShape<3> { static constexpr int TM = 64, TN = 16; };


template <class T, int V>
struct MfmaTile {
  static constexpr bool LOW = sizeof(T) == 2;
  static constexpr int TM = TileShape<V>::TM, TN = TileShape<V>::TN;
  static constexpr int RB = TM / 64, CB = TN / 16;  // 16 x 16 blocks per wave
  static constexpr int KC = LOW ? 32 : 16;          // k-chunk
  static constexpr int LD = LOW ? KC + 8 : KC + 1;  // padded k stride (elements)
  static constexpr int NA = TM * KC / AMMSE_BLOCK;  // staged A elements per thread
  static constexpr int NB = KC * TN / AMMSE_BLOCK;
  static constexpr size_t bytes = sizeof(T) * 2 * (TM + TN) * LD;
  static_assert(NA >= 1 && NB >= 1, "every thread stages one element of each operand");
};

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

template <class R>
constexpr size_t tile_bytes() {
  if constexpr (sizeof(R) == 8) {
    return sizeof(cx<R>) * KC * (TM + 1 + TN + 1);
  } else {
    return cmax(cmax(cmax(MfmaTile<float, 0>::bytes, MfmaTile<__bf16, 0>::bytes),
                     cmax(MfmaTile<float, 1>::bytes, MfmaTile<__bf16, 1>::bytes)),
                cmax(MfmaTile<float, 2>::bytes, MfmaTile<__bf16, 2>::bytes));
  }
}

// P (m x n) = op(A) * op(B) handed element by element to the epilogue
// epi(i, j, P[i][j]).  op(A) = A (m x k, row-major, lda) or, with CONJA,
// A^H where A is stored k x m row-major (lda).  op(B) = B (k x n, row-major,
// ldb) or, with CONJB, B^H where B is stored n x k row-major (ldb).
// All operands in global memory, staged through LDS tiles of 64 x 16.
template <class R, bool CONJA, bool CONJB, class Epi>
__device__ void block_gemm(int m, int n, int k, const cx<R>* __restrict__ A, long lda,
                           const cx<R>* __restrict__ B, long ldb, cx<R>* As, cx<R>* Bs,
                           Epi&& epi) {
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
          // scalar parts, so that the staged value stays in registers
          R vx = R(0), vy = R(0);
          if (gi < m && gk < k) {
            const cx<R> t = CONJA ? A[(long)gk * lda + gi] : A[(long)gi * lda + gk];
            vx = t.x;
            vy = CONJA ? -t.y : t.y;
          }
          As[kk * (TM + 1) + row].x = vx;
          As[kk * (TM + 1) + row].y = vy;
        }
        for (int e = tid; e < KC * TN; e += AMMSE_BLOCK) {
          const int col = CONJB ? e / KC : e % TN, kk = CONJB ? e % KC : e / TN;
          const int gj = j0 + col, gk = k0 + kk;
          R vx = R(0), vy = R(0);
          if (gj < n && gk < k) {
            const cx<R> t = CONJB ? B[(long)gj * ldb + gk] : B[(long)gk * ldb + gj];
            vx = t.x;
            vy = CONJB ? -t.y : t.y;
          }
          Bs[kk * (TN + 1) + col].x = vx;
          Bs[kk * (TN + 1) + col].y = vy;
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
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gj = j0 + tx + 16 * j;
          if (gj < n) epi(gi, gj, acc[i][j]);
        }
      }
    }
  }
}

// MFMA channel products (FP32 storage): P = op(A) B into the epilogue as in
// block_gemm, products in T = float (v_mfma_f32_16x16x4f32)
// or T = bfloat16 (v_mfma_f32_16x16x32_bf16), float accumulation either way.
// Operand tiles are staged through LDS in planar form (real and imaginary
// planes, k contiguous per row / column, converted to T on the way in); the
// global loads of the next k-chunk are issued before the current chunk's
// products so that their latency overlaps the MFMA work.  Each of the four
// waves owns a strip of RB 16-row blocks of the output tile and its CB
// 16-column blocks; a complex product is three real accumulators: Re Re,
// Im Im and, with float operands, (Re + Im)(Re + Im) (three real products,
// Gauss), with bfloat16 operands Re Im + Im Re (two products, whose operand
// sums would need a conversion each).
// Complex bfloat16 in memory (operand copies of the mixed-precision mode).
struct alignas(4) bfc {   // one 32-bit word per complex element
  __bf16 x, y;
};
__device__ __forceinline__ cx<float> to_f(const cx<float>& v) { return v; }
__device__ __forceinline__ cx<float> to_f(const bfc& v) { return {(float)v.x, (float)v.y}; }
__device__ __forceinline__ bfc to_bfc(const cx<float>& v) { return {(__bf16)v.x, (__bf16)v.y}; }

// An epilogue functor may split each element into a load phase, L l =
// epi.pre(i, j) (reads only; any in-range indices), and epi(i, j, v, l) (the
// arithmetic and stores).  The tile products then issue the reads of a group
// of the lane's elements together and finish the group before reading the
// next, instead of waiting for each element's reads after the previous
// element's stores (which may alias them for all the compiler knows); the
// next tile's first k-chunk is fetched after the epilogue, so the groups'
// reads take the registers of that prefetch.
template <class E, class = void>
struct has_pre : std::false_type {};
template <class E>
struct has_pre<E, std::void_t<decltype(std::declval<std::remove_reference_t<E>&>().pre(0, 0))>>
    : std::true_type {};
template <class E, bool P>
struct PreType {
  struct type {};
};
template <class E>
struct PreType<E, true> {
  using type = decltype(std::declval<std::remove_reference_t<E>&>().pre(0, 0));
};

// Operands are float or bfloat16 complex in memory (TA, TB); either way they
// are converted to T on the way into LDS.
template <class T, int VAR, bool CONJA, bool CONJB, class Epi, class TA, class TB>
__device__ void block_gemm_mfma(int m, int n, int k, const TA* __restrict__ A, long lda,
                                const TB* __restrict__ B, long ldb, char* lds, Epi&& epi) {
  using Tl = MfmaTile<T, VAR>;
  constexpr int KC = Tl::KC, LD = Tl::LD, NA = Tl::NA, NB = Tl::NB;
  constexpr int TM = Tl::TM, TN = Tl::TN, RB = Tl::RB, CB = Tl::CB;
  T* AsR = (T*)lds;
  T* AsI = AsR + TM * LD;
  T* BsR = AsI + TM * LD;
  T* BsI = BsR + TN * LD;
  const int tid = phase_tid();
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int ntn = (n + TN - 1) / TN, nk = (k + KC - 1) / KC;
  const int steps = ((m + TM - 1) / TM) * ntn * nk;
  // staging coordinates: A along the contiguous global index, B along columns
  auto a_rk = [&](int q, int& row, int& kk) {
    const int e = tid + AMMSE_BLOCK * q;
    if (CONJA) {
      row = e % TM;
      kk = e / TM;
    } else {
      kk = e % KC;
      row = e / KC;
    }
  };
  auto b_ck = [&](int q, int& col, int& kk) {
    const int e = tid + AMMSE_BLOCK * q;
    if (CONJB) {
      kk = e % KC;
      col = e / KC;
    } else {
      col = e % TN;
      kk = e / TN;
    }
  };
  TA ra[NA];   // raw operand values: converted when stashed, so the
  TB rb[NB];   // prefetch loads stay in flight during the products
  // step cursor (k-chunk, tile row, tile column), advanced step by step (no
  // divisions): at the top of a step it moves to the next step, which is the
  // one the prefetch then loads
  int ck = 0, ci = 0, cj = 0;
  auto advance = [&]() __attribute__((always_inline)) {
    if (++ck == nk) {
      ck = 0;
      if (++cj == ntn) {
        cj = 0;
        ++ci;
      }
    }
  };
  auto fetch = [&]() __attribute__((always_inline)) {
    const int k0 = ck * KC, i0 = ci * TM, j0 = cj * TN;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int row, kk;
      a_rk(q, row, kk);
      const int gi = i0 + row, gk = k0 + kk;
      ra[q] = TA{};
      if (gi < m && gk < k) ra[q] = CONJA ? A[(long)gk * lda + gi] : A[(long)gi * lda + gk];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int col, kk;
      b_ck(q, col, kk);
      const int gj = j0 + col, gk = k0 + kk;
      rb[q] = TB{};
      if (gj < n && gk < k) rb[q] = CONJB ? B[(long)gj * ldb + gk] : B[(long)gk * ldb + gj];
    }
  };
  floatx4_t P[RB][CB][3];
  fetch();
  for (int s = 0; s < steps; ++s) {
    const int kc = ck, i0t = ci * TM, j0t = cj * TN;
    advance();
    if (kc == 0) {
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int q = 0; q < 3; ++q) P[i][j][q] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    }
    __syncthreads();   // the previous chunk's products are done with the tiles
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int row, kk;
      a_rk(q, row, kk);
      const cx<float> va = to_f(ra[q]);
      AsR[row * LD + kk] = (T)va.x;
      AsI[row * LD + kk] = (T)(CONJA ? -va.y : va.y);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int col, kk;
      b_ck(q, col, kk);
      const cx<float> vb = to_f(rb[q]);
      BsR[col * LD + kk] = (T)vb.x;
      BsI[col * LD + kk] = (T)(CONJB ? -vb.y : vb.y);
    }
    __syncthreads();
    constexpr int EG = 2;   // lane elements per load group of the epilogue
    // (only where the prefetch it displaces holds at least as many registers)
    constexpr bool PRE = has_pre<Epi>::value &&
                         EG * sizeof(typename PreType<Epi, has_pre<Epi>::value>::type) <=
                             NA * sizeof(TA) + NB * sizeof(TB);
    using L = typename PreType<Epi, PRE>::type;
    L pl[EG];               // load phase of the epilogue's current group (PRE)
    const bool last = kc == nk - 1;
    // group g: 16 x 16 block g / (4 / EG) of the lane's blocks, rows EG (g % (4 / EG)) on
    auto preload = [&](int g) __attribute__((always_inline)) {
      if constexpr (PRE) {
        const int blk = g / (4 / EG), r0 = EG * (g % (4 / EG));
        const int i = blk / CB, j = blk - i * CB;
        const int i0 = i0t, j0 = j0t;
        const int gj = min(j0 + 16 * j + li, n - 1);
#pragma unroll
        for (int r = 0; r < EG; ++r)
          pl[r] = epi.pre(min(i0 + 16 * (RB * wave + i) + 4 * lk + r0 + r, m - 1), gj);
      }
    };
    if (!(PRE && last) && s + 1 < steps) fetch();
    if constexpr (Tl::LOW) {
      bf16x8_t axr[RB], axi[RB], bxr[CB], bxi[CB];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int ar = (16 * (RB * wave + i) + li) * LD + 8 * lk;
        axr[i] = *(const bf16x8_t*)(AsR + ar);
        axi[i] = *(const bf16x8_t*)(AsI + ar);
      }
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int br = (16 * j + li) * LD + 8 * lk;
        bxr[j] = *(const bf16x8_t*)(BsR + br);
        bxi[j] = *(const bf16x8_t*)(BsI + br);
      }
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          P[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(axr[i], bxr[j], P[i][j][0], 0, 0, 0);
          P[i][j][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(axi[i], bxi[j], P[i][j][1], 0, 0, 0);
          P[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(axr[i], bxi[j], P[i][j][2], 0, 0, 0);
          P[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(axi[i], bxr[j], P[i][j][2], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        float axr[RB], axi[RB], bxr[CB], bxi[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          const int ar = (16 * (RB * wave + i) + li) * LD + kk + lk;
          axr[i] = AsR[ar];
          axi[i] = AsI[ar];
        }
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const int br = (16 * j + li) * LD + kk + lk;
          bxr[j] = BsR[br];
          bxi[j] = BsI[br];
        }
        // three real products per complex product (Gauss): Ar Br, Ai Bi and
        // (Ar + Ai)(Br + Bi), whose difference from the first two is the
        // imaginary part
        float axs[RB], bxs[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i) axs[i] = axr[i] + axi[i];
#pragma unroll
        for (int j = 0; j < CB; ++j) bxs[j] = bxr[j] + bxi[j];
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            P[i][j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(axr[i], bxr[j], P[i][j][0], 0, 0, 0);
            P[i][j][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(axi[i], bxi[j], P[i][j][1], 0, 0, 0);
            P[i][j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(axs[i], bxs[j], P[i][j][2], 0, 0, 0);
          }
      }
    }
    if (last) {
      const int i0 = i0t, j0 = j0t;
      if constexpr (PRE) {
        preload(0);
#pragma unroll
        for (int g = 0; g < RB * CB * (4 / EG); ++g) {
          const int blk = g / (4 / EG), r0 = EG * (g % (4 / EG));
          const int i = blk / CB, j = blk - i * CB;
          const int gj = j0 + 16 * j + li;
#pragma unroll
          for (int r = 0; r < EG; ++r) {
            const int gi = i0 + 16 * (RB * wave + i) + 4 * lk + r0 + r;
            const float p0 = P[i][j][0][r0 + r], p1 = P[i][j][1][r0 + r], p2 = P[i][j][2][r0 + r];
            if (gi < m && gj < n) epi(gi, gj, cx<float>{p0 - p1, Tl::LOW ? p2 : p2 - p0 - p1}, pl[r]);
          }
          if (g + 1 < RB * CB * (4 / EG)) preload(g + 1);
        }
        if (s + 1 < steps) fetch();
      } else {
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gi = i0 + 16 * (RB * wave + i) + 4 * lk + r;
            if (gi >= m) continue;
#pragma unroll
            for (int j = 0; j < CB; ++j) {
              const int gj = j0 + 16 * j + li;
              const float p0 = P[i][j][0][r], p1 = P[i][j][1][r], p2 = P[i][j][2][r];
              if (gj < n) epi(gi, gj, cx<float>{p0 - p1, Tl::LOW ? p2 : p2 - p0 - p1});
            }
          }
      }
    }
  }
  __syncthreads();
}

// Products with few output rows (m <= 32: the gradient products and the
// antenna-side Gram matrices of small-antenna instances), where the tile
// shapes above (64 or 128 rows) would spend most of their MFMA work on padding
// rows: output tiles of TM = 16 TMB rows and TN = 16 TNB columns, one 16 x 16
// block per group of waves, and the k-chunks of a step split over the
// KS = 4 / (TMB TNB) groups (each group's chunk in its own LDS slot); at the
// end of a tile the groups' partial accumulators are summed through LDS
// before the epilogue.  Same staging, conversion and prefetch as above.
template <class T, int TMB, int TNB, bool CONJA, bool CONJB, class Epi, class TA, class TB>
__device__ void block_gemm_mfma_ks(int m, int n, int k, const TA* __restrict__ A, long lda,
                                   const TB* __restrict__ B, long ldb, char* lds, Epi&& epi) {
  constexpr bool LOW = sizeof(T) == 2;
  constexpr int KC = LOW ? 32 : 16, LD = LOW ? KC + 8 : KC + 1;
  constexpr int TM = 16 * TMB, TN = 16 * TNB, NBLK = TMB * TNB, KS = 4 / NBLK;
  constexpr int CH_A = TM * KC, CH_B = KC * TN;               // elements per chunk
  constexpr int NA = KS * CH_A / AMMSE_BLOCK, NB = KS * CH_B / AMMSE_BLOCK;
  constexpr int SLOT = 2 * (TM + TN) * LD;                     // T elements per slot
  static_assert(KS * NBLK == 4 && NA >= 1 && NB >= 1, "four waves, every thread stages");
  static_assert(KS * SLOT * sizeof(T) <= tile_bytes<float>(), "slots fit the tile area");
  static_assert(4 * 64 * 12 * sizeof(float) <= tile_bytes<float>(), "partials fit the tile area");
  T* base = (T*)lds;
  const int tid = phase_tid();
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int blk = wave % NBLK, kg = wave / NBLK;
  const int rbk = blk / TNB, cbk = blk % TNB;
  const int ntn = (n + TN - 1) / TN, nk = (k + KC - 1) / KC;
  const int nks = (nk + KS - 1) / KS;                          // steps per tile
  const int steps = ((m + TM - 1) / TM) * ntn * nks;
  auto a_rk = [&](int q, int& slot, int& row, int& kk) {
    const int e = tid + AMMSE_BLOCK * q;
    slot = e / CH_A;
    const int f = e - slot * CH_A;
    if (CONJA) {
      row = f % TM;
      kk = f / TM;
    } else {
      kk = f % KC;
      row = f / KC;
    }
  };
  auto b_ck = [&](int q, int& slot, int& col, int& kk) {
    const int e = tid + AMMSE_BLOCK * q;
    slot = e / CH_B;
    const int f = e - slot * CH_B;
    if (CONJB) {
      kk = f % KC;
      col = f / KC;
    } else {
      col = f % TN;
      kk = f / TN;
    }
  };
  TA ra[NA];
  TB rb[NB];
  // step cursor (step within the tile, tile row, tile column), advanced step
  // by step (no divisions): at the top of a step it moves to the next step,
  // which is the one the prefetch then loads
  int ck = 0, ci = 0, cj = 0;
  auto advance = [&]() __attribute__((always_inline)) {
    if (++ck == nks) {
      ck = 0;
      if (++cj == ntn) {
        cj = 0;
        ++ci;
      }
    }
  };
  auto fetch = [&]() __attribute__((always_inline)) {
    const int c0 = ck * KS;                                     // first chunk of the step
    const int i0 = ci * TM, j0 = cj * TN;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int slot, row, kk;
      a_rk(q, slot, row, kk);
      const int gi = i0 + row, gk = (c0 + slot) * KC + kk;
      ra[q] = TA{};
      if (gi < m && gk < k) ra[q] = CONJA ? A[(long)gk * lda + gi] : A[(long)gi * lda + gk];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int slot, col, kk;
      b_ck(q, slot, col, kk);
      const int gj = j0 + col, gk = (c0 + slot) * KC + kk;
      rb[q] = TB{};
      if (gj < n && gk < k) rb[q] = CONJB ? B[(long)gj * ldb + gk] : B[(long)gk * ldb + gj];
    }
  };
  floatx4_t P[3];
  fetch();
  for (int s = 0; s < steps; ++s) {
    const int kc = ck, i0t = ci * TM, j0t = cj * TN;
    advance();
    if (kc == 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) P[q] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    }
    __syncthreads();   // the previous step's products (and partial sums) are done with LDS
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int slot, row, kk;
      a_rk(q, slot, row, kk);
      const cx<float> va = to_f(ra[q]);
      T* As = base + slot * SLOT;
      As[row * LD + kk] = (T)va.x;
      As[TM * LD + row * LD + kk] = (T)(CONJA ? -va.y : va.y);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int slot, col, kk;
      b_ck(q, slot, col, kk);
      const cx<float> vb = to_f(rb[q]);
      T* Bs = base + slot * SLOT + 2 * TM * LD;
      Bs[col * LD + kk] = (T)vb.x;
      Bs[TN * LD + col * LD + kk] = (T)(CONJB ? -vb.y : vb.y);
    }
    __syncthreads();
    if (s + 1 < steps) fetch();
    const T* AsR = base + kg * SLOT;
    const T* AsI = AsR + TM * LD;
    const T* BsR = AsI + TM * LD;
    const T* BsI = BsR + TN * LD;
    if constexpr (LOW) {
      const int ar = (16 * rbk + li) * LD + 8 * lk, br = (16 * cbk + li) * LD + 8 * lk;
      const bf16x8_t axr = *(const bf16x8_t*)(AsR + ar), axi = *(const bf16x8_t*)(AsI + ar);
      const bf16x8_t bxr = *(const bf16x8_t*)(BsR + br), bxi = *(const bf16x8_t*)(BsI + br);
      P[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(axr, bxr, P[0], 0, 0, 0);
      P[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(axi, bxi, P[1], 0, 0, 0);
      P[2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(axr, bxi, P[2], 0, 0, 0);
      P[2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(axi, bxr, P[2], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int ar = (16 * rbk + li) * LD + kk + lk, br = (16 * cbk + li) * LD + kk + lk;
        const float axr = AsR[ar], axi = AsI[ar], bxr = BsR[br], bxi = BsI[br];
        P[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(axr, bxr, P[0], 0, 0, 0);
        P[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(axi, bxi, P[1], 0, 0, 0);
        P[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(axr + axi, bxr + bxi, P[2], 0, 0, 0);
      }
    }
    if (kc == nks - 1) {
      if constexpr (KS > 1) {   // sum the k-groups' partials into group 0
        float* red = (float*)lds;
        __syncthreads();        // every wave is done reading the tiles
        if (kg > 0) {
#pragma unroll
          for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[(wave * 12 + q * 4 + r) * 64 + lane] = P[q][r];
        }
        __syncthreads();
        if (kg == 0) {
#pragma unroll
          for (int g = 1; g < KS; ++g)
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
              for (int r = 0; r < 4; ++r) P[q][r] += red[((blk + g * NBLK) * 12 + q * 4 + r) * 64 + lane];
        }
      }
      if (kg == 0) {
        const int i0 = i0t, j0 = j0t;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = i0 + 16 * rbk + 4 * lk + r, gj = j0 + 16 * cbk + li;
          const float p0 = P[0][r], p1 = P[1][r], p2 = P[2][r];
          if (gi < m && gj < n) epi(gi, gj, cx<float>{p0 - p1, LOW ? p2 : p2 - p0 - p1});
        }
      }
    }
  }
  __syncthreads();
}

// MFMA product with the tile shape chosen at run time (uniform per workgroup).
// Products with B not conjugated and m <= 64 output rows take a 64-row tile,
// and those of the form op(A) = A^H with m <= 32 the k-split small-row tiles.
template <class T, bool CONJA, bool CONJB, class Epi, class TA, class TB>
__device__ __forceinline__ void mfma_dispatch(int m, int n, int k, const TA* A, long lda,
                                              const TB* B, long ldb, char* tiles, int tile,
                                              Epi&& epi) {
  if constexpr (!CONJB) {
    if (CONJA && m <= 32) {
      if (m <= 16) {
        if (n <= 16)
          block_gemm_mfma_ks<T, 1, 1, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
        else
          block_gemm_mfma_ks<T, 1, 2, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
      } else {
        if (n <= 16)
          block_gemm_mfma_ks<T, 2, 1, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
        else
          block_gemm_mfma_ks<T, 2, 2, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
      }
      return;
    }
    // 64-row tiles: the autotuned 128 x 16 shape would be half padding
    if (m <= 64) tile = (n <= 16) ? 3 : 2;
    if (tile == 3) {
      block_gemm_mfma<T, 3, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
      return;
    }
  }
  if (tile == 1)
    block_gemm_mfma<T, 1, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
  else if (tile == 2)
    block_gemm_mfma<T, 2, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
  else
    block_gemm_mfma<T, 0, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
}

// Channel product dispatch: MFMA for FP32 storage (bfloat16 products when
// lowp; tile: output tile shape, see TileShape), LDS-tiled FMA for FP64.
template <class R, bool CONJA, bool CONJB = false, class Epi>
__device__ __forceinline__ void channel_gemm(int m, int n, int k, const cx<R>* A, long lda,
                                             const cx<R>* B, long ldb, char* tiles, bool lowp,
                                             int tile, Epi&& epi) {
  if constexpr (sizeof(R) == 4) {
    if (lowp)
      mfma_dispatch<__bf16, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, tile, epi);
    else
      mfma_dispatch<float, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, tile, epi);
  } else {
    (void)tile;
    cx<R>* As = (cx<R>*)tiles;
    block_gemm<R, CONJA, CONJB>(m, n, k, A, lda, B, ldb, As, As + KC * (TM + 1), epi);
  }
}

// The same product on the 64 x 64 tile shape only (float products for FP32
// storage), with no per-product choice by size: for kernels whose products
// are all of that shape and whose register budget leaves no room for the
// other variants' code.
template <class R, bool CONJA, bool CONJB = false, class Epi>
__device__ __forceinline__ void channel_gemm64(int m, int n, int k, const cx<R>* A, long lda,
                                               const cx<R>* B, long ldb, char* tiles, Epi&& epi) {
  if constexpr (sizeof(R) == 4) {
    block_gemm_mfma<float, 0, CONJA, CONJB>(m, n, k, A, lda, B, ldb, tiles, epi);
  } else {
    cx<R>* As = (cx<R>*)tiles;
    block_gemm<R, CONJA, CONJB>(m, n, k, A, lda, B, ldb, As, As + KC * (TM + 1), epi);
  }
}

// Mixed-precision products from bfloat16 copies of both operands.
template <bool CONJA, class Epi>
__device__ __forceinline__ void channel_gemm_bf16(int m, int n, int k, const bfc* A, long lda,
                                                  const bfc* B, long ldb, char* tiles, int tile,
                                                  Epi&& epi) {
  mfma_dispatch<__bf16, CONJA, false>(m, n, k, A, lda, B, ldb, tiles, tile, epi);
}

}  // namespace ammse_dev
