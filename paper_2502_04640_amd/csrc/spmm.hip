// Y Q product over the block-tiled dense Q (the Euclidean gradient / Hessian
// product of the local solver and the Lanczos operator of the certificate).
//
// Q is symmetric, so (Y Q)[a][j] = sum_i Q[i][j] Yt[i][a] with Yt = Y^T kept
// frame-major ([3N][r]).  Each workgroup (256 threads) owns a chunk of
// 256*V columns and a slab of rows: every thread streams one 16-byte vector
// of Q per row (V = 2 doubles, 4 floats or 8 bf16), coalesced across the
// wave, and multiplies it by the r values of Yt for that row, which are the
// same for the whole workgroup and staged once in LDS.  Row slabs give enough
// workgroups to fill 256 CUs; their partial sums are added by a second,
// deterministic pass.  Q is read exactly once per product: HBM-bound, with
// 2 r FLOP per stored element.
#include <type_traits>

#include "problem.h"

namespace xm {
namespace {

// Launch shape (tuned on MI355X; see the design notes for the sweep):
//   kTargetBlocks  workgroups the row slabs aim for,
//   kMaxRows       rows of a slab (bounds the LDS staging of Yt),
//   kUnroll        rows in flight per thread.
#ifndef XM_SPMM_TARGET
#define XM_SPMM_TARGET 1024
#endif
#ifndef XM_SPMM_MAXROWS
#define XM_SPMM_MAXROWS 512
#endif
#ifndef XM_SPMM_UNROLL
#define XM_SPMM_UNROLL 8
#endif
constexpr int kB = 256;
constexpr int kMaxRows = XM_SPMM_MAXROWS;
constexpr int kTargetBlocks = XM_SPMM_TARGET;

// Q is streamed once per product.  FP64 Q is read with non-temporal loads
// (measured 7 % faster for the r = 1 product of the certificate); for FP32 Q
// they raise the register count of the r = 5 product past 3 waves per SIMD and
// lose, so FP32 keeps ordinary loads.
template <typename E, int K>
__device__ __forceinline__ void load_nt(const E* p, E (&out)[K]) {
  typedef E vec __attribute__((ext_vector_type(K)));
  const vec v = __builtin_nontemporal_load(reinterpret_cast<const vec*>(p));
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = v[k];
}

template <typename TQ>
struct QVec;
template <>
struct QVec<double> {
  static constexpr int V = 2;
  static constexpr int dtype = XM_F64;
  template <typename TA>
  __device__ static void load(const double* p, TA* out) {
    double v[2];
    load_nt<double, 2>(p, v);
    out[0] = v[0]; out[1] = v[1];
  }
};
template <>
struct QVec<float> {
  static constexpr int V = 4;
  static constexpr int dtype = XM_F32;
  template <typename TA>
  __device__ static void load(const float* p, TA* out) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
  }
};
template <>
struct QVec<uint16_t> {
  static constexpr int V = 8;
  static constexpr int dtype = XM_BF16;
  template <typename TA>
  __device__ static void load(const uint16_t* p, TA* out) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      out[2 * k] = __uint_as_float(w[k] << 16);
      out[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
    }
  }
};

template <typename TQ, typename TV, typename TA, int R>
__global__ __launch_bounds__(kB) void spmm_split_kernel(const TQ* __restrict__ Q, int32_t ld, int32_t n3,
                                                        const TV* __restrict__ Yt, int32_t rows_per_split,
                                                        TA* __restrict__ part) {
  constexpr int V = QVec<TQ>::V;
  __shared__ TA ys[kMaxRows * R];
  const int split = blockIdx.y;
  const int i0 = split * rows_per_split;
  const int i1 = min(n3, i0 + rows_per_split);
  const int nrows = i1 - i0;
  for (int e = threadIdx.x; e < nrows * R; e += kB) ys[e] = static_cast<TA>(Yt[static_cast<int64_t>(i0) * R + e]);
  __syncthreads();
  const int j = (blockIdx.x * kB + threadIdx.x) * V;
  TA acc[V][R];
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int a = 0; a < R; ++a) acc[v][a] = TA(0);
  if (j < ld && nrows > 0) {
    const TQ* q = Q + static_cast<int64_t>(i0) * ld + j;
#pragma unroll XM_SPMM_UNROLL
    for (int i = 0; i < nrows; ++i) {
      TA qv[V];
      QVec<TQ>::load(q + static_cast<int64_t>(i) * ld, qv);
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const TA y = ys[i * R + a];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v][a] += qv[v] * y;
      }
    }
  }
  TA* out = part + static_cast<int64_t>(split) * n3 * R;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    if (j + v < n3) {
#pragma unroll
      for (int a = 0; a < R; ++a) out[static_cast<int64_t>(j + v) * R + a] = acc[v][a];
    }
  }
}

// Upper-triangle tile product.  Grid (chunk c of kB*V columns, slab s of RS
// rows).  colpart[s][j][a] = sum_{i in slab, i <= j} Q[i][j] Yt[i][a];
// rowpart[c][i][a] = sum_{j in chunk, j > i} Q[i][j] Yt[j][a].
//
// Rows are taken in batches of 8.  Lane l holds row b ^ pi(l) of the batch in
// register slot b, pi(l) = (l >> 3) & 7: the butterfly partner of a lane at the
// step with mask 32 (16, 8) then holds, in the slot the lane keeps, the row the
// lane sends, so the three halving steps need no selects.  Within a batch a
// wave still reads 8 whole row segments, each in 128-byte pieces.
//
// Slabs are 256 rows (RS) unless that leaves fewer than kSymMinBlocks
// workgroups on or above the diagonal (a small matrix, e.g. the 10^4-order
// G^{-1} of the factored product); then 128 or 64.  FP32 matrices settle for
// half as many workgroups (each streams twice the values per load; measured
// at N = 10155: 64-row slabs cost the FP32 product more in partial sums than
// they gain in parallelism).
#ifndef XM_SYM_MIN_BLOCKS
#define XM_SYM_MIN_BLOCKS 512
#endif
#ifndef XM_SYM_PERM
#define XM_SYM_PERM 1
#endif
#ifndef XM_SYM_XLANE
#define XM_SYM_XLANE 1
#endif
// cross-lane moves of the butterfly: lane-swap and DPP instructions (no LDS
// traffic), slot b holding row b in every lane
#ifndef XM_SYM_XLANE_F32
#define XM_SYM_XLANE_F32 1
#endif
template <typename TA>
struct SymMode {
  static constexpr bool xlane = XM_SYM_XLANE && (sizeof(TA) == 8 || XM_SYM_XLANE_F32);
  static constexpr bool perm = XM_SYM_PERM && !xlane;  // lane-permuted slots (else selects in the butterfly)
};
#ifndef XM_SYM_BATCH
#define XM_SYM_BATCH 8
#endif
constexpr int kSymBatch = XM_SYM_BATCH;  // rows per butterfly batch: 8 (3 halving steps) or 4 (2)
static_assert(kSymBatch == 8 || (kSymBatch == 4 && XM_SYM_PERM && !XM_SYM_XLANE),
              "batch of 4 rows needs the lane permutation");
constexpr int kSymShift = (kSymBatch == 8) ? 3 : 4;  // lane >> kSymShift selects the row of a lane

// Without the lane permutation the row of every slot is the same for the whole
// wave, so the Yt values of the batch can come from uniform (scalar) loads.
#ifndef XM_SYM_SCALAR_Y
#define XM_SYM_SCALAR_Y 0
#endif
constexpr bool kSymScalarY = XM_SYM_SCALAR_Y && !XM_SYM_PERM && !XM_SYM_XLANE;

// The kSymBatch row segments of a batch (zero where a row is past the slab or,
// in a tile that crosses the diagonal, where all V columns of the lane lie left
// of the row, whose values would be masked to zero anyway).
template <bool kMask, typename TQ, typename TA>
__device__ __forceinline__ void sym_load(const TQ* __restrict__ q, int32_t ld, int i_base, int nb, int pi, int jcol,
                                         TA (&qv)[kSymBatch][QVec<TQ>::V]) {
  constexpr int V = QVec<TQ>::V;
#pragma unroll
  for (int b = 0; b < kSymBatch; ++b) {
    const int row = b ^ pi;
    if (row < nb && (!kMask || jcol + V - 1 >= i_base + row)) {
      QVec<TQ>::load(q + static_cast<int64_t>(row) * ld, qv[b]);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) qv[b][v] = TA(0);
    }
  }
}

template <bool kMask, typename TQ, typename TA, typename TV, int R>
__device__ __forceinline__ void sym_fma(const TA (&qv)[kSymBatch][QVec<TQ>::V], int i_base, int pi, int jcol,
                                        const TA* __restrict__ ys, const TV* __restrict__ Yt, int32_t n3,
                                        const TA (&xc)[QVec<TQ>::V][R], TA (&acc)[QVec<TQ>::V][R],
                                        TA (&p)[kSymBatch][R]) {
  constexpr int V = QVec<TQ>::V;
#pragma unroll
  for (int b = 0; b < kSymBatch; ++b) {
    const int row = b ^ pi;
    const int i = i_base + row;  // global row
#pragma unroll
    for (int a = 0; a < R; ++a) p[b][a] = TA(0);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      TA qc = qv[b][v], qr = qv[b][v];
      if (kMask) {
        qc = (jcol + v >= i) ? qc : TA(0);
        qr = (jcol + v > i) ? qr : TA(0);
      }
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const TA y = kSymScalarY ? static_cast<TA>(Yt[static_cast<int64_t>(min(i, n3 - 1)) * R + a]) : ys[row * R + a];
        acc[v][a] += qc * y;
        p[b][a] += qr * xc[v][a];
      }
    }
  }
}

template <bool kMask, typename TQ, typename TA, typename TV, int R>
__device__ __forceinline__ void sym_batch(const TQ* __restrict__ q, int32_t ld, int i_base, int nb, int pi, int jcol,
                                          const TA* __restrict__ ys, const TV* __restrict__ Yt, int32_t n3,
                                          const TA (&xc)[QVec<TQ>::V][R], TA (&acc)[QVec<TQ>::V][R],
                                          TA (&p)[kSymBatch][R]) {
  constexpr int V = QVec<TQ>::V;
  TA qv[kSymBatch][V];
#pragma unroll
  for (int b = 0; b < kSymBatch; ++b) {
    const int row = b ^ pi;
    // in a tile that crosses the diagonal, a lane whose V columns all lie left
    // of the row loads nothing (its values would be masked to zero below)
    if (row < nb && (!kMask || jcol + V - 1 >= i_base + row)) {
      QVec<TQ>::load(q + static_cast<int64_t>(row) * ld, qv[b]);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) qv[b][v] = TA(0);
    }
  }
#pragma unroll
  for (int b = 0; b < kSymBatch; ++b) {
    const int row = b ^ pi;
    const int i = i_base + row;  // global row
#pragma unroll
    for (int a = 0; a < R; ++a) p[b][a] = TA(0);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      TA qc = qv[b][v], qr = qv[b][v];
      if (kMask) {
        qc = (jcol + v >= i) ? qc : TA(0);
        qr = (jcol + v > i) ? qr : TA(0);
      }
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const TA y = kSymScalarY ? static_cast<TA>(Yt[static_cast<int64_t>(min(i, n3 - 1)) * R + a]) : ys[row * R + a];
        acc[v][a] += qc * y;
        p[b][a] += qr * xc[v][a];
      }
    }
  }
}

// Small matrices (the G^{-1} of the factored product) give about two
// workgroups per CU, too few to hide the latency of each batch's loads behind
// other waves: there the kernel loads the next batch before the arithmetic of
// the current one (kPre), at the price of its registers.  Measured at N = 10155
// (G^{-1} of 10154 rows): FP64 r = 1 (the certificate's Lanczos) 109 -> 86 us,
// FP32 r = 5 68 -> 66 us; FP64 r = 5 loses (163 -> 194 us: the doubled
// registers halve the waves), and so does the 30465-row FP32 Q (389 -> 500 us).
template <typename TQ, int R>
constexpr bool sym_prefetch(int64_t active_blocks) {
  return active_blocks < 1024 && (sizeof(TQ) == 4 || R <= 2);
}

#ifndef XM_SYM_WAVES
#define XM_SYM_WAVES 0
#endif
#if XM_SYM_WAVES > 0
#define XM_SYM_ATTR __attribute__((amdgpu_waves_per_eu(XM_SYM_WAVES)))
#else
#define XM_SYM_ATTR
#endif
// x + (the value of x in the lane at distance 32 / 16), by the lane-swap
// instructions: with X' Y' = swap(X, Y), X' + Y' is X summed over the two
// halves in the lower half (the even rows of 16) and Y summed in the upper
// half (the odd rows), so one swap serves a halving step of the butterfly
template <int D>
__device__ __forceinline__ float xlane_pair_sum(float x, float y) {
  static_assert(D == 16 || D == 32, "lane distance 16 or 32");
  const unsigned a = __builtin_bit_cast(unsigned, x), b = __builtin_bit_cast(unsigned, y);
  unsigned r0, r1;
  if constexpr (D == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    r0 = r[0]; r1 = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    r0 = r[0]; r1 = r[1];
  }
  // the empty asm keeps the two results apart: without it this compiler folds
  // the float view of the pair into r0 + r0 (the integer view is compiled right)
  asm("" : "+v"(r0), "+v"(r1));
  return __builtin_bit_cast(float, r0) + __builtin_bit_cast(float, r1);
}
template <int D>
__device__ __forceinline__ double xlane_pair_sum(double x, double y) {
  static_assert(D == 16 || D == 32, "lane distance 16 or 32");
  const uint64_t a = __builtin_bit_cast(uint64_t, x), b = __builtin_bit_cast(uint64_t, y);
  const unsigned alo = static_cast<unsigned>(a), ahi = static_cast<unsigned>(a >> 32);
  const unsigned blo = static_cast<unsigned>(b), bhi = static_cast<unsigned>(b >> 32);
  unsigned r0lo, r0hi, r1lo, r1hi;
  if constexpr (D == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    r0lo = lo[0]; r1lo = lo[1]; r0hi = hi[0]; r1hi = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    r0lo = lo[0]; r1lo = lo[1]; r0hi = hi[0]; r1hi = hi[1];
  }
  asm("" : "+v"(r0lo), "+v"(r1lo), "+v"(r0hi), "+v"(r1hi));  // as for float
  return __builtin_bit_cast(double, (static_cast<uint64_t>(r0hi) << 32) | r0lo) +
         __builtin_bit_cast(double, (static_cast<uint64_t>(r1hi) << 32) | r1lo);
}
// the value of x in another lane of the same row of 16 (a DPP move; kCtrl one
// of the row permutations below, every lane a valid source)
constexpr int kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
template <int kCtrl>
__device__ __forceinline__ float dpp_get(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, 0xF, 0xF, false));
}
template <int kCtrl>
__device__ __forceinline__ double dpp_get(double x) {
  const uint64_t a = __builtin_bit_cast(uint64_t, x);
  const unsigned lo = static_cast<unsigned>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<unsigned>(a)), kCtrl, 0xF, 0xF, false));
  const unsigned hi = static_cast<unsigned>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<unsigned>(a >> 32)), kCtrl, 0xF, 0xF, false));
  return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

template <typename TQ, typename TV, typename TA, int R, int RS, bool kPre>
__global__ __launch_bounds__(kB) XM_SYM_ATTR void spmm_sym_kernel(const TQ* __restrict__ Q, int32_t ld, int32_t n3,
                                                      const TV* __restrict__ Yt, TA* __restrict__ colpart,
                                                      TA* __restrict__ rowpart) {
  constexpr int V = QVec<TQ>::V;
  constexpr int C = kB * V;
  const int c = blockIdx.x, sl = blockIdx.y;
  const int j0 = c * C;
  const int i0 = sl * RS;
  const int i1 = min(n3, i0 + RS);
  if (j0 + C - 1 < i0) return;  // wholly below the diagonal (uniform per workgroup)
  const int nrows = i1 - i0;
  __shared__ TA ys[RS * R];
  __shared__ TA rp[kB / 64][RS * R];
  // rows past the end of Q stay zero: a ragged last batch multiplies them by zero
  for (int e = threadIdx.x; e < RS * R; e += kB)
    ys[e] = (e < nrows * R) ? static_cast<TA>(Yt[static_cast<int64_t>(i0) * R + e]) : TA(0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr bool kSymXlane = SymMode<TA>::xlane, kSymPerm = SymMode<TA>::perm;
  const int pi = kSymPerm ? (lane >> kSymShift) & (kSymBatch - 1) : 0;
  const int j = j0 + threadIdx.x * V;
  TA xc[V][R];
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int a = 0; a < R; ++a) xc[v][a] = (j + v < n3) ? static_cast<TA>(Yt[static_cast<int64_t>(j + v) * R + a]) : TA(0);
  __syncthreads();
  TA acc[V][R];
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int a = 0; a < R; ++a) acc[v][a] = TA(0);
  const bool crossing = j0 < i1;
  const bool active = j < ld;  // lanes past the padded width read nothing
  const TQ* qbase = Q + static_cast<int64_t>(i0) * ld + (active ? j : 0);
  // kPre: qv holds the current batch, loaded one iteration ahead
  TA qv[kSymBatch][V];
  if (kPre) {
    const int nb = active ? min(kSymBatch, nrows) : 0;
    if (crossing)
      sym_load<true, TQ, TA>(qbase, ld, i0, nb, pi, j, qv);
    else
      sym_load<false, TQ, TA>(qbase, ld, i0, nb, pi, j, qv);
  }
  for (int ib = 0; ib < nrows; ib += kSymBatch) {
    TA p[kSymBatch][R];
    if (kPre) {
      TA qn[kSymBatch][V];
      const int ibn = ib + kSymBatch;
      const int nbn = (active && ibn < nrows) ? min(kSymBatch, nrows - ibn) : 0;
      if (crossing) {
        sym_load<true, TQ, TA>(qbase + static_cast<int64_t>(ibn) * ld, ld, i0 + ibn, nbn, pi, j, qn);
        sym_fma<true, TQ, TA, TV, R>(qv, i0 + ib, pi, j, ys + ib * R, Yt, n3, xc, acc, p);
      } else {
        sym_load<false, TQ, TA>(qbase + static_cast<int64_t>(ibn) * ld, ld, i0 + ibn, nbn, pi, j, qn);
        sym_fma<false, TQ, TA, TV, R>(qv, i0 + ib, pi, j, ys + ib * R, Yt, n3, xc, acc, p);
      }
#pragma unroll
      for (int b = 0; b < kSymBatch; ++b)
#pragma unroll
        for (int v = 0; v < V; ++v) qv[b][v] = qn[b][v];
    } else {
      const int nb = active ? min(kSymBatch, nrows - ib) : 0;
      if (crossing)
        sym_batch<true, TQ, TA, TV, R>(qbase + static_cast<int64_t>(ib) * ld, ld, i0 + ib, nb, pi, j, ys + ib * R,
                                       Yt, n3, xc, acc, p);
      else
        sym_batch<false, TQ, TA, TV, R>(qbase + static_cast<int64_t>(ib) * ld, ld, i0 + ib, nb, pi, j, ys + ib * R,
                                        Yt, n3, xc, acc, p);
    }
    // three halving steps (masks 32, 16, 8) leave row pi, summed over the 8
    // lanes that share the low 3 lane bits; masks 4, 2, 1 finish the wave sum
#pragma unroll
    for (int a = 0; a < R; ++a) {
      TA t4[4], t2[2];
      TA t1;
      if (kSymXlane) {
        // rows 0-3 / 4-7 to the lower / upper 32 lanes, then the even / odd
        // rows of 16, then the two halves of each row of 16 (mirror), each
        // lane keeping row 4 b5 + 2 b4 + b3 of its lane bits; the last three
        // steps sum the 8 lanes that share them
#pragma unroll
        for (int k = 0; k < 4; ++k) t4[k] = xlane_pair_sum<32>(p[k][a], p[k + 4][a]);
#pragma unroll
        for (int k = 0; k < 2; ++k) t2[k] = xlane_pair_sum<16>(t4[k], t4[k + 2]);
        const bool h8 = lane & 8;
        const TA send = h8 ? t2[0] : t2[1], keep = h8 ? t2[1] : t2[0];
        t1 = keep + dpp_get<kDppMirror>(send);
        t1 += dpp_get<kDppHalfMirror>(t1);
        t1 += dpp_get<kDppQuadXor2>(t1);
        t1 += dpp_get<kDppQuadXor1>(t1);
      } else if (kSymBatch == 4) {
#pragma unroll
        for (int k = 0; k < 2; ++k) t2[k] = p[k][a] + __shfl_xor(p[(k + 2) % kSymBatch][a], 32);
        t1 = t2[0] + __shfl_xor(t2[1], 16);
        t1 += __shfl_xor(t1, 8);
      } else if (kSymPerm) {
#pragma unroll
        for (int k = 0; k < 4; ++k) t4[k] = p[k][a] + __shfl_xor(p[(k + 4) % kSymBatch][a], 32);
#pragma unroll
        for (int k = 0; k < 2; ++k) t2[k] = t4[k] + __shfl_xor(t4[k + 2], 16);
        t1 = t2[0] + __shfl_xor(t2[1], 8);
      } else {
        const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          t4[k] = (h32 ? p[(k + 4) % kSymBatch][a] : p[k][a]) +
                  __shfl_xor(h32 ? p[k][a] : p[(k + 4) % kSymBatch][a], 32);
#pragma unroll
        for (int k = 0; k < 2; ++k) t2[k] = (h16 ? t4[k + 2] : t4[k]) + __shfl_xor(h16 ? t4[k] : t4[k + 2], 16);
        t1 = (h8 ? t2[1] : t2[0]) + __shfl_xor(h8 ? t2[0] : t2[1], 8);
      }
      if (!kSymXlane) {
        t1 += __shfl_xor(t1, 4);
        t1 += __shfl_xor(t1, 2);
        t1 += __shfl_xor(t1, 1);
      }
      if ((lane & ((1 << kSymShift) - 1)) == 0) {
        const int lr = kSymXlane ? ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1)
                                 : (lane >> kSymShift) & (kSymBatch - 1);
        const int row = ib + lr;
        if (row < nrows) rp[wave][row * R + a] = t1;
      }
    }
  }
  TA* cp = colpart + static_cast<int64_t>(sl) * n3 * R;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    if (j + v < n3) {
#pragma unroll
      for (int a = 0; a < R; ++a) cp[static_cast<int64_t>(j + v) * R + a] = acc[v][a];
    }
  }
  __syncthreads();
  TA* rpo = rowpart + static_cast<int64_t>(c) * n3 * R + static_cast<int64_t>(i0) * R;
  for (int e = threadIdx.x; e < nrows * R; e += kB) {
    TA sum = rp[0][e];
#pragma unroll
    for (int w = 1; w < kB / 64; ++w) sum += rp[w][e];
    rpo[e] = sum;
  }
}

// out[j][a] = sum_{s <= j / RS} colpart[s][j][a] + sum_{c >= j / C} rowpart[c][j][a]
// 64 outputs per workgroup, 4 threads per output (every 4th partial each),
// the 4 sums added in a fixed order: deterministic.
template <typename TA, typename TV, int R, int C, int RS>
__global__ __launch_bounds__(kB) void spmm_sym_reduce_kernel(const TA* __restrict__ colpart,
                                                             const TA* __restrict__ rowpart, int32_t n3,
                                                             int32_t nchunks, TV* __restrict__ out) {
  __shared__ TA sums[4][64];
  const int64_t m = static_cast<int64_t>(n3) * R;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  TA s = TA(0);
  if (e < m) {
    const int jrow = static_cast<int>(e / R);
    const int smax = jrow / RS;
    for (int k = g; k <= smax; k += 4) s += colpart[static_cast<int64_t>(k) * m + e];
    for (int k = jrow / C + g; k < nchunks; k += 4) s += rowpart[static_cast<int64_t>(k) * m + e];
  }
  sums[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && e < m) {
    const int l = threadIdx.x;
    out[e] = static_cast<TV>((sums[0][l] + sums[1][l]) + (sums[2][l] + sums[3][l]));
  }
}

template <typename TA, typename TV>
__global__ void spmm_reduce_kernel(const TA* __restrict__ part, int32_t splits, int64_t m, TV* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (e >= m) return;
  TA s = TA(0);
  for (int k = 0; k < splits; ++k) s += part[static_cast<int64_t>(k) * m + e];
  out[e] = static_cast<TV>(s);
}

template <typename Ts, typename Td>
__global__ void transpose_rows_kernel(const Ts* __restrict__ in, int32_t rows, int32_t cols, Td* __restrict__ out) {
  // out[c][r] = in[r][c]; one thread per output element
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (e >= static_cast<int64_t>(rows) * cols) return;
  const int64_t c = e / rows, r = e % rows;
  out[e] = static_cast<Td>(in[r * cols + c]);
}

struct Split {
  int32_t splits, rows;
  unsigned col_blocks;
};

Split choose_split(int32_t n3, int32_t ld, int V) {
  Split sp;
  sp.col_blocks = cdiv(ld, static_cast<size_t>(kB) * V);
  const int target = kTargetBlocks;
  int splits = static_cast<int>((target + sp.col_blocks - 1) / sp.col_blocks);
  splits = std::max(1, std::min(splits, static_cast<int>(cdiv(n3, 32))));
  int rows = static_cast<int>(cdiv(n3, splits));
  if (rows > kMaxRows) rows = kMaxRows;
  sp.rows = rows;
  sp.splits = static_cast<int32_t>(cdiv(n3, rows));
  return sp;
}

template <typename TQ, typename TV, typename TA, int R>
void launch(const xm_problem* p, const TQ* Q, const TV* Yt, TV* out, hipStream_t s, Scratch* sc) {
  const Split sp = choose_split(p->n3, p->ld, QVec<TQ>::V);
  TA* part = take<TA>(sc, const_cast<xm_problem*>(p)->spmm_scratch, static_cast<size_t>(sp.splits) * p->n3 * R, s);
  xm_problem::TimedLaunch* ev = nullptr;
  if (p->timing && !(sc && sc->base)) {
    auto* mp = const_cast<xm_problem*>(p);
    if (mp->events_used == mp->events.size()) {
      xm_problem::TimedLaunch t{};
      XM_HIP(hipEventCreate(&t.start));
      XM_HIP(hipEventCreate(&t.stop));
      mp->events.push_back(t);
    }
    ev = &mp->events[mp->events_used++];
    ev->dtype = QVec<TQ>::dtype;
    ev->bytes = static_cast<double>(p->n3) * p->n3 * sizeof(TQ);
    XM_HIP(hipEventRecord(ev->start, s));
  }
  hipLaunchKernelGGL((spmm_split_kernel<TQ, TV, TA, R>), dim3(sp.col_blocks, sp.splits), dim3(kB), 0, s, Q,
                     p->ld, p->n3, Yt, sp.rows, part);
  XM_LAUNCH_CHECK("spmm_split_kernel");
  if (ev) XM_HIP(hipEventRecord(ev->stop, s));
  const int64_t m = static_cast<int64_t>(p->n3) * R;
  hipLaunchKernelGGL((spmm_reduce_kernel<TA, TV>), dim3(cdiv(m, kB)), dim3(kB), 0, s, part, sp.splits, m, out);
  XM_LAUNCH_CHECK("spmm_reduce_kernel");
}

// workgroups of an (nchunks x nslabs) grid that are not wholly below the diagonal
int64_t sym_active_blocks(int32_t n, int32_t ld, int C, int RS) {
  const int nchunks = static_cast<int>(cdiv(ld, C)), nslabs = static_cast<int>(cdiv(n, RS));
  int64_t active = 0;
  for (int c = 0; c < nchunks; ++c) active += std::min<int64_t>(nslabs, (static_cast<int64_t>(c) * C + C - 1) / RS + 1);
  return active;
}

template <typename TQ, typename TV, typename TA, int R, int RS>
void sym_product_rs(const TQ* M, int32_t ld, int32_t n, const TV* Yt, TV* out, DevBuf<char>& scratch,
                    Scratch* sc, xm_problem::TimedLaunch* ev, hipStream_t s) {
  constexpr int V = QVec<TQ>::V;
  constexpr int C = kB * V;
  const int nchunks = static_cast<int>(cdiv(ld, C));
  const int nslabs = static_cast<int>(cdiv(n, RS));
  const size_t per = static_cast<size_t>(n) * R;
  TA* colpart = take<TA>(sc, scratch, (static_cast<size_t>(nslabs) + nchunks) * per, s);
  TA* rowpart = colpart + static_cast<size_t>(nslabs) * per;
  if (ev) XM_HIP(hipEventRecord(ev->start, s));
  const int64_t active = sym_active_blocks(n, ld, C, RS);
  if (sym_prefetch<TQ, R>(active))
    hipLaunchKernelGGL((spmm_sym_kernel<TQ, TV, TA, R, RS, true>), dim3(nchunks, nslabs), dim3(kB), 0, s, M, ld, n,
                       Yt, colpart, rowpart);
  else
    hipLaunchKernelGGL((spmm_sym_kernel<TQ, TV, TA, R, RS, false>), dim3(nchunks, nslabs), dim3(kB), 0, s, M, ld, n,
                       Yt, colpart, rowpart);
  XM_LAUNCH_CHECK("spmm_sym_kernel");
  if (ev) XM_HIP(hipEventRecord(ev->stop, s));
  hipLaunchKernelGGL((spmm_sym_reduce_kernel<TA, TV, R, C, RS>), dim3(cdiv(per, 64)), dim3(kB), 0, s, colpart,
                     rowpart, n, nchunks, out);
  XM_LAUNCH_CHECK("spmm_sym_reduce_kernel");
}

// out (n x R) = M Yt for a symmetric n x n matrix M (row-major, leading
// dimension ld, zero padding columns) read through its upper triangle.
template <typename TQ, typename TV, typename TA, int R>
void sym_product(const TQ* M, int32_t ld, int32_t n, const TV* Yt, TV* out, DevBuf<char>& scratch, Scratch* sc,
                 xm_problem::TimedLaunch* ev, hipStream_t s) {
  constexpr int C = kB * QVec<TQ>::V;
  const int64_t kSymMinBlocks = sizeof(TQ) == 8 ? XM_SYM_MIN_BLOCKS : XM_SYM_MIN_BLOCKS / 2;
  if (sym_active_blocks(n, ld, C, 256) >= kSymMinBlocks)
    sym_product_rs<TQ, TV, TA, R, 256>(M, ld, n, Yt, out, scratch, sc, ev, s);
  else if (sym_active_blocks(n, ld, C, 128) >= kSymMinBlocks)
    sym_product_rs<TQ, TV, TA, R, 128>(M, ld, n, Yt, out, scratch, sc, ev, s);
  else
    sym_product_rs<TQ, TV, TA, R, 64>(M, ld, n, Yt, out, scratch, sc, ev, s);
}

// HIP events around a launch when timing is on (never inside a fixed-scratch
// call, which creates nothing)
xm_problem::TimedLaunch* timed_launch(const xm_problem* p, int dtype, double bytes, const Scratch* sc) {
  if (!p->timing || (sc && sc->base)) return nullptr;
  auto* mp = const_cast<xm_problem*>(p);
  if (mp->events_used == mp->events.size()) {
    xm_problem::TimedLaunch t{};
    XM_HIP(hipEventCreate(&t.start));
    XM_HIP(hipEventCreate(&t.stop));
    mp->events.push_back(t);
  }
  xm_problem::TimedLaunch* ev = &mp->events[mp->events_used++];
  ev->dtype = dtype;
  ev->bytes = bytes;
  return ev;
}

template <typename TQ, typename TV, typename TA, int R>
void launch_sym(const xm_problem* p, const TQ* Q, const TV* Yt, TV* out, hipStream_t s, Scratch* sc) {
  xm_problem::TimedLaunch* ev =
      timed_launch(p, QVec<TQ>::dtype, 0.5 * static_cast<double>(p->n3) * (p->n3 + 1) * sizeof(TQ), sc);
  sym_product<TQ, TV, TA, R>(Q, p->ld, p->n3, Yt, out, const_cast<xm_problem*>(p)->spmm_scratch, sc, ev, s);
}

// ---- factored product: Q = A_rr + B Gm B^T, Gm = -G^{-1} --------------------
// B = A_rt without the column of the anchored frame 0, G the grounded
// Laplacian (Prop. "Scaled-Rotation-Only Formulation", App. A).  Q Yt is formed
// without Q in three passes:
//   1. per frame i: out[i] = sum_{s in row i} A_rr[s] Yt[col s] and
//      W[i-1] = sum_s A_rt[(col s, i)]^T Yt[col s] (i >= 1): both read the same
//      gathered Yt rows, so they share one pass over the co-visibility pattern;
//   2. V = Gm W, the symmetric dense product above on the (N-1)^2 matrix;
//   3. per frame i: out[i] += sum_s A_rt[s] V[col s - 1] (col s >= 1).
// One wavefront per frame, lanes over the frame's co-visible frames; the
// factors are structure of arrays, so every factor load is coalesced across
// the wave (a block-major layout, each lane reading its block's 12 entries in
// 16-byte pieces, measured slower: 0.168 -> 0.187 ms per FP32 r = 5 product);
// Yt is first copied to rows padded to 16 bytes, so that a frame's 3r values
// come in whole 16-byte loads.  Fixed-order wave sums: deterministic.

template <typename T>
struct V16;
template <>
struct V16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int K = 4;
};
template <>
struct V16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int K = 2;
};
template <typename T, int R>
constexpr int padded_row() {
  return (3 * R + V16<T>::K - 1) / V16<T>::K * V16<T>::K;
}

// Ytp[j][e] = Yt[3j + e / R][e % R] for e < 3R, 0 for the padding (Yt in the
// product's precision or, for a mixed product, FP64 rounded here)
template <typename T, int R, typename TS>
__global__ void pad_rows_kernel(const TS* __restrict__ Yt, int32_t N, T* __restrict__ Ytp) {
  constexpr int RP = padded_row<T, R>();
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (e >= static_cast<int64_t>(N) * RP) return;
  const int64_t j = e / RP;
  const int k = static_cast<int>(e - j * RP);
  Ytp[e] = (k < 3 * R) ? static_cast<T>(Yt[j * 3 * R + k]) : T(0);
}

// Each lane takes kFactU blocks of the row per step (64 apart), all their loads
// issued before the arithmetic: the gathers are latency-bound otherwise.
#ifndef XM_FACT_U
#define XM_FACT_U 2
#endif
constexpr int kFactU = XM_FACT_U;
// The factors and their index arrays are streamed once per product with
// non-temporal loads: they then leave the last-level cache to the FP32 G^{-1}
// (206 MB at N = 10155), whose product in the same factored product went from
// 57.7 to 51.5 us.
template <typename E>
__device__ __forceinline__ E fact_ld(const E* p) {
  return __builtin_nontemporal_load(p);
}

// One pass over the co-visibility pattern forms both A_rr Y^T and W = B^T Y^T
// (they share the gather of the padded Yt rows).  The column indices of a
// step's blocks are loaded one step ahead, so a step waits for one round trip
// (its factor loads and its gathers, issued together), not two.
template <typename T, int R>
__global__ __launch_bounds__(kB) void fact_rows_kernel(int32_t N, int64_t S, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const T* __restrict__ fac, const T* __restrict__ Ytp,
                                                       T* __restrict__ out, T* __restrict__ W) {
  constexpr int RP = padded_row<T, R>();
  constexpr int K = V16<T>::K;
  constexpr int NP = Pow2Up<4 * R>::v;
  typedef typename V16<T>::type vec;
  const int i = blockIdx.x * (kB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= N) return;  // whole wavefronts only
  // acc[c * R + a]: (A_rr Y^T)[3i + c][a]; acc[3R + a]: W[i - 1][a]; zero padding up to NP
  T acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = T(0);
  const int32_t beg = row_ptr[i], end = row_ptr[i + 1];
  int32_t cn[kFactU];
#pragma unroll
  for (int u = 0; u < kFactU; ++u) {
    const int32_t s = beg + lane + 64 * u;
    cn[u] = s < end ? fact_ld(col + s) : -1;
  }
  for (int32_t s0 = beg + lane; s0 < end; s0 += 64 * kFactU) {
    int32_t cc[kFactU];
#pragma unroll
    for (int u = 0; u < kFactU; ++u) {
      const int32_t sn = s0 + 64 * (u + kFactU);
      cc[u] = cn[u];
      cn[u] = sn < end ? fact_ld(col + sn) : -1;  // the next step's column, in flight during this one
    }
    T y[kFactU][RP], m[kFactU][9], t[kFactU][3];
#pragma unroll
    for (int u = 0; u < kFactU; ++u) {
      const int32_t s = s0 + 64 * u;
      const bool ok = cc[u] >= 0;  // a block past the row end contributes zero
      const int32_t sc = ok ? s : s0;
      const vec* yp = reinterpret_cast<const vec*>(Ytp + static_cast<int64_t>(ok ? cc[u] : 0) * RP);
#pragma unroll
      for (int q = 0; q < RP / K; ++q) {
        const vec v = yp[q];
#pragma unroll
        for (int k = 0; k < K; ++k) y[u][q * K + k] = v[k];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) m[u][k] = ok ? fact_ld(fac + k * S + sc) : T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) t[u][c] = ok ? fact_ld(fac + (12 + c) * S + sc) : T(0);
    }
#pragma unroll
    for (int u = 0; u < kFactU; ++u)
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int a = 0; a < R; ++a) {
          const T yv = y[u][d * R + a];
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[c * R + a] += m[u][3 * c + d] * yv;
          acc[3 * R + a] += t[u][d] * yv;
        }
  }
  // the 4R sums, each lane writing the one it holds
  const T v = group_split_sum<NP, 64>(acc, lane);
  const int q = group_split_index<NP, 64>(lane);
  if ((lane & (64 / NP - 1)) == 0) {
    if (q < 3 * R) out[3 * static_cast<int64_t>(i) * R + q] = v;
    else if (q < 4 * R && i > 0) W[static_cast<int64_t>(i - 1) * R + (q - 3 * R)] = v;
  }
}

// out[i] = part[i] + sum_s A_rt[s] V[col s - 1] (part: pass 1's result; the
// same array as out unless a mixed product widens to FP64 here), the column
// indices one step ahead as above
template <typename T, int R, typename TO>
__global__ __launch_bounds__(kB) void fact_cols_kernel(int32_t N, int64_t S, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const T* __restrict__ fac, const T* __restrict__ V,
                                                       const T* part, TO* out) {
  constexpr int NP = Pow2Up<3 * R>::v;
  const int i = blockIdx.x * (kB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= N) return;  // whole wavefronts only
  T acc[NP];  // acc[c * R + a]: out[3i + c][a]; zero padding up to NP
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = T(0);
  const int32_t beg = row_ptr[i], end = row_ptr[i + 1];
  int32_t cn[kFactU];
#pragma unroll
  for (int u = 0; u < kFactU; ++u) {
    const int32_t s = beg + lane + 64 * u;
    cn[u] = s < end ? fact_ld(col + s) : 0;
  }
  for (int32_t s0 = beg + lane; s0 < end; s0 += 64 * kFactU) {
    int32_t cc[kFactU];
#pragma unroll
    for (int u = 0; u < kFactU; ++u) {
      const int32_t sn = s0 + 64 * (u + kFactU);
      cc[u] = cn[u];
      cn[u] = sn < end ? fact_ld(col + sn) : 0;
    }
    T v[kFactU][R], b[kFactU][3];
#pragma unroll
    for (int u = 0; u < kFactU; ++u) {
      const int32_t s = s0 + 64 * u;
      const int j = cc[u];
      const bool ok = j > 0;  // frame 0 is anchored (no column of B); past the end: zero
      const T* vp = V + static_cast<int64_t>(ok ? j - 1 : 0) * R;
#pragma unroll
      for (int a = 0; a < R; ++a) v[u][a] = vp[a];
#pragma unroll
      for (int c = 0; c < 3; ++c) b[u][c] = ok ? fact_ld(fac + (9 + c) * S + s) : T(0);
    }
#pragma unroll
    for (int u = 0; u < kFactU; ++u)
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c * R + a] += b[u][c] * v[u][a];
  }
  const T v = group_split_sum<NP, 64>(acc, lane);
  const int q = group_split_index<NP, 64>(lane);
  if ((lane & (64 / NP - 1)) == 0 && q < 3 * R) {
    const int64_t o = 3 * static_cast<int64_t>(i) * R + q;
    out[o] = static_cast<TO>(part[o] + v);
  }
}

// Grouped form of passes 1 and 3, used when the frame groups' unions fit in
// LDS.  The frames are taken in groups of kFactGroup consecutive in the
// Cuthill-McKee order of the co-visibility graph (the groups of the assembly's
// correction products); one workgroup per group, one wavefront per frame.  The
// group's co-visible frames (its union, which the assembly lists) are staged
// in LDS once, so each gathered row comes from LDS: on clustered scenes a
// group's union holds about a quarter of its blocks' rows, and the gathers
// otherwise dominate the requests from the vector caches to L2, which bound
// these passes.  lidx[s] is the position of block s's column in its row's
// group union (-1 for the anchored frame 0, staged after the union in pass 1
// and without a column of B in pass 3).
constexpr int kFactGroup = kFrameGroup;
constexpr int kFactGroupThreads = 64 * kFactGroup;

template <typename T, int R, typename TS>
__global__ __launch_bounds__(kFactGroupThreads) void fact_rows_group_kernel(
    int32_t N, int64_t S, const int32_t* __restrict__ order, const int64_t* __restrict__ ustart,
    const int32_t* __restrict__ uid, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ lidx,
    const T* __restrict__ fac, const TS* __restrict__ Yt, T* __restrict__ out, T* __restrict__ W) {
  constexpr int RP = padded_row<T, R>();
  constexpr int K = V16<T>::K;
  constexpr int NP = Pow2Up<4 * R>::v;
  typedef typename V16<T>::type vec;
  extern __shared__ __align__(16) unsigned char fact_smem[];
  T* ys = reinterpret_cast<T*>(fact_smem);  // [U + 1][RP]: the union's Yt rows, then frame 0's
  const int g = blockIdx.x;
  const int64_t u0 = ustart[g];
  const int U = static_cast<int>(ustart[g + 1] - u0);
  for (int e = threadIdx.x; e < (U + 1) * RP; e += kFactGroupThreads) {
    const int k = e / RP, q = e - k * RP;
    const int j = (k < U) ? uid[u0 + k] : 0;
    ys[e] = (q < 3 * R) ? static_cast<T>(Yt[static_cast<int64_t>(j) * 3 * R + q]) : T(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int a = g * kFactGroup + (threadIdx.x >> 6);
  if (a >= N) return;  // whole wavefronts, after the only barrier
  const int i = order[a];
  T acc[NP];  // as in fact_rows_kernel
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = T(0);
  const int32_t beg = row_ptr[i], end = row_ptr[i + 1];
  for (int32_t s0 = beg + lane; s0 < end; s0 += 64 * kFactU) {
    int32_t lk[kFactU];
    T m[kFactU][9], t[kFactU][3];
#pragma unroll
    for (int u = 0; u < kFactU; ++u) {
      const int32_t s = s0 + 64 * u;
      const bool ok = s < end;  // a block past the row end contributes zero
      const int32_t sc = ok ? s : s0;
      lk[u] = fact_ld(lidx + sc);
#pragma unroll
      for (int k = 0; k < 9; ++k) m[u][k] = ok ? fact_ld(fac + k * S + sc) : T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) t[u][c] = ok ? fact_ld(fac + (12 + c) * S + sc) : T(0);
    }
#pragma unroll
    for (int u = 0; u < kFactU; ++u) {
      const vec* yp = reinterpret_cast<const vec*>(ys + (lk[u] >= 0 ? lk[u] : U) * RP);
      T y[RP];
#pragma unroll
      for (int q = 0; q < RP / K; ++q) {
        const vec v = yp[q];
#pragma unroll
        for (int k = 0; k < K; ++k) y[q * K + k] = v[k];
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int b = 0; b < R; ++b) {
          const T yv = y[d * R + b];
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[c * R + b] += m[u][3 * c + d] * yv;
          acc[3 * R + b] += t[u][d] * yv;
        }
    }
  }
  const T v = group_split_sum<NP, 64>(acc, lane);
  const int q = group_split_index<NP, 64>(lane);
  if ((lane & (64 / NP - 1)) == 0) {
    if (q < 3 * R) out[3 * static_cast<int64_t>(i) * R + q] = v;
    else if (q < 4 * R && i > 0) W[static_cast<int64_t>(i - 1) * R + (q - 3 * R)] = v;
  }
}

template <typename T, int R, typename TO>
__global__ __launch_bounds__(kFactGroupThreads) void fact_cols_group_kernel(
    int32_t N, int64_t S, const int32_t* __restrict__ order, const int64_t* __restrict__ ustart,
    const int32_t* __restrict__ uid, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ lidx,
    const T* __restrict__ fac, const T* __restrict__ V, const T* part, TO* out) {
  constexpr int NP = Pow2Up<3 * R>::v;
  extern __shared__ __align__(16) unsigned char fact_smem[];
  T* vs = reinterpret_cast<T*>(fact_smem);  // [U][R]: V rows of the union (all its frames are >= 1)
  const int g = blockIdx.x;
  const int64_t u0 = ustart[g];
  const int U = static_cast<int>(ustart[g + 1] - u0);
  for (int e = threadIdx.x; e < U * R; e += kFactGroupThreads) {
    const int k = e / R, b = e - k * R;
    vs[e] = V[static_cast<int64_t>(uid[u0 + k] - 1) * R + b];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int a = g * kFactGroup + (threadIdx.x >> 6);
  if (a >= N) return;  // whole wavefronts, after the only barrier
  const int i = order[a];
  T acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = T(0);
  const int32_t beg = row_ptr[i], end = row_ptr[i + 1];
  for (int32_t s0 = beg + lane; s0 < end; s0 += 64 * kFactU) {
    int32_t lk[kFactU];
    T bb[kFactU][3];
#pragma unroll
    for (int u = 0; u < kFactU; ++u) {
      const int32_t s = s0 + 64 * u;
      const bool ok = s < end;
      const int32_t sc = ok ? s : s0;
      lk[u] = ok ? fact_ld(lidx + sc) : -1;  // -1: past the row end, or frame 0 (no column of B)
#pragma unroll
      for (int c = 0; c < 3; ++c) bb[u][c] = ok ? fact_ld(fac + (9 + c) * S + sc) : T(0);
    }
#pragma unroll
    for (int u = 0; u < kFactU; ++u) {
      const bool ok = lk[u] >= 0;
      const T* vp = vs + (ok ? lk[u] : 0) * R;
#pragma unroll
      for (int b = 0; b < R; ++b) {
        const T vv = ok ? vp[b] : T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c * R + b] += bb[u][c] * vv;
      }
    }
  }
  const T v = group_split_sum<NP, 64>(acc, lane);
  const int q = group_split_index<NP, 64>(lane);
  if ((lane & (64 / NP - 1)) == 0 && q < 3 * R) {
    const int64_t o = 3 * static_cast<int64_t>(i) * R + q;
    out[o] = static_cast<TO>(part[o] + v);
  }
}

// the factors of one precision: the sparse blocks (structure of arrays) and -G^{-1}
template <typename T>
struct Factors {
  const T *fac, *Gm;
};
Factors<double> factors(const xm_problem* p, double*) { return {p->fac.ptr, p->Gm.ptr}; }
Factors<float> factors(const xm_problem* p, float*) {
  require(p->fac32.ptr != nullptr, XM_EINVAL, "the FP32 factors were not kept (XM_KEEP_F32)");
  return {p->fac32.ptr, p->Gm32.ptr};
}

// doubles of the factored product's own temporaries (padded Yt, W, V)
size_t factored_scratch_doubles(int32_t N) { return 24 * static_cast<size_t>(N) + 16 * static_cast<size_t>(N - 1); }

// bytes of the partial sums of sym_product for an n x n matrix, value size b,
// accumulator size a (the slab height it would choose)
size_t sym_scratch_bytes(int32_t n, int32_t ld, int V, size_t a, int R) {
  const int C = kB * V;
  const int64_t kSymMinBlocks = V == 2 ? XM_SYM_MIN_BLOCKS : XM_SYM_MIN_BLOCKS / 2;
  int RS = 64;
  if (sym_active_blocks(n, ld, C, 256) >= kSymMinBlocks) RS = 256;
  else if (sym_active_blocks(n, ld, C, 128) >= kSymMinBlocks) RS = 128;
  const size_t nchunks = cdiv(ld, C), nslabs = cdiv(n, RS);
  return (nslabs + nchunks) * static_cast<size_t>(n) * R * a;
}

// TIO: the type of Yt and out; a mixed product (FP64 vectors, FP32 factors)
// rounds Yt in pass 1 and widens the result in pass 3, with pass 1's result
// in `part` (FP32, 3N x R), instead of converting both vectors separately.
template <typename T, int R, typename TIO>
void launch_factored(const xm_problem* p, const TIO* Yt, TIO* out, hipStream_t s, Scratch* sc, T* part) {
  auto* mp = const_cast<xm_problem*>(p);
  const Factors<T> f = factors(p, static_cast<T*>(nullptr));
  const int32_t N = p->N, ng = N - 1;
  constexpr int RP = padded_row<T, R>();
  // scratch, in doubles: padded Yt (N rows of at most 24 values), W, V (ng x 8 each)
  double* base = take<double>(sc, mp->fact_scratch, factored_scratch_doubles(N), s);
  T* Ytp = reinterpret_cast<T*>(base);
  T* W = reinterpret_cast<T*>(base + 24 * static_cast<size_t>(N));
  T* Vv = W + static_cast<size_t>(ng) * R;
  const int64_t S = p->nnzb;
  xm_problem::TimedLaunch* ev =
      timed_launch(p, sizeof(T) == 8 ? XM_STATS_FACTORED : XM_STATS_FACTORED + 1,
                   (0.5 * static_cast<double>(ng) * (ng + 1) + static_cast<double>(S) * 15.0) * sizeof(T), sc);
  if (ev) XM_HIP(hipEventRecord(ev->start, s));
  // each pass grouped when the largest group union (and, for pass 1, frame 0's
  // row) fits in half the LDS a workgroup may take: with one workgroup per CU
  // nothing overlaps its staging, and pass 1 at r = 5 in FP32 (145 KB at
  // N = 10155) measured slower grouped (66 against 53 us)
  const size_t lds_rows = (static_cast<size_t>(std::max(p->grp_maxu, 0)) + 1) * RP * sizeof(T);
  const size_t lds_cols = static_cast<size_t>(std::max(p->grp_maxu, 1)) * R * sizeof(T);
  const bool grouped_rows = p->grp_maxu >= 0 && lds_rows <= p->lds_max / 2;
  const bool grouped_cols = p->grp_maxu >= 0 && lds_cols <= p->lds_max / 2;
  const unsigned ngroups = cdiv(N, kFactGroup);
  const unsigned gb = cdiv(N, kB / 64);
  // bytes of pass 1: the 12 factor values and the index of every block, each
  // Y^T row once (the staged union rows when grouped), A_rr Y^T and W written
  const double rows_bytes =
      static_cast<double>(S) * (12.0 * sizeof(T) + 4.0) +
      (grouped_rows ? static_cast<double>(p->grp_uid.n + ngroups) * 3 * R * sizeof(T)
                    : static_cast<double>(N) * RP * sizeof(T)) +
      (3.0 * N + (N - 1)) * R * sizeof(T);
  xm_problem::TimedLaunch* evr =
      timed_launch(p, sizeof(T) == 8 ? XM_STATS_FACT_ROWS : XM_STATS_FACT_ROWS + 1, rows_bytes, sc);
  if (!grouped_rows) {
    hipLaunchKernelGGL((pad_rows_kernel<T, R, TIO>), dim3(cdiv(static_cast<size_t>(N) * RP, kB)), dim3(kB), 0, s, Yt,
                       N, Ytp);
    XM_LAUNCH_CHECK("pad_rows_kernel");
  }
  if (evr) XM_HIP(hipEventRecord(evr->start, s));
  if (grouped_rows) {
    hipLaunchKernelGGL((fact_rows_group_kernel<T, R, TIO>), dim3(ngroups), dim3(kFactGroupThreads), lds_rows, s, N,
                       S, p->order.ptr, p->grp_ustart.ptr, p->grp_uid.ptr, p->row_ptr.ptr, p->lidx.ptr, f.fac, Yt,
                       part, W);
    XM_LAUNCH_CHECK("fact_rows_group_kernel");
  } else {
    hipLaunchKernelGGL((fact_rows_kernel<T, R>), dim3(gb), dim3(kB), 0, s, N, S, p->row_ptr.ptr, p->col.ptr, f.fac,
                       Ytp, part, W);
    XM_LAUNCH_CHECK("fact_rows_kernel");
  }
  if (evr) XM_HIP(hipEventRecord(evr->stop, s));
  xm_problem::TimedLaunch* evg = timed_launch(p, sizeof(T) == 8 ? XM_STATS_GINV : XM_STATS_GINV + 1,
                                              0.5 * static_cast<double>(ng) * (ng + 1) * sizeof(T), sc);
  sym_product<T, T, T, R>(f.Gm, p->ldg, ng, W, Vv, mp->spmm_scratch, sc, evg, s);
  if (grouped_cols) {
    hipLaunchKernelGGL((fact_cols_group_kernel<T, R, TIO>), dim3(ngroups), dim3(kFactGroupThreads), lds_cols, s, N,
                       S, p->order.ptr, p->grp_ustart.ptr, p->grp_uid.ptr, p->row_ptr.ptr, p->lidx.ptr, f.fac, Vv,
                       part, out);
    XM_LAUNCH_CHECK("fact_cols_group_kernel");
  } else {
    hipLaunchKernelGGL((fact_cols_kernel<T, R, TIO>), dim3(gb), dim3(kB), 0, s, N, S, p->row_ptr.ptr, p->col.ptr,
                       f.fac, Vv, part, out);
    XM_LAUNCH_CHECK("fact_cols_kernel");
  }
  if (ev) XM_HIP(hipEventRecord(ev->stop, s));
}

// part: pass 1's result for a mixed product (T other than TIO); else out serves
template <typename T, typename TIO = T>
void dispatch_factored(const xm_problem* p, const TIO* Yt, int r, TIO* out, hipStream_t s, Scratch* sc,
                       T* part = nullptr) {
  if constexpr (std::is_same<T, TIO>::value) part = out;
  switch (r) {
    case 1: launch_factored<T, 1, TIO>(p, Yt, out, s, sc, part); return;
    case 2: launch_factored<T, 2, TIO>(p, Yt, out, s, sc, part); return;
    case 3: launch_factored<T, 3, TIO>(p, Yt, out, s, sc, part); return;
    case 4: launch_factored<T, 4, TIO>(p, Yt, out, s, sc, part); return;
    case 5: launch_factored<T, 5, TIO>(p, Yt, out, s, sc, part); return;
    case 6: launch_factored<T, 6, TIO>(p, Yt, out, s, sc, part); return;
    case 7: launch_factored<T, 7, TIO>(p, Yt, out, s, sc, part); return;
    case 8: launch_factored<T, 8, TIO>(p, Yt, out, s, sc, part); return;
    default: throw Error(XM_EINVAL, "rank must be in [1, 8]");
  }
}

// out[a][e] = in[map[a]][e] over N rows of w values: with map = order it takes
// a frame-major array into the frame order, with map = pos back out of it
template <typename T>
__global__ void permute_frames_kernel(const T* __restrict__ in, const int32_t* __restrict__ map, int32_t N, int w,
                                      T* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (e >= static_cast<int64_t>(N) * w) return;
  const int64_t a = e / w;
  out[e] = in[static_cast<int64_t>(map[a]) * w + (e - a * w)];
}

template <typename TQ, typename TV, typename TA>
void dispatch_r_ordered(const xm_problem* p, const TQ* Q, const TV* Yt, int r, TV* out, hipStream_t s, int role,
                        Scratch* sc) {
  if (p->spmm_kind[role][QVec<TQ>::dtype] == XM_SPMM_UPPER) {
    switch (r) {
      case 1: launch_sym<TQ, TV, TA, 1>(p, Q, Yt, out, s, sc); return;
      case 2: launch_sym<TQ, TV, TA, 2>(p, Q, Yt, out, s, sc); return;
      case 3: launch_sym<TQ, TV, TA, 3>(p, Q, Yt, out, s, sc); return;
      case 4: launch_sym<TQ, TV, TA, 4>(p, Q, Yt, out, s, sc); return;
      case 5: launch_sym<TQ, TV, TA, 5>(p, Q, Yt, out, s, sc); return;
      case 6: launch_sym<TQ, TV, TA, 6>(p, Q, Yt, out, s, sc); return;
      case 7: launch_sym<TQ, TV, TA, 7>(p, Q, Yt, out, s, sc); return;
      case 8: launch_sym<TQ, TV, TA, 8>(p, Q, Yt, out, s, sc); return;
      default: throw Error(XM_EINVAL, "rank must be in [1, 8]");
    }
  }
  switch (r) {
    case 1: launch<TQ, TV, TA, 1>(p, Q, Yt, out, s, sc); break;
    case 2: launch<TQ, TV, TA, 2>(p, Q, Yt, out, s, sc); break;
    case 3: launch<TQ, TV, TA, 3>(p, Q, Yt, out, s, sc); break;
    case 4: launch<TQ, TV, TA, 4>(p, Q, Yt, out, s, sc); break;
    case 5: launch<TQ, TV, TA, 5>(p, Q, Yt, out, s, sc); break;
    case 6: launch<TQ, TV, TA, 6>(p, Q, Yt, out, s, sc); break;
    case 7: launch<TQ, TV, TA, 7>(p, Q, Yt, out, s, sc); break;
    case 8: launch<TQ, TV, TA, 8>(p, Q, Yt, out, s, sc); break;
    default: throw Error(XM_EINVAL, "rank must be in [1, 8]");
  }
}

// The stored Q is in the frame order (that of the assembly): Yt goes into that
// order, the product is taken there, and its rows come back to frame order.
template <typename TQ, typename TV, typename TA>
void dispatch_r(const xm_problem* p, const TQ* Q, const TV* Yt, int r, TV* out, hipStream_t s, int role,
                Scratch* sc) {
  require(r >= 1 && r <= 8, XM_EINVAL, "rank must be in [1, 8]");
  auto* mp = const_cast<xm_problem*>(p);
  const int32_t N = p->N;
  const int w = 3 * r;
  const size_t n = static_cast<size_t>(N) * w;
  TV* Yp = take<TV>(sc, mp->perm_scratch, 2 * n, s);  // two [N][3r] arrays
  TV* Op = Yp + n;
  hipLaunchKernelGGL((permute_frames_kernel<TV>), dim3(cdiv(n, kB)), dim3(kB), 0, s, Yt, p->order.ptr, N, w, Yp);
  XM_LAUNCH_CHECK("permute_frames_kernel");
  dispatch_r_ordered<TQ, TV, TA>(p, Q, Yp, r, Op, s, role, sc);
  hipLaunchKernelGGL((permute_frames_kernel<TV>), dim3(cdiv(n, kB)), dim3(kB), 0, s, Op, p->pos.ptr, N, w, out);
  XM_LAUNCH_CHECK("permute_frames_kernel");
}

}  // namespace

template <>
void spmm_yt<float>(const xm_problem* p, xm_dtype qtype, const float* Yt, int r, float* out, hipStream_t s,
                    int role, Scratch* sc);

template <>
void spmm_yt<double>(const xm_problem* p, xm_dtype qtype, const double* Yt, int r, double* out, hipStream_t s,
                     int role, Scratch* sc) {
  require(role == XM_ROLE_RESIDUAL || role == XM_ROLE_CURVATURE, XM_EINVAL, "unknown product role");
  if (qtype != XM_F64) {
    // FP64 vectors with a reduced-precision Q (the truncated-CG products of the
    // FP64 stage of a reduced-precision solve): rounded to FP32, multiplied
    // with FP32 accumulation, widened back
    require(r >= 1 && r <= 8, XM_EINVAL, "rank must be in [1, 8]");
    auto* mp = const_cast<xm_problem*>(p);
    const size_t n = static_cast<size_t>(p->n3) * r;
    float* a = take<float>(sc, mp->mixed_scratch, 2 * n, s);
    if (qtype == XM_F32 && p->spmm_kind[role][XM_F32] == XM_SPMM_FACTORED) {
      // the factored passes round and widen themselves (bitwise the same result)
      dispatch_factored<float, double>(p, Yt, r, out, s, sc, a);
      return;
    }
    float* b = a + n;
    transpose_rows<double, float>(Yt, 1, static_cast<int>(n), a, s);
    spmm_yt<float>(p, qtype, a, r, b, s, role, sc);
    transpose_rows<float, double>(b, 1, static_cast<int>(n), out, s);
    return;
  }
  if (p->spmm_kind[role][XM_F64] == XM_SPMM_FACTORED) {
    dispatch_factored<double>(p, Yt, r, out, s, sc);
    return;
  }
  require(p->Q64.ptr != nullptr, XM_EINVAL, "the dense FP64 Q was not kept");
  dispatch_r<double, double, double>(p, p->Q64.ptr, Yt, r, out, s, role, sc);
}

template <>
void spmm_yt<float>(const xm_problem* p, xm_dtype qtype, const float* Yt, int r, float* out, hipStream_t s,
                    int role, Scratch* sc) {
  require(role == XM_ROLE_RESIDUAL || role == XM_ROLE_CURVATURE, XM_EINVAL, "unknown product role");
  if (qtype == XM_F32 && p->spmm_kind[role][XM_F32] == XM_SPMM_FACTORED) {
    dispatch_factored<float>(p, Yt, r, out, s, sc);
    return;
  }
  if (qtype == XM_F32) {
    require(p->Q32.ptr != nullptr, XM_EINVAL, "the FP32 copy of Q was not kept (XM_KEEP_F32)");
    dispatch_r<float, float, float>(p, p->Q32.ptr, Yt, r, out, s, role, sc);
  } else if (qtype == XM_BF16) {
    require(p->Q16.ptr != nullptr, XM_EINVAL, "the BF16 copy of Q was not kept (XM_KEEP_BF16)");
    dispatch_r<uint16_t, float, float>(p, p->Q16.ptr, Yt, r, out, s, role, sc);
  } else {
    throw Error(XM_EINVAL, "FP32 vectors are multiplied with the FP32 or BF16 Q");
  }
}

size_t product_scratch_bytes(const xm_problem* p, xm_dtype qtype, int r, int role, bool fp64_vectors) {
  require(r >= 1 && r <= 8, XM_EINVAL, "rank must be in [1, 8]");
  require(role == XM_ROLE_RESIDUAL || role == XM_ROLE_CURVATURE, XM_EINVAL, "unknown product role");
  require(qtype == XM_F64 || qtype == XM_F32 || qtype == XM_BF16, XM_EINVAL, "unknown dtype");
  constexpr size_t kAlign = 256;  // worst-case padding of one take()
  size_t total = 0;
  if (fp64_vectors && qtype != XM_F64) total += 2 * static_cast<size_t>(p->n3) * r * sizeof(float) + kAlign;
  const int kind = p->spmm_kind[role][qtype];
  const size_t vb = (qtype == XM_F64) ? 8 : 4;  // vector and accumulator size
  if (kind == XM_SPMM_FACTORED && qtype != XM_BF16) {
    total += factored_scratch_doubles(p->N) * sizeof(double) + kAlign;
    total += sym_scratch_bytes(p->N - 1, p->ldg, qtype == XM_F64 ? 2 : 4, vb, r) + kAlign;
    return total;
  }
  total += 2 * static_cast<size_t>(p->N) * 3 * r * vb + kAlign;
  const int V = (qtype == XM_F64) ? 2 : (qtype == XM_F32 ? 4 : 8);
  if (kind == XM_SPMM_UPPER) {
    total += sym_scratch_bytes(p->n3, p->ld, V, vb, r) + kAlign;
  } else {
    const Split sp = choose_split(p->n3, p->ld, V);
    total += static_cast<size_t>(sp.splits) * p->n3 * r * vb + kAlign;
  }
  return total;
}

template <typename Ts, typename Td>
void transpose_rows(const Ts* in, int rows, int cols, Td* out, hipStream_t s) {
  const int64_t m = static_cast<int64_t>(rows) * cols;
  if (m == 0) return;
  hipLaunchKernelGGL((transpose_rows_kernel<Ts, Td>), dim3(cdiv(m, kB)), dim3(kB), 0, s, in, rows, cols, out);
  XM_LAUNCH_CHECK("transpose_rows_kernel");
}

template void transpose_rows<double, double>(const double*, int, int, double*, hipStream_t);
template void transpose_rows<double, float>(const double*, int, int, float*, hipStream_t);
template void transpose_rows<float, double>(const float*, int, int, double*, hipStream_t);
template void transpose_rows<float, float>(const float*, int, int, float*, hipStream_t);

}  // namespace xm
