// Assembly of the rotation-only data matrix Q (Prop. "Scaled-Rotation-Only
// Formulation", App. A) on the GPU, in FP64.
//
// With h = [u; 1], the SBA cost of one landmark k with observations O_k and
// total weight W_k = sum w, minimised over p_k, is
//   sum_{o,o' in O_k} (delta_oo' w_o - w_o w_o' / W_k) x_{i(o)} h_o . x_{i(o')} h_o'
// for x_i = [Y_i, t_i] (r x 4).  Every ordered observation pair of a landmark
// therefore adds a 4x4 block to the frame pair (i(o), i(o')) of a 4N x 4N
// matrix H; its rotation part is A_rr, its mixed part A_rt and its
// translation part the weighted co-visibility Laplacian A_tt.  The
// translations are then removed with frame 0 grounded:
//   Q = A_rr - A_rt[:,1:] A_tt[1:,1:]^{-1} A_rt[:,1:]^T.
//
// GPU steps (no global atomics; the reduction order is fixed, so Q is
// bitwise reproducible):
//   validate -> radix-sort observations by landmark -> per-landmark weight
//   and pair counts -> emit (frame pair key, observation pair) for every
//   ordered pair -> radix-sort by key -> one wavefront per distinct frame
//   pair sums its 4x4 contributions (lane-strided, butterfly reduction) and
//   writes the A_rr block into Q, the A_rt / A_tt entries into the sparse
//   pattern -> dense grounded Laplacian G -> in-place block sweep
//   (Gauss-Jordan) to -G^{-1} -> P = A_rt G^{-1} and Q -= P A_rt^T by two
//   sparse-row x dense products -> symmetrise -> tr(Q) -> FP32/BF16 copies.
#include <hip/hip_runtime.h>

#include <cmath>

#include "problem.h"

namespace xm {
namespace {

constexpr int kB = 256;

// ---------------------------------------------------------------------------
__global__ void validate_kernel(int32_t N, int32_t M, int64_t n, const int32_t* __restrict__ frame,
                                const int32_t* __restrict__ landmark, const void* __restrict__ u,
                                int u_f32, const void* __restrict__ w, int w_f32, int* flags) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (e >= n) return;
  const int32_t f = frame[e], l = landmark[e];
  if (f < 0 || f >= N || l < 0 || l >= M) flags[0] = 1;
  double a, b, c;
  if (u_f32) {
    const float* uf = static_cast<const float*>(u);
    a = uf[3 * e]; b = uf[3 * e + 1]; c = uf[3 * e + 2];
  } else {
    const double* ud = static_cast<const double*>(u);
    a = ud[3 * e]; b = ud[3 * e + 1]; c = ud[3 * e + 2];
  }
  if (!isfinite(a) || !isfinite(b) || !isfinite(c)) flags[1] = 1;
  if (w) {
    const double wv = w_f32 ? static_cast<double>(static_cast<const float*>(w)[e])
                            : static_cast<const double*>(w)[e];
    if (!(wv > 0.0) || !isfinite(wv)) flags[2] = 1;
  }
}

// sort keys: the landmark of each observation, or M (past every landmark, so
// that masked-out observations sort to the end) where mask[e] == 0
__global__ void iota_kernel(const int32_t* __restrict__ landmark, const uint8_t* __restrict__ mask, int32_t M,
                            int64_t n, uint32_t* keys, uint64_t* vals) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (e >= n) return;
  keys[e] = (mask && !mask[e]) ? static_cast<uint32_t>(M) : static_cast<uint32_t>(landmark[e]);
  vals[e] = static_cast<uint64_t>(e);
}

// number of observations kept by the mask (integer sum: order-independent)
__global__ void count_kept_kernel(const uint8_t* __restrict__ mask, int64_t n, unsigned long long* count) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  const bool k = e < n && mask[e] != 0;
  const unsigned long long b = __ballot(k);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, static_cast<unsigned long long>(__popcll(b)));
}

__global__ void gather_obs_kernel(const uint64_t* __restrict__ order, int64_t n,
                                  const int32_t* __restrict__ frame, const int32_t* __restrict__ landmark,
                                  const void* __restrict__ u, int u_f32, const void* __restrict__ w,
                                  int w_f32, int32_t* fr_s, int32_t* lm_s, double* u_s, double* w_s,
                                  int64_t* perm) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (p >= n) return;
  const int64_t o = static_cast<int64_t>(order[p]);
  perm[p] = o;
  fr_s[p] = frame[o];
  lm_s[p] = landmark[o];
  if (u_f32) {
    const float* uf = static_cast<const float*>(u);
    u_s[3 * p] = uf[3 * o]; u_s[3 * p + 1] = uf[3 * o + 1]; u_s[3 * p + 2] = uf[3 * o + 2];
  } else {
    const double* ud = static_cast<const double*>(u);
    u_s[3 * p] = ud[3 * o]; u_s[3 * p + 1] = ud[3 * o + 1]; u_s[3 * p + 2] = ud[3 * o + 2];
  }
  w_s[p] = w ? (w_f32 ? static_cast<double>(static_cast<const float*>(w)[o])
                      : static_cast<const double*>(w)[o])
             : 1.0;
}

// ptr[k] = first position p with seg(p) >= k, for k in [0, nseg]; seg() sorted.
__global__ void segment_offsets_kernel(const int32_t* __restrict__ seg, int64_t n, int64_t nseg,
                                       int64_t* ptr) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (p > n) return;
  const int64_t lo = (p == 0) ? 0 : static_cast<int64_t>(seg[p - 1]) + 1;
  const int64_t hi = (p == n) ? nseg : static_cast<int64_t>(seg[p]);
  for (int64_t k = lo; k <= hi; ++k) ptr[k] = p;
}

__global__ void landmark_stats_kernel(const int64_t* __restrict__ lm_ptr, int32_t M,
                                      const double* __restrict__ w_s, double* Wl, int64_t* cnt) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= M) return;
  const int64_t a = lm_ptr[k], b = lm_ptr[k + 1];
  double W = 0.0;
  for (int64_t p = a; p < b; ++p) W += w_s[p];
  Wl[k] = W;
  const int64_t L = b - a;
  cnt[k] = (L >= 2) ? L * L : 0;
}

__global__ void emit_pairs_kernel(const int64_t* __restrict__ lm_ptr, int32_t M, int32_t N,
                                  const int32_t* __restrict__ fr_s, const int64_t* __restrict__ poff,
                                  uint32_t* keys, uint64_t* vals) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= M) return;
  const int64_t p0 = lm_ptr[k], L = lm_ptr[k + 1] - p0;
  if (L < 2) return;
  int64_t q = poff[k];
  for (int64_t a = 0; a < L; ++a) {
    const uint32_t fa = static_cast<uint32_t>(fr_s[p0 + a]) * static_cast<uint32_t>(N);
    for (int64_t b = 0; b < L; ++b, ++q) {
      keys[q] = fa + static_cast<uint32_t>(fr_s[p0 + b]);
      vals[q] = (static_cast<uint64_t>(p0 + a) << 32) | static_cast<uint64_t>(p0 + b);
    }
  }
}

__global__ void head_flags_kernel(const uint32_t* __restrict__ keys, int64_t n, int64_t* flags) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (p >= n) return;
  flags[p] = (p == 0 || keys[p] != keys[p - 1]) ? 1 : 0;
}

__global__ void segment_starts_kernel(const uint32_t* __restrict__ keys, const int64_t* __restrict__ sidx,
                                      int64_t n, int64_t* seg_start, uint32_t* seg_key) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (p > n) return;
  if (p == n) {
    seg_start[sidx[n]] = n;
    return;
  }
  if (p == 0 || keys[p] != keys[p - 1]) {
    seg_start[sidx[p]] = p;
    seg_key[sidx[p]] = keys[p];
  }
}

// One group of kRedLanes lanes per frame pair: sum the 4x4 contributions of
// its observation pairs (strided over the group, then a fixed tree by
// recursive halving, so each lane ends with one of the 16 sums), write
// the rotation block into Q and the A_rt / A_tt entries.  A frame pair holds
// about ten observation pairs on average (the diagonal ones hundreds), so a
// group narrower than the wavefront wastes fewer lanes and reduction steps.
#ifndef XM_RED_LANES
#define XM_RED_LANES 16
#endif
constexpr int kRedLanes = XM_RED_LANES;
static_assert(kRedLanes == 16 || kRedLanes == 32 || kRedLanes == 64, "lane groups of 16 to 64");
// One 64-byte record per observation (landmark order) for the pair reduction:
// keypoint u, weight w and w / sqrt(W_k) (W_k the weight sum of its landmark,
// so that w_a w_b / W_k is the product of the two records' last entries).  A
// pair's two gathers, which come from scattered landmarks in frame-pair order,
// then touch one cache line each instead of four (keypoint, weight, landmark
// index, landmark weight).
__global__ void obs_record_kernel(int64_t n, const double* __restrict__ u_s, const double* __restrict__ w_s,
                                  const int32_t* __restrict__ lm_s, const double* __restrict__ Wl,
                                  double* __restrict__ rec) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (e >= n) return;
  const double w = w_s[e];
  double* r = rec + 8 * e;
  r[0] = u_s[3 * e];
  r[1] = u_s[3 * e + 1];
  r[2] = u_s[3 * e + 2];
  r[3] = w;
  r[4] = w / sqrt(Wl[lm_s[e]]);
  r[5] = r[6] = r[7] = 0.0;
}

__global__ __launch_bounds__(kB) void reduce_blocks_kernel(
    const int64_t* __restrict__ seg_start, const uint32_t* __restrict__ seg_key, int64_t S, int32_t N,
    const uint64_t* __restrict__ vals, const double* __restrict__ rec, const int32_t* __restrict__ pos, double* Q,
    int32_t ld, double* Art, double* Att, double* fac) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * (kB / kRedLanes) + threadIdx.x / kRedLanes;
  const int lane = threadIdx.x % kRedLanes;
  if (s >= S) return;
  const int64_t lo = seg_start[s], hi = seg_start[s + 1];
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int64_t q = lo + lane; q < hi; q += kRedLanes) {
    const uint64_t v = vals[q];
    const int64_t pa = static_cast<int64_t>(v >> 32), pb = static_cast<int64_t>(v & 0xffffffffull);
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* ra = reinterpret_cast<const d2*>(rec + 8 * pa);
    const d2* rb = reinterpret_cast<const d2*>(rec + 8 * pb);
    const d2 a0 = ra[0], a1 = ra[1], a2 = ra[2], b0 = rb[0], b1 = rb[1], b2 = rb[2];
    // w_a [a = b] - w_a w_b / W_k
    const double coef = ((pa == pb) ? a1[1] : 0.0) - a2[0] * b2[0];
    const double ha[4] = {a0[0], a0[1], a1[0], 1.0};
    const double hb[4] = {b0[0], b0[1], b1[0], 1.0};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double ca = coef * ha[a];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a * 4 + b] += ca * hb[b];
    }
  }
  // the 16 sums over the group: lane l with l % (kRedLanes / 16) = 0 holds
  // entry (a, b) = (q / 4, q % 4) of the 4x4 block, q = group_split_index(l)
  const double v = group_split_sum<16, kRedLanes>(acc, lane);
  if ((lane & (kRedLanes / 16 - 1)) != 0) return;
  const int q = group_split_index<16, kRedLanes>(lane), a = q >> 2, b = q & 3;
  if (a < 3 && b < 3) {
    if (Q) {  // Q is stored in the frame order: block (pos[i], pos[j])
      const uint32_t key = seg_key[s];
      const int64_t i = key / static_cast<uint32_t>(N), j = key % static_cast<uint32_t>(N);
      Q[(3 * static_cast<int64_t>(pos[i]) + a) * ld + 3 * static_cast<int64_t>(pos[j]) + b] = v;
    }
    fac[(3 * a + b) * S + s] = v;
  } else if (a < 3) {
    fac[(9 + a) * S + s] = v;
    Art[3 * s + a] = v;
  } else if (b == 3) {
    Att[s] = v;
  }
}

// ArtT[c][s] = Art[t][c] for the block s = (i, j) and its transpose t = (j, i)
// (binary search of i in row j: columns are sorted within a row); ArtT is
// structure of arrays, [3][S]
__global__ void transpose_art_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                     const double* __restrict__ Art, int32_t N, int64_t S, double* ArtT,
                                     int* flags) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (s >= S) return;
  // row i of block s: the last row whose start is <= s
  int lo = 0, hi = N - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (row_ptr[mid] <= s) lo = mid;
    else hi = mid - 1;
  }
  const int i = lo, j = col[s];
  int32_t a = row_ptr[j], b = row_ptr[j + 1] - 1;
  while (a < b) {
    const int32_t mid = (a + b) / 2;
    if (col[mid] < i) a = mid + 1;
    else b = mid;
  }
  if (a > b || col[a] != i) {  // the co-visibility pattern is symmetric: not reached
    flags[5] = 1;
    return;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) ArtT[c * S + s] = Art[3 * static_cast<int64_t>(a) + c];
}

__global__ void pattern_kernel(const uint32_t* __restrict__ seg_key, int64_t S, int32_t N,
                               int32_t* row_ptr, int32_t* col) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (p > S) return;
  const int64_t lo = (p == 0) ? 0 : static_cast<int64_t>(seg_key[p - 1] / static_cast<uint32_t>(N)) + 1;
  const int64_t hi = (p == S) ? N : static_cast<int64_t>(seg_key[p] / static_cast<uint32_t>(N));
  for (int64_t k = lo; k <= hi; ++k) row_ptr[k] = static_cast<int32_t>(p);
  if (p < S) col[p] = static_cast<int32_t>(seg_key[p] % static_cast<uint32_t>(N));
}

// A frame must have a positive diagonal Laplacian entry (otherwise it has no
// pair observation and its pose is unconstrained).
__global__ void check_diag_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                  const double* __restrict__ Att, int32_t N, int* flags) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= N) return;
  bool ok = false;
  for (int32_t s = row_ptr[i]; s < row_ptr[i + 1]; ++s)
    if (col[s] == i) ok = Att[s] > 0.0;
  if (!ok) flags[3] = 1;
}

__global__ void scatter_grounded_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                        const double* __restrict__ Att, int32_t N, double* G, int32_t ldg) {
  const int i = blockIdx.x;  // frame row
  if (i == 0 || i >= N) return;
  for (int32_t s = row_ptr[i] + threadIdx.x; s < row_ptr[i + 1]; s += blockDim.x) {
    const int j = col[s];
    if (j >= 1) G[static_cast<int64_t>(i - 1) * ldg + (j - 1)] = Att[s];
  }
}

// ---- block sweep (in-place inversion of the SPD grounded Laplacian) --------
// Sweeping the pivot set K of a symmetric A:
//   A_KK <- -A_KK^{-1}, A_iK <- A_iK A_KK^{-1}, A_Kj <- A_KK^{-1} A_Kj,
//   A_ij <- A_ij - A_iK A_KK^{-1} A_Kj   (i, j not in K).
// Sweeping every index in turn leaves -A^{-1}.  A stays symmetric, so only
// its upper triangle (64 x 64 tiles J >= I) is kept current; values of A_iK
// for i past K are read from A_Ki, and the lower triangle is copied from the
// upper one at the end.  The trailing update A_ij -= C_i P_j is a dense
// rank-kNB product per 64 x 64 tile on FP64 matrix cores; each step reads and
// writes the whole upper triangle, so wider pivot blocks mean fewer passes.
#ifndef XM_SWEEP_NB
#define XM_SWEEP_NB 128
#endif
constexpr int kNB = XM_SWEEP_NB;  // pivot block width: 64 or 128
static_assert(kNB == 64 || kNB == 128, "pivot blocks of 64 or 128");

// A_KK^{-1} by the symmetric sweep operator: with d = a_pp, pivot p maps
//   a_ij -> a_ij - a_ip a_pj / d,  a_ip -> a_ip / d,  a_pj -> a_pj / d,  a_pp -> -1/d,
// which keeps the block symmetric, so the pivot row is the pivot column.
// Thread t keeps column j = t % kNB of rows t / kNB + G c (G = kNB / 16 row
// groups, 16 values) in registers, so the serial work per pivot is the same
// at either block width; per pivot, the G threads of column p publish it
// through LDS (double-buffered, so one barrier per pivot suffices).
// After all pivots the block holds -A_KK^{-1}.  A last block with nb < kNB is
// padded with dscale * I.  Dinv (nb x nb) = A_KK^{-1}.
// Look-ahead (Dsave non-null): the block is formed here from the copy Dsave
// (upper triangle, row stride kNB) taken before the previous step's trailing
// update, minus that update's own terms sum_q Ct[q][k0+i] Pt[q][k0+j]
// (q < nbp), so the inversion need not wait for the whole update to finish.
constexpr int kPivotRows = 16;                          // rows per thread
constexpr int kPivotThreads = kNB * kNB / kPivotRows;   // 256 or 1024
constexpr int kPivotQC = 32;                            // panel rows per LDS chunk
__global__ __launch_bounds__(kPivotThreads) void sweep_pivot_kernel(
    const double* __restrict__ A, int32_t lda, int32_t k0, int32_t nb, double dscale,
    const double* __restrict__ Dsave, const double* __restrict__ Ct, const double* __restrict__ Pt, int32_t ldt,
    int32_t nbp, double* Dinv, int* flags) {
  constexpr int G = kNB / kPivotRows;  // row groups
  constexpr int RPT = kPivotRows;
  __shared__ double colp[2][kNB];
  __shared__ double Cs[kPivotQC][kNB], Ps[kPivotQC][kNB];
  const int t = threadIdx.x;
  const int j = t % kNB, ibase = t / kNB;
  double a[RPT];
  if (Dsave == nullptr) {
#pragma unroll
    for (int c = 0; c < RPT; ++c) {
      const int i = ibase + G * c;
      // only the upper triangle of A is current: (i, j) is read as (min, max)
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      a[c] = (i < nb && j < nb) ? A[static_cast<int64_t>(k0 + lo) * lda + k0 + hi] : (i == j ? dscale : 0.0);
    }
  } else {
    double acc[RPT];
#pragma unroll
    for (int c = 0; c < RPT; ++c) acc[c] = 0.0;
    for (int q0 = 0; q0 < nbp; q0 += kPivotQC) {
      for (int e = t; e < kPivotQC * kNB; e += kPivotThreads) {
        const int q = q0 + e / kNB, i = e % kNB;
        const bool ok = q < nbp && i < nb;
        Cs[e / kNB][i] = ok ? Ct[static_cast<int64_t>(q) * ldt + k0 + i] : 0.0;
        Ps[e / kNB][i] = ok ? Pt[static_cast<int64_t>(q) * ldt + k0 + i] : 0.0;
      }
      __syncthreads();
      for (int q = 0; q < kPivotQC; ++q) {
        const double pj = Ps[q][j];
#pragma unroll
        for (int c = 0; c < RPT; ++c) acc[c] += Cs[q][ibase + G * c] * pj;
      }
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < RPT; ++c) {
      const int i = ibase + G * c;
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      a[c] = (i < nb && j < nb) ? Dsave[lo * kNB + hi] - acc[c] : (i == j ? dscale : 0.0);
    }
  }
  // pivot p = G c0 + g sits in register c0 of the threads with ibase == g, so
  // with c0 unrolled the pivot row is a fixed register and every other entry
  // takes one FMA per pivot
#pragma unroll
  for (int c0 = 0; c0 < RPT; ++c0) {
#pragma nounroll
    for (int g = 0; g < G; ++g) {
      const int p = G * c0 + g;
      double* cp = colp[p & 1];
      if (j == p) {
#pragma unroll
        for (int c = 0; c < RPT; ++c) cp[ibase + G * c] = a[c];
      }
      __syncthreads();
      const double d = cp[p];
      if (!(d > 1e-11 * dscale)) {
        if (t == 0) flags[4] = 1;
        return;  // uniform across the block: every thread read the same d
      }
      double ci[RPT];  // column p at this thread's rows, all read before use
#pragma unroll
      for (int c = 0; c < RPT; ++c) ci[c] = cp[ibase + G * c];
      const double inv = 1.0 / d;
      const double f = cp[j] * inv;  // a_pj / d
      // a_ij - a_ip a_pj / d, and a_ip / d in the pivot column, as one
      // branch-free FMA: x = -f, keep = 1 off the pivot column, x = 1/d, keep = 0 on it
      const bool pc = j == p;
      const double x = pc ? inv : -f, keep = pc ? 0.0 : 1.0;
#pragma unroll
      for (int c = 0; c < RPT; ++c) a[c] = __builtin_fma(ci[c], x, a[c] * keep);
      if (ibase == g) a[c0] = (j == p) ? -inv : f;  // pivot row
    }
  }
#pragma unroll
  for (int c = 0; c < RPT; ++c) {
    const int i = ibase + G * c;
    if (i < nb && j < nb) Dinv[i * nb + j] = -a[c];
  }
}

// Ct[q][i] = sum_p A[i][k0+p] Dinv[p][q] (0 for i in K); Pt[q][i] = A[i][k0+q].
// Workgroup: the 64 x 64 block of Ct at columns q from qb = 64 blockIdx.y and
// rows i from i0 = 64 blockIdx.x, on FP64 matrix cores: each wave a 32 x 32
// quarter as 2 x 2 v_mfma_f64_16x16x4f64 blocks (A operand Dinv[p][q] as [q][p],
// B operand the panel as [p][i], so the 16 lanes of a result row hold
// consecutive i and the stores to Ct are contiguous).  The panel (rows of A for
// i < k0, rows of A_K. for i >= k0, since only the upper triangle is current)
// and Dinv go through LDS in chunks of 16 p, double-buffered; the workgroups
// with blockIdx.y = 0 also write the staged panel out as Pt.  One more column
// of workgroups (i0 >= n) copies the upper triangle of the next pivot block
// (k1, nb1 wide) into Dsave before this step's trailing update changes it.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kPanelKC = 16;
__global__ __launch_bounds__(kB) void sweep_panel_kernel(const double* __restrict__ A, int32_t lda, int32_t n,
                                                         int32_t k0, int32_t nb, const double* __restrict__ Dinv,
                                                         double* Ct, double* Pt, int32_t ldt, int32_t k1,
                                                         int32_t nb1, double* Dsave) {
  __shared__ double Ds[2][kPanelKC][64];  // Ds[k][q] = Dinv[p0 + k][qb + q]
  __shared__ double Ts[2][kPanelKC][64];  // Ts[k][i] = A[i0 + i][k0 + p0 + k]
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * 64, qb = blockIdx.y * 64;
  if (i0 >= n) {
    for (int e = t; e < 64 * kNB; e += kB) {
      const int r = qb + e / kNB, c = e % kNB;
      if (r < nb1 && c >= r && c < nb1) Dsave[r * kNB + c] = A[static_cast<int64_t>(k1 + r) * lda + k1 + c];
    }
    return;
  }
  const bool above = i0 < k0;  // the whole slice lies above K (k0 and i0 are multiples of 64)
  const bool write_pt = blockIdx.y == 0;
  constexpr int kPer = kPanelKC * 64 / kB;  // staged entries per thread and operand
  double rd[kPer], rt[kPer];
  auto fetch = [&](int p0) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = t + kB * m;
      {
        const int k = e >> 6, q = e & 63;
        const int pp = p0 + k;
        rd[m] = (pp < nb && qb + q < nb) ? Dinv[pp * nb + qb + q] : 0.0;
      }
      if (above) {  // 16 consecutive p per row i
        const int k = e & 15, i = e >> 4;
        rt[m] = (i0 + i < n && p0 + k < nb) ? A[static_cast<int64_t>(i0 + i) * lda + k0 + p0 + k] : 0.0;
      } else {      // 64 consecutive i per row p
        const int k = e >> 6, i = e & 63;
        rt[m] = (i0 + i < n && p0 + k < nb) ? A[static_cast<int64_t>(k0 + p0 + k) * lda + i0 + i] : 0.0;
      }
    }
  };
  auto stash = [&](int buf, int p0) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = t + kB * m;
      Ds[buf][e >> 6][e & 63] = rd[m];
      const int k = above ? (e & 15) : (e >> 6), i = above ? (e >> 4) : (e & 63);
      Ts[buf][k][i] = rt[m];
      if (write_pt && p0 + k < nb && i0 + i < n) Pt[static_cast<int64_t>(p0 + k) * ldt + i0 + i] = rt[m];
    }
  };
  const int lane = t & 63, wave = t >> 6;
  const int wq = (wave >> 1) * 32, wi = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  stash(0, 0);
  __syncthreads();
#pragma unroll
  for (int ch = 0; ch < kNB / kPanelKC; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < kNB / kPanelKC;
    if (more) fetch((ch + 1) * kPanelKC);
#pragma unroll
    for (int k = 0; k < kPanelKC; k += 4) {
      const double a0 = Ds[buf][k + lk][wq + lr], a1 = Ds[buf][k + lk][wq + 16 + lr];
      const double b0 = Ts[buf][k + lk][wi + lr], b1 = Ts[buf][k + lk][wi + 16 + lr];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (more) {
      stash(buf ^ 1, (ch + 1) * kPanelKC);
      __syncthreads();
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = qb + wq + 16 * a + lk + 4 * r;
        const int i = i0 + wi + 16 * b + lr;
        const bool inK = (i >= k0 && i < k0 + nb);
        if (q < nb && i < n) Ct[static_cast<int64_t>(q) * ldt + i] = inK ? 0.0 : acc[a][b][r];
      }
}

// A[i][j] -= sum_p Ct[p][i] Pt[p][j] on the 64 x 64 tiles J >= I.  Each wave
// forms a 32 x 32 quarter as 2 x 2 blocks of v_mfma_f64_16x16x4f64 over kNB / 4
// k-steps: lane l supplies A-operand [i = l % 16][k = l / 16] and B-operand
// [k = l / 16][j = l % 16]; register q of the result holds [l / 16 + 4 q][l % 16].
// The tile of A is loaded into registers first (its HBM latency overlaps the
// panel staging), the rank-kNB product is accumulated from zero and subtracted
// once at the end (one rounding at the scale of A).  The panels go through LDS
// in chunks of kSweepKC rows, double-buffered: the next chunk's loads are in
// flight while the current one is multiplied.
// Workgroup w takes tile tiles[w mod 8][w / 8] of a list cut into 8 contiguous
// runs, one per XCD (w runs on XCD w mod 8), each run ordered by 8 x 8 blocks
// of tiles, so that the panel slices a run needs at a time stay in its L2.
#ifndef XM_SWEEP_SB
#define XM_SWEEP_SB 8
#endif
#ifndef XM_SWEEP_KC
#define XM_SWEEP_KC 16
#endif
// The tile of G is streamed: read once and written once per step, and the
// whole upper triangle (0.4 GB at N = 10^4) does not stay in any cache between
// steps, so its loads and stores carry the non-temporal hint (measured 4 %
// faster at N = 10155).
#ifndef XM_SWEEP_NT
#define XM_SWEEP_NT 1
#endif
constexpr int kSweepKC = XM_SWEEP_KC;
__global__ __launch_bounds__(kB) void sweep_update_kernel(double* A, int32_t lda, int32_t n,
                                                          const double* __restrict__ Ct,
                                                          const double* __restrict__ Pt, int32_t ldt, int32_t nb,
                                                          const int32_t* __restrict__ tiles, int32_t ntiles) {
  const int per = (ntiles + 7) / 8;
  const int idx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (idx >= ntiles) return;
  __shared__ double Cs[2][kSweepKC][64];
  __shared__ double Ps[2][kSweepKC][64];
  const int i0 = 64 * tiles[2 * idx], j0 = 64 * tiles[2 * idx + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  double g[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wi + 16 * a + lk + 4 * q;
        const int j = j0 + wj + 16 * b + lr;
#if XM_SWEEP_NT
        g[a][b][q] = (i < n && j < n) ? __builtin_nontemporal_load(A + static_cast<int64_t>(i) * lda + j) : 0.0;
#else
        g[a][b][q] = (i < n && j < n) ? A[static_cast<int64_t>(i) * lda + j] : 0.0;
#endif
      }
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  // panel chunks of kSweepKC rows, double-buffered: thread t stages entries
  // t + kB m (m < kSweepKC * 64 / kB) of the chunk
  constexpr int kPer = kSweepKC * 64 / kB;
  double rc[kPer], rp[kPer];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = t + kB * m;
      const int pp = kc + (e >> 6), c = e & 63;
      rc[m] = (pp < nb && i0 + c < n) ? Ct[static_cast<int64_t>(pp) * ldt + i0 + c] : 0.0;
      rp[m] = (pp < nb && j0 + c < n) ? Pt[static_cast<int64_t>(pp) * ldt + j0 + c] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = t + kB * m;
      Cs[buf][e >> 6][e & 63] = rc[m];
      Ps[buf][e >> 6][e & 63] = rp[m];
    }
  };
  fetch(0);
  stash(0);
  __syncthreads();
#pragma unroll
  for (int ch = 0; ch < kNB / kSweepKC; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < kNB / kSweepKC;
    if (more) fetch((ch + 1) * kSweepKC);
#pragma unroll
    for (int k = 0; k < kSweepKC; k += 4) {
      const double a0 = Cs[buf][k + lk][wi + lr], a1 = Cs[buf][k + lk][wi + 16 + lr];
      const double b0 = Ps[buf][k + lk][wj + lr], b1 = Ps[buf][k + lk][wj + 16 + lr];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (more) {
      stash(buf ^ 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wi + 16 * a + lk + 4 * q;
        const int j = j0 + wj + 16 * b + lr;
#if XM_SWEEP_NT
        if (i < n && j < n) __builtin_nontemporal_store(g[a][b][q] - acc[a][b][q], A + static_cast<int64_t>(i) * lda + j);
#else
        if (i < n && j < n) A[static_cast<int64_t>(i) * lda + j] = g[a][b][q] - acc[a][b][q];
#endif
      }
}

// the upper tiles (I <= J) of a T x T tiling, blocked by SB x SB tiles in
// row-major block order, as (I, J) pairs
std::vector<int32_t> sweep_tile_list(int T) {
  constexpr int SB = XM_SWEEP_SB;
  std::vector<int32_t> out;
  for (int bi = 0; bi < T; bi += SB)
    for (int bj = bi; bj < T; bj += SB)
      for (int I = bi; I < std::min(T, bi + SB); ++I)
        for (int J = std::max(I, bj); J < std::min(T, bj + SB); ++J) {
          out.push_back(I);
          out.push_back(J);
        }
  return out;
}

__global__ void sweep_finish_kernel(double* A, int32_t lda, int32_t n, int32_t k0, int32_t nb,
                                    const double* __restrict__ Ct, int32_t ldt,
                                    const double* __restrict__ Dinv) {
  const int i = blockIdx.x * kB + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= n || p >= nb) return;
  if (i >= k0 && i < k0 + nb) {
    A[static_cast<int64_t>(k0 + p) * lda + i] = -Dinv[p * nb + (i - k0)];
  } else {
    const double c = Ct[static_cast<int64_t>(p) * ldt + i];
    A[static_cast<int64_t>(i) * lda + k0 + p] = c;
    A[static_cast<int64_t>(k0 + p) * lda + i] = c;
  }
}

// out[c][r] = in[r][c]  (64 x 64 tiles through LDS)
__global__ __launch_bounds__(kB) void transpose_kernel(const double* __restrict__ in, int32_t rows, int32_t cols,
                                                       int32_t ldi, double* out, int32_t ldo) {
  __shared__ double tile[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += kB) {
    const int r = e / 64, c = e % 64;
    tile[r][c] = (r0 + r < rows && c0 + c < cols) ? in[static_cast<int64_t>(r0 + r) * ldi + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += kB) {
    const int c = e / 64, r = e % 64;
    if (r0 + r < rows && c0 + c < cols) out[static_cast<int64_t>(c0 + c) * ldo + r0 + r] = tile[r][c];
  }
}

// Q[c][r] <- Q[r][c] for r < c: the lower triangle copied from the upper one,
// one 32 x 32 tile pair (I <= J) per block, staged through LDS so that both
// the read of tile (I, J) and the write of tile (J, I) are coalesced.
__global__ __launch_bounds__(kB) void symmetrize_kernel(double* Q, int32_t n, int32_t ld, float* Q32) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  __shared__ double a[32][33];
  const int r0 = I * 32, c0 = J * 32;
  for (int e = threadIdx.x; e < 32 * 32; e += kB) {
    const int r = e / 32, c = e % 32;
    const bool in = r0 + r < n && c0 + c < n;
    a[r][c] = in ? Q[static_cast<int64_t>(r0 + r) * ld + c0 + c] : 0.0;  // tile (I, J)
    // FP32 copy of the upper triangle (diagonal included) as it is read
    if (Q32 && in && r0 + r <= c0 + c)
      Q32[static_cast<int64_t>(r0 + r) * ld + c0 + c] = static_cast<float>(a[r][c]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += kB) {
    const int c = e / 32, r = e % 32;  // write row c0 + c of tile (J, I), consecutive r
    if (r0 + r < n && c0 + c < n && r0 + r < c0 + c) {
      Q[static_cast<int64_t>(c0 + c) * ld + r0 + r] = a[r][c];
      if (Q32) Q32[static_cast<int64_t>(c0 + c) * ld + r0 + r] = static_cast<float>(a[r][c]);
    }
  }
}

// columns n .. ld of every row (the padding of the FP32 copy of Q)
__global__ __launch_bounds__(kB) void zero_pad_kernel(float* Q32, int32_t n, int32_t ld) {
  const int i = blockIdx.x;
  for (int c = n + threadIdx.x; c < ld; c += kB) Q32[static_cast<int64_t>(i) * ld + c] = 0.0f;
}

__global__ __launch_bounds__(kB) void trace_kernel(const double* __restrict__ Q, int32_t n, int32_t ld,
                                                   double* out) {
  __shared__ double lds[4];
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += kB) v[0] += Q[static_cast<int64_t>(i) * ld + i];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) out[0] = v[0];
}

// largest diagonal entry of a matrix (one block; scale of the pivot test)
__global__ __launch_bounds__(kB) void diag_max_kernel(const double* __restrict__ A, int32_t n, int32_t ld,
                                                      double* out) {
  __shared__ double lds[kB];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) m = fmax(m, A[static_cast<int64_t>(i) * ld + i]);
  lds[threadIdx.x] = m;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = lds[0];
}

// q_kk = tr(Q_kk) / 3 per frame (the preconditioner of the local solver)
__global__ void diag_block_kernel(const double* __restrict__ Q, int32_t N, int32_t ld,
                                  const int32_t* __restrict__ pos, double* __restrict__ q) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const int64_t i = 3 * static_cast<int64_t>(pos[k]);
  q[k] = (Q[i * ld + i] + Q[(i + 1) * ld + i + 1] + Q[(i + 2) * ld + i + 2]) / 3.0;
}

// Q_kk^{1/2}, Q_kk^{-1/2} by a cyclic Jacobi eigendecomposition of each 3x3
// diagonal block; eigenvalues are floored at 1e-12 of their block's largest so
// that a degenerate block still gives an SPD scaling.  ext[k] = (min, max) eig.
__global__ void block_sqrt_kernel(const double* __restrict__ Q, int32_t N, int32_t ld,
                                  const int32_t* __restrict__ pos, double* __restrict__ Dh,
                                  double* __restrict__ Dmh, double* __restrict__ ext) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  double A[3][3], V[3][3];
  const int64_t i0 = 3 * static_cast<int64_t>(pos[k]);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      A[a][b] = 0.5 * (Q[(i0 + a) * ld + i0 + b] + Q[(i0 + b) * ld + i0 + a]);
      V[a][b] = (a == b) ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 30; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-32 * dia) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int m = 0; m < 3; ++m) {
          const double amp = A[m][p], amq = A[m][q];
          A[m][p] = c * amp - s * amq;
          A[m][q] = s * amp + c * amq;
        }
        for (int m = 0; m < 3; ++m) {
          const double apm = A[p][m], aqm = A[q][m];
          A[p][m] = c * apm - s * aqm;
          A[q][m] = s * apm + c * aqm;
        }
        for (int m = 0; m < 3; ++m) {
          const double vmp = V[m][p], vmq = V[m][q];
          V[m][p] = c * vmp - s * vmq;
          V[m][q] = s * vmp + c * vmq;
        }
      }
  }
  double lam[3];
  const double top = fmax(A[0][0], fmax(A[1][1], A[2][2]));
  for (int a = 0; a < 3; ++a) lam[a] = fmax(A[a][a], 1e-12 * top);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double hp = 0.0, hm = 0.0;
      for (int m = 0; m < 3; ++m) {
        hp += V[a][m] * sqrt(lam[m]) * V[b][m];
        hm += V[a][m] / sqrt(lam[m]) * V[b][m];
      }
      Dh[9 * static_cast<int64_t>(k) + 3 * a + b] = hp;
      Dmh[9 * static_cast<int64_t>(k) + 3 * a + b] = hm;
    }
  ext[2 * k] = fmin(lam[0], fmin(lam[1], lam[2]));
  ext[2 * k + 1] = fmax(lam[0], fmax(lam[1], lam[2]));
}

// four values per thread (32-byte loads, 16-byte stores; in and out are
// allocation starts, so every group of four is aligned)
constexpr int kF32Per = 4;
__global__ void to_f32_kernel(const double* __restrict__ in, int64_t n, float* out) {
  const int64_t e = (static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x) * kF32Per;
  if (e + kF32Per <= n) {
    const double2 a = *reinterpret_cast<const double2*>(in + e);
    const double2 b = *reinterpret_cast<const double2*>(in + e + 2);
    *reinterpret_cast<float4*>(out + e) = make_float4(static_cast<float>(a.x), static_cast<float>(a.y),
                                                      static_cast<float>(b.x), static_cast<float>(b.y));
  } else {
    for (int64_t k = e; k < n; ++k) out[k] = static_cast<float>(in[k]);
  }
}

// Zero row i of Q from column c0 = 3 floor(i / 3) rounded down to a multiple
// of 64 to the end of the row (padding included): every entry the assembly
// reads before the lower triangle is copied from the upper one.
__global__ __launch_bounds__(kB) void zero_upper_kernel(double* Q, int32_t ld) {
  const int i = blockIdx.x;
  const int c0 = (3 * (i / 3)) & ~63;
  double2* row = reinterpret_cast<double2*>(Q + static_cast<int64_t>(i) * ld + c0);
  const int n2 = (ld - c0) / 2;
  for (int e = threadIdx.x; e < n2; e += kB) row[e] = make_double2(0.0, 0.0);
}

// round-to-nearest-even FP64 -> BF16 (through FP32; NaN not expected here)
__global__ void to_bf16_kernel(const double* __restrict__ in, int64_t n, uint16_t* out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (e >= n) return;
  const uint32_t x = __float_as_uint(static_cast<float>(in[e]));
  const uint32_t lsb = (x >> 16) & 1u;
  out[e] = static_cast<uint16_t>((x + 0x7fffu + lsb) >> 16);
}

// HIP events around every launch of one kernel on a stream; total() waits
// for the last one and returns the summed device time in milliseconds.
// ---- frame grouping for the two sparse-dense products ---------------------
// P = B Gm and the correction B P^T both read, for every stored block (i, j),
// a whole row j of a dense operand: frame by frame that is ~300 dense rows per
// frame, and the products are bound by the traffic of those rows from the
// caches.  Frames that are close in a Cuthill-McKee order of the co-visibility
// graph share most of their co-visible frames, so kGroup consecutive frames in
// that order are processed by one workgroup: each dense row of their union is
// read once and applied to every frame of the group that sees it (a 4x cut in
// rows read on clustered scenes).  The order is a breadth-first search from
// the anchored frame 0 in which each new level is sorted by the position of its
// first discoverer, then by frame index: deterministic.
constexpr int kGroup = kFrameGroup;
constexpr int32_t kUnset = 0x7f7f7f7f;  // key of a frame not reached yet (memset byte 0x7f)

// key[u] = min position (in the order) of a frontier frame adjacent to u, for unplaced u
__global__ __launch_bounds__(kB) void cm_expand_kernel(const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ order, int32_t lo, int32_t hi,
                                                       const int32_t* __restrict__ pos, int32_t* key) {
  const int p = lo + blockIdx.x * (kB / 64) + (threadIdx.x >> 6);
  if (p >= hi) return;  // whole wavefronts only
  const int v = order[p];
  for (int32_t s = row_ptr[v] + (threadIdx.x & 63); s < row_ptr[v + 1]; s += 64) {
    const int u = col[s];
    if (pos[u] < 0) atomicMin(key + u, p);
  }
}

// flag[u] = 1 for the frames reached in this level (unplaced, with a key)
__global__ void cm_flag_kernel(const int32_t* __restrict__ pos, const int32_t* __restrict__ key, int32_t N,
                               int64_t* flag) {
  const int u = blockIdx.x * kB + threadIdx.x;
  if (u < N) flag[u] = (pos[u] < 0 && key[u] != kUnset) ? 1 : 0;
}

// compact the reached frames in index order: (key - lo, frame) pairs for a stable sort by key
__global__ void cm_compact_kernel(const int32_t* __restrict__ pos, const int32_t* __restrict__ key,
                                  const int64_t* __restrict__ slot, int32_t N, int32_t lo, uint32_t* ks,
                                  uint64_t* vs) {
  const int u = blockIdx.x * kB + threadIdx.x;
  if (u >= N || !(pos[u] < 0 && key[u] != kUnset)) return;
  ks[slot[u]] = static_cast<uint32_t>(key[u] - lo);
  vs[slot[u]] = static_cast<uint64_t>(u);
}

__global__ void cm_place_kernel(const uint64_t* __restrict__ vs, int64_t count, int32_t hi, int32_t* order,
                                int32_t* pos) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kB + threadIdx.x;
  if (t >= count) return;
  const int u = static_cast<int>(vs[t]);
  order[hi + t] = u;
  pos[u] = static_cast<int32_t>(hi + t);
}

// frames never reached (a disconnected view graph, rejected later): appended in index order
__global__ void cm_rest_kernel(const int64_t* __restrict__ slot, const int32_t* __restrict__ pos0, int32_t N,
                               int32_t hi, int32_t* order, int32_t* pos) {
  const int u = blockIdx.x * kB + threadIdx.x;
  if (u >= N || pos0[u] >= 0) return;
  order[hi + slot[u]] = u;
  pos[u] = static_cast<int32_t>(hi + slot[u]);
}

__global__ void cm_unplaced_kernel(const int32_t* __restrict__ pos, int32_t N, int64_t* flag) {
  const int u = blockIdx.x * kB + threadIdx.x;
  if (u < N) flag[u] = pos[u] < 0 ? 1 : 0;
}

// Bitmap in LDS of the frames j >= 1 co-visible with some frame of group g
// (the anchored frame 0 has no column in B).  Returns the number of words.
__device__ void group_bitmap(int g, int32_t N, const int32_t* __restrict__ order,
                             const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, uint32_t* bits) {
  const int nw = (N + 31) / 32;
  for (int w = threadIdx.x; w < nw; w += kB) bits[w] = 0u;
  __syncthreads();
  for (int f = 0; f < kGroup; ++f) {
    const int a = g * kGroup + f;
    if (a >= N) break;
    const int i = order[a];
    for (int32_t s = row_ptr[i] + threadIdx.x; s < row_ptr[i + 1]; s += kB) {
      const int j = col[s];
      if (j > 0) atomicOr(bits + (j >> 5), 1u << (j & 31));
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kB) void group_count_kernel(int32_t N, const int32_t* __restrict__ order,
                                                         const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col, int64_t* ucount) {
  extern __shared__ uint32_t bits[];
  __shared__ int partial[kB];
  group_bitmap(blockIdx.x, N, order, row_ptr, col, bits);
  const int nw = (N + 31) / 32;
  int c = 0;
  for (int w = threadIdx.x; w < nw; w += kB) c += __popc(bits[w]);
  partial[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int k = 0; k < kB; ++k) t += partial[k];
    ucount[blockIdx.x] = t;
  }
}

// uid[k]: the union of group g in increasing frame order (k from ustart[g]);
// coef[k][f][q] = A_rt[3 order[g kGroup + f] + q][uid[k]] for q < 3 (rows of 4,
// the last one 0; zero where frame f does not see uid[k]; coef is cleared
// beforehand); lidx[s] = k - ustart[g] for the stored block s = (i, uid[k]) of
// a frame i of the group, -1 for s = (i, 0)
__global__ __launch_bounds__(kB) void group_fill_kernel(int32_t N, const int32_t* __restrict__ order,
                                                        const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ Art,
                                                        const int64_t* __restrict__ ustart, int32_t* uid,
                                                        double* coef, int32_t* lidx) {
  extern __shared__ uint32_t bits[];
  const int nw = (N + 31) / 32;
  int* wpre = reinterpret_cast<int*>(bits + nw);  // exclusive prefix of set bits per word
  const int g = blockIdx.x;
  group_bitmap(g, N, order, row_ptr, col, bits);
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < nw; ++w) {
      wpre[w] = t;
      t += __popc(bits[w]);
    }
  }
  __syncthreads();
  const int64_t base = ustart[g];
  for (int w = threadIdx.x; w < nw; w += kB) {
    uint32_t b = bits[w];
    int r = wpre[w];
    while (b) {
      const int t = __ffs(b) - 1;
      uid[base + r++] = 32 * w + t;
      b &= b - 1;
    }
  }
  for (int f = 0; f < kGroup; ++f) {
    const int a = g * kGroup + f;
    if (a >= N) break;
    const int i = order[a];
    for (int32_t s = row_ptr[i] + threadIdx.x; s < row_ptr[i + 1]; s += kB) {
      const int j = col[s];
      if (j == 0) {
        lidx[s] = -1;
        continue;
      }
      const int w = j >> 5;
      const int64_t k = base + wpre[w] + __popc(bits[w] & ((1u << (j & 31)) - 1u));
      lidx[s] = static_cast<int32_t>(k - base);
#pragma unroll
      for (int q = 0; q < 3; ++q) coef[(k * kGroup + f) * 4 + q] = Art[3 * static_cast<int64_t>(s) + q];
    }
  }
}

// Grouped sparse-dense product on FP64 matrix cores.  For group g (frames at
// positions a = g kGroup + f of the order) and column c:
//   out[3a+q][c] = sum_{k in union of g} coef[k][f][q] D[uid[k]-1][c],
// i.e. the 48 output rows of the group are a dense (48 x |union|) coefficient
// block (zeros where a frame does not see a union frame) times the gathered
// union rows of D.  P pass: D = Gm (N-1 x N-1), out = P with rows in the order.
// Q pass: D = P^T (columns in the order), out = Q (stored in the order), to
// which the correction is added on the upper triangle (c >= 3a).
//
// Workgroup = group x 64 kCPL columns.  The union is taken in chunks of 16
// rows: the chunk's rows of D (16 x 64 kCPL) and coefficients (16 x 16 x 4) are
// staged in LDS, double-buffered: the next chunk's global loads are in flight
// while the current one is multiplied.  Each wave takes 16 kCPL columns as
// 3 x kCPL tiles of v_mfma_f64_16x16x4f64 per 4 union rows, the tile (q, u)
// holding rows 3f + q and columns kCPL j + u (f, j < 16): lane l supplies
// A[f = l % 16][k = l / 16] for the three q from one 32-byte read of
// coef[k][f][0..3] and B[k = l / 16][j = l % 16] for the kCPL values of u from
// one read of the union row, and holds C[l / 16 + 4 r][l % 16] in register r.
#ifndef XM_GROUP_CPL
#define XM_GROUP_CPL 2
#endif
constexpr int kCPL = XM_GROUP_CPL;            // output columns per lane (= MFMA column tiles per wave)
constexpr int kGroupCols = 64 * kCPL;         // columns per workgroup: 4 waves x 16 lanes x kCPL
constexpr int kChunk = 16;
typedef double v4d_a __attribute__((ext_vector_type(4), aligned(32)));
typedef double vcol __attribute__((ext_vector_type(kCPL), aligned(8 * kCPL)));
template <bool UPPER>
__global__ __launch_bounds__(kB) void group_product_kernel(int32_t N, const int32_t* __restrict__ tile_start,
                                                           int32_t ntiles, const int64_t* __restrict__ ustart,
                                                           const int32_t* __restrict__ uid,
                                                           const double* __restrict__ coef,
                                                           const double* __restrict__ D, int32_t ldd, int32_t K,
                                                           double* __restrict__ out, int32_t ldo) {
  __shared__ vcol Bs[2][kChunk][kGroupCols / kCPL];
  __shared__ v4d_a As[2][kChunk][kGroup];
  // workgroup w -> (column tile y, group g): tile-major over the pairs that
  // produce output (tile y holds the groups g < tile_start[y + 1] - tile_start[y]),
  // so that the workgroups in flight read few column slices of D
  const int w = blockIdx.x;
  int lo = 0, hi = ntiles - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (tile_start[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  const int g = w - tile_start[lo];
  const int row0 = 3 * kGroup * g;
  const int cbase = lo * kGroupCols;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int kr = lane >> 4, lj = lane & 15;
  // staging: thread t loads row t / 16 of the chunk, four kCPL-wide pieces of
  // the tile from column 4 kCPL (t % 16), and coefficient row t / 16, frame t % 16
  constexpr int SW = 4 * kCPL;
  const int sr = t >> 4, sc = (t & 15) * SW;
  const int gc = cbase + sc;
  const bool sfull = gc + SW <= K;
  const int64_t k0 = ustart[g], k1 = ustart[g + 1];
  struct Stage {
    vcol b[4];
    v4d_a a;
  };
  auto fetch = [&](int64_t kc, Stage& st) {
    const int64_t k = kc + sr;
    if (k < k1) {
      st.a = *reinterpret_cast<const v4d_a*>(coef + (k * kGroup + (t & 15)) * 4);
      const double* drow = D + static_cast<int64_t>(uid[k] - 1) * ldd + gc;
      if (sfull) {
#pragma unroll
        for (int p = 0; p < 4; ++p) st.b[p] = *reinterpret_cast<const vcol*>(drow + kCPL * p);
      } else {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int e = 0; e < kCPL; ++e) st.b[p][e] = (gc + kCPL * p + e < K) ? drow[kCPL * p + e] : 0.0;
      }
    } else {
      st.a = v4d_a{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int e = 0; e < kCPL; ++e) st.b[p][e] = 0.0;
    }
  };
  auto stash = [&](int buf, const Stage& st) {
#pragma unroll
    for (int p = 0; p < 4; ++p) Bs[buf][sr][(t & 15) * 4 + p] = st.b[p];
    As[buf][sr][t & 15] = st.a;
  };
  v4d acc[3][kCPL];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int u = 0; u < kCPL; ++u) acc[q][u] = v4d{0.0, 0.0, 0.0, 0.0};
  const int n3 = 3 * N;
  const int cl = cbase + wave * 16 * kCPL + kCPL * lj;  // this lane's kCPL output columns
  if (UPPER) {
    // the Q pass adds to the stored Q: its tile is the accumulators' start
    // (loaded here, so the loads overlap the first chunk's staging)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = kr + 4 * r;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int orow = row0 + 3 * f + q;
        if (orow >= n3) continue;
        const double* o = out + static_cast<int64_t>(orow) * ldo;
        const int cmin = row0 + 3 * f;
        if (cl + kCPL <= K && cl >= cmin) {
          const vcol v = *reinterpret_cast<const vcol*>(o + cl);
#pragma unroll
          for (int u = 0; u < kCPL; ++u) acc[q][u][r] = v[u];
        } else {
#pragma unroll
          for (int u = 0; u < kCPL; ++u)
            if (cl + u < K && cl + u >= cmin) acc[q][u][r] = o[cl + u];
        }
      }
    }
  }
  auto multiply = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < kChunk / 4; ++ks) {
      const v4d_a av = As[buf][4 * ks + kr][lj];
      const vcol bv = Bs[buf][4 * ks + kr][wave * 16 + lj];
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int u = 0; u < kCPL; ++u)
          acc[q][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[u], acc[q][u], 0, 0, 0);
    }
  };
  // chunk c sits in LDS buffer c % 2; the next chunk's global loads are in
  // flight (in registers) while chunk c is multiplied
  Stage st;
  fetch(k0, st);
  stash(0, st);
  __syncthreads();
  const int64_t nchunks = (k1 - k0 + kChunk - 1) / kChunk;
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) fetch(k0 + (c + 1) * kChunk, st);
    multiply(c & 1);
    if (more) {
      stash((c + 1) & 1, st);
      __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int f = kr + 4 * r;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int orow = row0 + 3 * f + q;
      if (orow >= n3) continue;
      double* o = out + static_cast<int64_t>(orow) * ldo;
      const int cmin = UPPER ? row0 + 3 * f : 0;
      if (cl + kCPL <= K && cl >= cmin) {
        vcol v;
#pragma unroll
        for (int u = 0; u < kCPL; ++u) v[u] = acc[q][u][r];
        *reinterpret_cast<vcol*>(o + cl) = v;
      } else {
#pragma unroll
        for (int u = 0; u < kCPL; ++u)
          if (cl + u < K && cl + u >= cmin) o[cl + u] = acc[q][u][r];
      }
    }
  }
}

// Cuthill-McKee order of the co-visibility graph from frame 0 (order:
// position -> frame, pos: frame -> position); one host round trip per level.
void cm_order(int32_t N, const int32_t* row_ptr, const int32_t* col, DevBuf<int32_t>& order, DevBuf<int32_t>& pos,
              hipStream_t s) {
  order.alloc(N);
  pos.alloc(N);
  DevBuf<int32_t> key(N);
  DevBuf<int64_t> flag(N), slot(N + 1);
  DevBuf<uint32_t> ks(N), kt(N);
  DevBuf<uint64_t> vs(N), vt(N);
  XM_HIP(hipMemsetAsync(pos.ptr, 0xff, N * sizeof(int32_t), s));
  XM_HIP(hipMemsetAsync(key.ptr, 0x7f, N * sizeof(int32_t), s));
  const int32_t zero = 0;
  XM_HIP(hipMemcpyAsync(order.ptr, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
  XM_HIP(hipMemcpyAsync(pos.ptr, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
  int32_t lo = 0, hi = 1;
  const unsigned gn = cdiv(N, kB);
  while (hi < N) {
    hipLaunchKernelGGL(cm_expand_kernel, dim3(cdiv(hi - lo, kB / 64)), dim3(kB), 0, s, row_ptr, col, order.ptr, lo,
                       hi, pos.ptr, key.ptr);
    XM_LAUNCH_CHECK("cm_expand_kernel");
    hipLaunchKernelGGL(cm_flag_kernel, dim3(gn), dim3(kB), 0, s, pos.ptr, key.ptr, N, flag.ptr);
    XM_LAUNCH_CHECK("cm_flag_kernel");
    exclusive_scan_i64(flag.ptr, slot.ptr, N, s);  // synchronises
    int64_t count = 0;
    XM_HIP(hipMemcpy(&count, slot.ptr + N, sizeof(int64_t), hipMemcpyDeviceToHost));
    if (count == 0) break;
    hipLaunchKernelGGL(cm_compact_kernel, dim3(gn), dim3(kB), 0, s, pos.ptr, key.ptr, slot.ptr, N, lo, ks.ptr,
                       vs.ptr);
    XM_LAUNCH_CHECK("cm_compact_kernel");
    int bits = 1;
    while ((int64_t(1) << bits) < (hi - lo)) ++bits;
    radix_sort_pairs(ks.ptr, vs.ptr, kt.ptr, vt.ptr, count, bits, s);
    hipLaunchKernelGGL(cm_place_kernel, dim3(cdiv(count, kB)), dim3(kB), 0, s, vs.ptr, count, hi, order.ptr,
                       pos.ptr);
    XM_LAUNCH_CHECK("cm_place_kernel");
    lo = hi;
    hi += static_cast<int32_t>(count);
  }
  if (hi < N) {
    DevBuf<int32_t> pos0(N);
    XM_HIP(hipMemcpyAsync(pos0.ptr, pos.ptr, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(cm_unplaced_kernel, dim3(gn), dim3(kB), 0, s, pos.ptr, N, flag.ptr);
    XM_LAUNCH_CHECK("cm_unplaced_kernel");
    exclusive_scan_i64(flag.ptr, slot.ptr, N, s);
    hipLaunchKernelGGL(cm_rest_kernel, dim3(gn), dim3(kB), 0, s, slot.ptr, pos0.ptr, N, hi, order.ptr, pos.ptr);
    XM_LAUNCH_CHECK("cm_rest_kernel");
  }
  XM_HIP(hipStreamSynchronize(s));
}

struct LaunchTimer {
  std::vector<hipEvent_t> ev;
  void start(hipStream_t s) { ev.push_back(record(s)); }
  void stop(hipStream_t s) { ev.push_back(record(s)); }
  static hipEvent_t record(hipStream_t s) {
    hipEvent_t e;
    XM_HIP(hipEventCreate(&e));
    XM_HIP(hipEventRecord(e, s));
    return e;
  }
  double total() {
    double ms = 0.0;
    if (!ev.empty()) XM_HIP(hipEventSynchronize(ev.back()));
    for (size_t k = 0; k + 1 < ev.size(); k += 2) {
      float t = 0.f;
      XM_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      ms += t;
    }
    return ms;
  }
  ~LaunchTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

int bits_for(uint64_t v) {  // number of bits needed to represent values < v
  int b = 1;
  while (b < 64 && (uint64_t(1) << b) < v) ++b;
  return b;
}


// rows row0 .. row0 + nrows of Q in frame-index order (Q is stored in the frame order)
__global__ void q_rows_kernel(const double* __restrict__ Q, int32_t ld, int32_t n3, const int32_t* __restrict__ pos,
                              int32_t row0, double* __restrict__ out) {
  const int t = blockIdx.x;  // grid: x = row, y = column tile
  const int c = blockIdx.y * kB + threadIdx.x;
  if (c >= n3) return;
  const int r = row0 + t;
  const int64_t pr = 3 * static_cast<int64_t>(pos[r / 3]) + r % 3;
  const int64_t pc = 3 * static_cast<int64_t>(pos[c / 3]) + c % 3;
  out[static_cast<int64_t>(t) * n3 + c] = Q[pr * ld + pc];
}

}  // namespace

std::unique_ptr<xm_problem> build_problem(int32_t N, int32_t M, int64_t n_obs, const int32_t* frame,
                                          const int32_t* landmark, const void* u, xm_dtype u_dtype,
                                          const void* w, xm_dtype w_dtype, const uint8_t* mask, uint32_t copies,
                                          hipStream_t s) {
  require(N >= 2 && N < 65536, XM_EINVAL, "N must be in [2, 65535]");
  require(M >= 1, XM_EINVAL, "M must be >= 1");
  require(n_obs >= 1 && n_obs < (int64_t(1) << 31), XM_EINVAL, "n_obs must be in [1, 2^31)");
  require(frame && landmark && u, XM_EINVAL, "frame, landmark and u must be non-NULL");
  require(u_dtype == XM_F64 || u_dtype == XM_F32, XM_EINVAL, "u_dtype must be XM_F64 or XM_F32");
  require(!w || w_dtype == XM_F64 || w_dtype == XM_F32, XM_EINVAL, "w_dtype must be XM_F64 or XM_F32");
  require((copies & ~(XM_KEEP_F32 | XM_KEEP_BF16 | 1u)) == 0, XM_EINVAL, "unknown bits in copies");

  hipEvent_t ev0, ev1;
  XM_HIP(hipEventCreate(&ev0));
  XM_HIP(hipEventCreate(&ev1));
  XM_HIP(hipEventRecord(ev0, s));

  auto P = std::make_unique<xm_problem>();
  P->N = N; P->M = M; P->n_obs = n_obs; P->n_in = n_obs; P->n3 = 3 * N;
  P->ld = static_cast<int32_t>(round_up(3 * static_cast<size_t>(N), 64));
  const int u32 = (u_dtype == XM_F32), w32 = (w_dtype == XM_F32);
  int64_t n = n_obs;

  // a1: validate
  DevBuf<int> flags(8);
  XM_HIP(hipMemsetAsync(flags.ptr, 0, 8 * sizeof(int), s));
  hipLaunchKernelGGL(validate_kernel, dim3(cdiv(n, kB)), dim3(kB), 0, s, N, M, n, frame, landmark, u, u32,
                     w, w32, flags.ptr);
  XM_LAUNCH_CHECK("validate_kernel");
  int hflags[8];
  XM_HIP(hipMemcpyAsync(hflags, flags.ptr, sizeof(hflags), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  require(!hflags[0], XM_EINVAL, "frame or landmark index out of range");
  require(!hflags[1], XM_EINVAL, "non-finite keypoint u");
  require(!hflags[2], XM_EINVAL, "weights must be finite and > 0");
  if (mask) {
    // observations with mask 0 are left out: they sort past every landmark and
    // only the first n (kept) sorted entries are gathered
    DevBuf<unsigned long long> cnt(1);
    XM_HIP(hipMemsetAsync(cnt.ptr, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(count_kept_kernel, dim3(cdiv(n_obs, kB)), dim3(kB), 0, s, mask, n_obs, cnt.ptr);
    XM_LAUNCH_CHECK("count_kept_kernel");
    unsigned long long kept = 0;
    XM_HIP(hipMemcpyAsync(&kept, cnt.ptr, sizeof(kept), hipMemcpyDeviceToHost, s));
    XM_HIP(hipStreamSynchronize(s));
    require(kept >= 1, XM_EINVAL, "the mask keeps no observation");
    n = static_cast<int64_t>(kept);
    P->n_obs = n;
  }

  // a1: sort observations by landmark
  {
    DevBuf<uint32_t> keys(n_obs), ktmp(n_obs);
    DevBuf<uint64_t> vals(n_obs), vtmp(n_obs);
    hipLaunchKernelGGL(iota_kernel, dim3(cdiv(n_obs, kB)), dim3(kB), 0, s, landmark, mask, M, n_obs, keys.ptr,
                       vals.ptr);
    XM_LAUNCH_CHECK("iota_kernel");
    radix_sort_pairs(keys.ptr, vals.ptr, ktmp.ptr, vtmp.ptr, n_obs,
                     bits_for(static_cast<uint64_t>(M) + (mask ? 1 : 0)), s);
    P->fr_s.alloc(n); P->lm_s.alloc(n); P->u_s.alloc(3 * n); P->w_s.alloc(n); P->perm.alloc(n);
    hipLaunchKernelGGL(gather_obs_kernel, dim3(cdiv(n, kB)), dim3(kB), 0, s, vals.ptr, n, frame, landmark, u,
                       u32, w, w32, P->fr_s.ptr, P->lm_s.ptr, P->u_s.ptr, P->w_s.ptr, P->perm.ptr);
    XM_LAUNCH_CHECK("gather_obs_kernel");
    XM_HIP(hipStreamSynchronize(s));
  }
  P->lm_ptr.alloc(M + 1);
  hipLaunchKernelGGL(segment_offsets_kernel, dim3(cdiv(n + 1, kB)), dim3(kB), 0, s, P->lm_s.ptr, n,
                     static_cast<int64_t>(M), P->lm_ptr.ptr);
  XM_LAUNCH_CHECK("segment_offsets_kernel");
  P->Wl.alloc(M);
  DevBuf<int64_t> poff(M + 1);
  hipLaunchKernelGGL(landmark_stats_kernel, dim3(cdiv(M, kB)), dim3(kB), 0, s, P->lm_ptr.ptr, M, P->w_s.ptr,
                     P->Wl.ptr, poff.ptr);
  XM_LAUNCH_CHECK("landmark_stats_kernel");
  exclusive_scan_i64(poff.ptr, poff.ptr, M, s);
  int64_t npairs = 0;
  XM_HIP(hipMemcpyAsync(&npairs, poff.ptr + M, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  require(npairs > 0, XM_EGRAPH, "no landmark is observed twice");
  require(npairs < (int64_t(1) << 31), XM_EINVAL, "too many observation pairs (sum of squared track lengths)");
  P->n_pairs = npairs;

  // a2-i: emit and sort observation pairs by frame pair
  DevBuf<uint32_t> pkeys(npairs);
  DevBuf<uint64_t> pvals(npairs);
  {
    DevBuf<uint32_t> ktmp(npairs);
    DevBuf<uint64_t> vtmp(npairs);
    hipLaunchKernelGGL(emit_pairs_kernel, dim3(cdiv(M, kB)), dim3(kB), 0, s, P->lm_ptr.ptr, M, N, P->fr_s.ptr,
                       poff.ptr, pkeys.ptr, pvals.ptr);
    XM_LAUNCH_CHECK("emit_pairs_kernel");
    radix_sort_pairs(pkeys.ptr, pvals.ptr, ktmp.ptr, vtmp.ptr, npairs,
                     bits_for(static_cast<uint64_t>(N) * static_cast<uint64_t>(N)), s);
  }
  poff.release();
  DevBuf<int64_t> sidx(npairs + 1);
  hipLaunchKernelGGL(head_flags_kernel, dim3(cdiv(npairs, kB)), dim3(kB), 0, s, pkeys.ptr, npairs, sidx.ptr);
  XM_LAUNCH_CHECK("head_flags_kernel");
  exclusive_scan_i64(sidx.ptr, sidx.ptr, npairs, s);
  int64_t S = 0;
  XM_HIP(hipMemcpyAsync(&S, sidx.ptr + npairs, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  P->nnzb = S;
  DevBuf<int64_t> seg_start(S + 1);
  DevBuf<uint32_t> seg_key(S);
  hipLaunchKernelGGL(segment_starts_kernel, dim3(cdiv(npairs + 1, kB)), dim3(kB), 0, s, pkeys.ptr, sidx.ptr,
                     npairs, seg_start.ptr, seg_key.ptr);
  XM_LAUNCH_CHECK("segment_starts_kernel");
  sidx.release();

  // Q storage (zeroed on and right of the diagonal blocks; the lower triangle
  // is written from the upper one at the end) and the per-block reduction
  const size_t qn = static_cast<size_t>(P->n3) * P->ld;
  P->Q64.alloc(qn);
  hipLaunchKernelGGL(zero_upper_kernel, dim3(P->n3), dim3(kB), 0, s, P->Q64.ptr, P->ld);
  XM_LAUNCH_CHECK("zero_upper_kernel");
  P->row_ptr.alloc(N + 1);
  P->col.alloc(S);
  hipLaunchKernelGGL(pattern_kernel, dim3(cdiv(S + 1, kB)), dim3(kB), 0, s, seg_key.ptr, S, N, P->row_ptr.ptr,
                     P->col.ptr);
  XM_LAUNCH_CHECK("pattern_kernel");
  // frame order (Cuthill-McKee): Q is stored and assembled in it
  cm_order(N, P->row_ptr.ptr, P->col.ptr, P->order, P->pos, s);
  P->Art.alloc(3 * S);
  P->Att.alloc(S);
  P->fac.alloc(15 * S);
  {
    DevBuf<double> rec(8 * static_cast<size_t>(n));
    hipLaunchKernelGGL(obs_record_kernel, dim3(cdiv(n, kB)), dim3(kB), 0, s, n, P->u_s.ptr, P->w_s.ptr,
                       P->lm_s.ptr, P->Wl.ptr, rec.ptr);
    XM_LAUNCH_CHECK("obs_record_kernel");
    hipLaunchKernelGGL(reduce_blocks_kernel, dim3(cdiv(S, kB / kRedLanes)), dim3(kB), 0, s, seg_start.ptr,
                       seg_key.ptr, S, N, pvals.ptr, rec.ptr, P->pos.ptr, P->Q64.ptr, P->ld, P->Art.ptr, P->Att.ptr,
                       P->fac.ptr);
    XM_LAUNCH_CHECK("reduce_blocks_kernel");
  }
  hipLaunchKernelGGL(check_diag_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, s, P->row_ptr.ptr, P->col.ptr,
                     P->Att.ptr, N, flags.ptr);
  XM_LAUNCH_CHECK("check_diag_kernel");
  hipLaunchKernelGGL(transpose_art_kernel, dim3(cdiv(S, kB)), dim3(kB), 0, s, P->row_ptr.ptr, P->col.ptr,
                     P->Art.ptr, N, S, P->fac.ptr + 12 * S, flags.ptr);
  XM_LAUNCH_CHECK("transpose_art_kernel");
  XM_HIP(hipMemcpyAsync(hflags, flags.ptr, sizeof(hflags), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  pkeys.release(); pvals.release(); seg_start.release(); seg_key.release();
  require(!hflags[3], XM_EGRAPH, "a frame has no observation shared with another frame");
  require(!hflags[5], XM_EINVAL, "internal: co-visibility pattern is not symmetric");

  // a2-ii: translations.  G = A_tt[1:,1:] (dense), swept to -G^{-1}.
  const int32_t ng = N - 1;
  P->ldg = static_cast<int32_t>(round_up(ng, 64));
  P->Gm.alloc(static_cast<size_t>(ng) * P->ldg);
  XM_HIP(hipMemsetAsync(P->Gm.ptr, 0, P->Gm.bytes(), s));
  hipLaunchKernelGGL(scatter_grounded_kernel, dim3(N), dim3(kB), 0, s, P->row_ptr.ptr, P->col.ptr, P->Att.ptr,
                     N, P->Gm.ptr, P->ldg);
  XM_LAUNCH_CHECK("scatter_grounded_kernel");
  {
    // scale for the pivot test: largest diagonal of G
    double dscale = 0.0;
    {
      DevBuf<double> dm(1);
      hipLaunchKernelGGL(diag_max_kernel, dim3(1), dim3(kB), 0, s, P->Gm.ptr, ng, P->ldg, dm.ptr);
      XM_LAUNCH_CHECK("diag_max_kernel");
      XM_HIP(hipMemcpyAsync(&dscale, dm.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
      XM_HIP(hipStreamSynchronize(s));
    }
    require(dscale > 0.0, XM_EGRAPH, "the grounded Laplacian has no positive diagonal entry");
    // Dinv of the current and of the next step; Dsave: copy of the next pivot block
    DevBuf<double> Dinv(2 * kNB * kNB), Dsave(kNB * kNB);
    DevBuf<double> Ct(static_cast<size_t>(kNB) * P->ldg), Pt(static_cast<size_t>(kNB) * P->ldg);
    const std::vector<int32_t> htiles = sweep_tile_list(static_cast<int>(cdiv(ng, 64)));
    const int32_t ntiles = static_cast<int32_t>(htiles.size() / 2);
    DevBuf<int32_t> tiles(htiles.size());
    XM_HIP(hipMemcpy(tiles.ptr, htiles.data(), htiles.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    const unsigned ublocks = 8 * cdiv(ntiles, 8);
    // The inversion of the next pivot block runs on a second stream while the
    // trailing update of the current step runs on s (look-ahead).
    struct SideStream {
      hipStream_t st = nullptr;
      hipEvent_t panel_done = nullptr, pivot_done = nullptr;
      ~SideStream() {
        if (panel_done) (void)hipEventDestroy(panel_done);
        if (pivot_done) (void)hipEventDestroy(pivot_done);
        if (st) (void)hipStreamDestroy(st);
      }
    } side;
    XM_HIP(hipStreamCreateWithFlags(&side.st, hipStreamNonBlocking));
    XM_HIP(hipEventCreateWithFlags(&side.panel_done, hipEventDisableTiming));
    XM_HIP(hipEventCreateWithFlags(&side.pivot_done, hipEventDisableTiming));
    LaunchTimer t_sweep;
    hipLaunchKernelGGL(sweep_pivot_kernel, dim3(1), dim3(kPivotThreads), 0, s, P->Gm.ptr, P->ldg, 0,
                       std::min(kNB, ng), dscale, nullptr, nullptr, nullptr, 0, 0, Dinv.ptr, flags.ptr);
    XM_LAUNCH_CHECK("sweep_pivot_kernel");
    for (int32_t k0 = 0, step = 0; k0 < ng; k0 += kNB, ++step) {
      const int32_t nb = std::min(kNB, ng - k0);
      const int32_t k1 = k0 + kNB, nb1 = std::max(0, std::min(kNB, ng - k1));
      double* Dk = Dinv.ptr + (step & 1) * kNB * kNB;
      double* Dn = Dinv.ptr + ((step + 1) & 1) * kNB * kNB;
      if (step > 0) XM_HIP(hipStreamWaitEvent(s, side.pivot_done, 0));
      hipLaunchKernelGGL(sweep_panel_kernel, dim3(cdiv(ng, 64) + (nb1 > 0 ? 1 : 0), kNB / 64), dim3(kB), 0, s,
                         P->Gm.ptr, P->ldg, ng, k0, nb, Dk, Ct.ptr, Pt.ptr, P->ldg, k1, nb1, Dsave.ptr);
      XM_LAUNCH_CHECK("sweep_panel_kernel");
      if (nb1 > 0) {
        XM_HIP(hipEventRecord(side.panel_done, s));
        XM_HIP(hipStreamWaitEvent(side.st, side.panel_done, 0));
        hipLaunchKernelGGL(sweep_pivot_kernel, dim3(1), dim3(kPivotThreads), 0, side.st, P->Gm.ptr, P->ldg, k1,
                           nb1, dscale, Dsave.ptr, Ct.ptr, Pt.ptr, P->ldg, nb, Dn, flags.ptr);
        XM_LAUNCH_CHECK("sweep_pivot_kernel");
        XM_HIP(hipEventRecord(side.pivot_done, side.st));
      }
      t_sweep.start(s);
      hipLaunchKernelGGL(sweep_update_kernel, dim3(ublocks), dim3(kB), 0, s, P->Gm.ptr, P->ldg, ng, Ct.ptr,
                         Pt.ptr, P->ldg, nb, tiles.ptr, ntiles);
      XM_LAUNCH_CHECK("sweep_update_kernel");
      t_sweep.stop(s);
      hipLaunchKernelGGL(sweep_finish_kernel, dim3(cdiv(ng, kB), nb), dim3(kB), 0, s, P->Gm.ptr, P->ldg, ng, k0,
                         nb, Ct.ptr, P->ldg, Dk);
      XM_LAUNCH_CHECK("sweep_finish_kernel");
    }
    {
      const unsigned T = cdiv(ng, 32);
      hipLaunchKernelGGL(symmetrize_kernel, dim3(T, T), dim3(kB), 0, s, P->Gm.ptr, ng, P->ldg, nullptr);
      XM_LAUNCH_CHECK("symmetrize_kernel(G)");
    }
    XM_HIP(hipMemcpyAsync(hflags, flags.ptr, sizeof(hflags), hipMemcpyDeviceToHost, s));
    XM_HIP(hipStreamSynchronize(s));
    require(!hflags[4], XM_EGRAPH, "the view graph is disconnected (grounded Laplacian is singular)");
    // per step: the upper triangle of G read and written once, nb * ng^2 FMA-pairs over it
    const double g2 = static_cast<double>(ng) * ng;
    P->build_stats.push_back({"sweep_update_kernel", static_cast<int>(cdiv(ng, kNB)), t_sweep.total(),
                              cdiv(ng, kNB) * 8.0 * g2, static_cast<double>(ng) * g2});
  }

  // P = A_rt[:,1:] (-G^{-1})   (3N x (N-1)), then Pt = P^T, then Q += A_rt[:,1:] Pt,
  // both products over groups of frames consecutive in the Cuthill-McKee order
  {
    const int32_t ngroups = static_cast<int32_t>(cdiv(N, kGroup));
    const int nw = (N + 31) / 32;
    const size_t lds = 2 * static_cast<size_t>(nw) * sizeof(uint32_t);
    DevBuf<int64_t> ucount(ngroups);
    DevBuf<int64_t>& ustart = P->grp_ustart;
    DevBuf<int32_t>& uid = P->grp_uid;
    ustart.alloc(ngroups + 1);
    hipLaunchKernelGGL(group_count_kernel, dim3(ngroups), dim3(kB), lds, s, N, P->order.ptr, P->row_ptr.ptr,
                       P->col.ptr, ucount.ptr);
    XM_LAUNCH_CHECK("group_count_kernel");
    exclusive_scan_i64(ucount.ptr, ustart.ptr, ngroups, s);
    std::vector<int64_t> hcount(ngroups + 1);
    XM_HIP(hipMemcpyAsync(hcount.data(), ustart.ptr, (ngroups + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    XM_HIP(hipStreamSynchronize(s));
    const int64_t total = hcount[ngroups];
    int64_t maxu = 0;
    for (int32_t g = 0; g < ngroups; ++g) maxu = std::max(maxu, hcount[g + 1] - hcount[g]);
    uid.alloc(std::max<int64_t>(total, 1));
    P->lidx.alloc(std::max<int64_t>(P->nnzb, 1));
    DevBuf<double> coef(std::max<int64_t>(total, 1) * 4 * kGroup);
    XM_HIP(hipMemsetAsync(coef.ptr, 0, coef.bytes(), s));
    hipLaunchKernelGGL(group_fill_kernel, dim3(ngroups), dim3(kB), lds, s, N, P->order.ptr, P->row_ptr.ptr,
                       P->col.ptr, P->Art.ptr, ustart.ptr, uid.ptr, coef.ptr, P->lidx.ptr);
    XM_LAUNCH_CHECK("group_fill_kernel");
    P->grp_maxu = static_cast<int32_t>(maxu);
    {
      int dev = 0, lmax = 0;
      XM_HIP(hipGetDevice(&dev));
      XM_HIP(hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      P->lds_max = static_cast<size_t>(std::max(lmax, 0));
    }
    // workgroup lists of the two passes: tile-major (group, column tile) pairs;
    // the Q pass only takes the pairs with columns right of the group's first row
    auto tile_list = [&](int32_t K, bool upper, DevBuf<int32_t>& ts) {
      const int32_t nt = static_cast<int32_t>(cdiv(K, kGroupCols));
      std::vector<int32_t> h(nt + 1, 0);
      for (int32_t y = 0; y < nt; ++y) {
        const int64_t gmax = upper ? std::min<int64_t>(ngroups, ((y + 1) * int64_t(kGroupCols) + 3 * kGroup - 1) /
                                                                     (3 * kGroup))
                                   : ngroups;
        h[y + 1] = h[y] + static_cast<int32_t>(gmax);
      }
      ts.alloc(nt + 1);
      XM_HIP(hipMemcpy(ts.ptr, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      return std::make_pair(nt, h[nt]);
    };
    DevBuf<int32_t> tsP, tsQ;
    const auto lp = tile_list(ng, false, tsP);
    const auto lq = tile_list(P->n3, true, tsQ);
    const int32_t ldp = static_cast<int32_t>(round_up(ng, 64));
    DevBuf<double> Pm(static_cast<size_t>(P->n3) * ldp);
    LaunchTimer t_gather, t_gather_q;
    t_gather.start(s);
    hipLaunchKernelGGL((group_product_kernel<false>), dim3(lp.second), dim3(kB), 0, s, N, tsP.ptr, lp.first,
                       ustart.ptr, uid.ptr, coef.ptr, P->Gm.ptr, P->ldg, ng, Pm.ptr, ldp);
    XM_LAUNCH_CHECK("group_product_kernel(P)");
    t_gather.stop(s);
    DevBuf<double> Ptr(static_cast<size_t>(ng) * P->ld);
    hipLaunchKernelGGL(transpose_kernel, dim3(cdiv(ng, 64), cdiv(P->n3, 64)), dim3(kB), 0, s, Pm.ptr, P->n3, ng,
                       ldp, Ptr.ptr, P->ld);
    XM_LAUNCH_CHECK("transpose_kernel");
    Pm.release();
    t_gather_q.start(s);
    hipLaunchKernelGGL((group_product_kernel<true>), dim3(lq.second), dim3(kB), 0, s, N, tsQ.ptr, lq.first,
                       ustart.ptr, uid.ptr, coef.ptr, Ptr.ptr, P->ld, P->n3, P->Q64.ptr, P->ld);
    XM_LAUNCH_CHECK("group_product_kernel(Q)");
    t_gather_q.stop(s);
    XM_HIP(hipStreamSynchronize(s));
    // P pass: G^{-1} read once, P written once, 3 FMAs per (stored block, column);
    // Q pass: P^T read once, the upper triangle written once, half the columns
    const double nnz_off = static_cast<double>(S);  // every stored block of A_rt (the few with j = 0 are skipped)
    P->build_stats.push_back({"group_product_kernel (P)", 1, t_gather.total(),
                              8.0 * (static_cast<double>(ng) * ng + 3.0 * N * ng), 6.0 * nnz_off * ng});
    P->build_stats.push_back({"group_product_kernel (Q)", 1, t_gather_q.total(),
                              8.0 * (static_cast<double>(ng) * P->n3 + 0.5 * static_cast<double>(P->n3) * P->n3),
                              6.0 * nnz_off * P->n3 * 0.5});
  }
  {
    // the FP32 copy of Q (XM_KEEP_F32) is written while the lower triangle is filled
    float* q32 = nullptr;
    if (copies & XM_KEEP_F32) {
      P->Q32.alloc(qn);
      hipLaunchKernelGGL(zero_pad_kernel, dim3(P->n3), dim3(kB), 0, s, P->Q32.ptr, P->n3, P->ld);
      XM_LAUNCH_CHECK("zero_pad_kernel");
      q32 = P->Q32.ptr;
    }
    const unsigned T = cdiv(P->n3, 32);
    hipLaunchKernelGGL(symmetrize_kernel, dim3(T, T), dim3(kB), 0, s, P->Q64.ptr, P->n3, P->ld, q32);
    XM_LAUNCH_CHECK("symmetrize_kernel");
    DevBuf<double> tr(1);
    hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(kB), 0, s, P->Q64.ptr, P->n3, P->ld, tr.ptr);
    XM_LAUNCH_CHECK("trace_kernel");
    double htr = 0.0;
    XM_HIP(hipMemcpyAsync(&htr, tr.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
    XM_HIP(hipStreamSynchronize(s));
    P->qbar = htr / P->n3;
  }
  P->qkk.alloc(N);
  hipLaunchKernelGGL(diag_block_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, s, P->Q64.ptr, N, P->ld, P->pos.ptr,
                     P->qkk.ptr);
  XM_LAUNCH_CHECK("diag_block_kernel");
  {
    P->Dhalf.alloc(9 * static_cast<size_t>(N));
    P->Dmhalf.alloc(9 * static_cast<size_t>(N));
    DevBuf<double> ext(2 * static_cast<size_t>(N));
    hipLaunchKernelGGL(block_sqrt_kernel, dim3(cdiv(N, kB)), dim3(kB), 0, s, P->Q64.ptr, N, P->ld, P->pos.ptr,
                       P->Dhalf.ptr,
                       P->Dmhalf.ptr, ext.ptr);
    XM_LAUNCH_CHECK("block_sqrt_kernel");
    std::vector<double> he(2 * static_cast<size_t>(N));
    XM_HIP(hipMemcpyAsync(he.data(), ext.ptr, he.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    XM_HIP(hipStreamSynchronize(s));
    P->dmin = he[0];
    P->dmax = he[1];
    for (int k = 0; k < N; ++k) {
      P->dmin = std::min(P->dmin, he[2 * k]);
      P->dmax = std::max(P->dmax, he[2 * k + 1]);
    }
  }
  if (copies & XM_KEEP_F32) {
    // FP32 factors for the factored curvature product
    auto to32 = [&](const DevBuf<double>& src, DevBuf<float>& dst) {
      dst.alloc(src.n);
      hipLaunchKernelGGL(to_f32_kernel, dim3(cdiv(src.n, kF32Per * kB)), dim3(kB), 0, s, src.ptr,
                         static_cast<int64_t>(src.n), dst.ptr);
      XM_LAUNCH_CHECK("to_f32_kernel");
    };
    to32(P->fac, P->fac32);
    to32(P->Gm, P->Gm32);
    // FP32 curvature products from the factors once the dense upper triangle
    // no longer stays resident in the 256 MiB last-level cache
    const double upper_bytes = 0.5 * static_cast<double>(P->n3) * (P->n3 + 1) * sizeof(float);
    if (upper_bytes > 256.0 * 1024 * 1024) P->spmm_kind[XM_ROLE_CURVATURE][XM_F32] = XM_SPMM_FACTORED;
  }
  if (copies & XM_KEEP_BF16) {
    P->Q16.alloc(qn);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(cdiv(qn, kB)), dim3(kB), 0, s, P->Q64.ptr, static_cast<int64_t>(qn),
                       P->Q16.ptr);
    XM_LAUNCH_CHECK("to_bf16_kernel");
  }
  P->copies = 1u | copies;
  XM_HIP(hipEventRecord(ev1, s));
  XM_HIP(hipEventSynchronize(ev1));
  float ms = 0.f;
  XM_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  P->build_ms = ms;
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  return P;
}

void get_q_rows(const xm_problem* p, int32_t row0, int32_t nrows, double* out, hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(q_rows_kernel, dim3(nrows, cdiv(p->n3, kB)), dim3(kB), 0, s, p->Q64.ptr, p->ld, p->n3,
                     p->pos.ptr, row0, out);
  XM_LAUNCH_CHECK("q_rows_kernel");
}

}  // namespace xm
