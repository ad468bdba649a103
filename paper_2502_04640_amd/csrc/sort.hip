// Stable LSD radix sort of (u32 key, u64 value) pairs and exclusive prefix sums.
//
// Used by the Q assembly to group observations by landmark and observation
// pairs by frame pair, so that the per-block reductions run without global
// atomics and in a fixed order (bitwise reproducible FP64 Q).
//
// Radix pass (8-bit digits, tiles of 4096 elements, 256 threads):
//   hist:    per-tile digit counts in LDS          -> counts[digit][tile]
//   scan:    exclusive scan of counts (digit-major) -> global output offsets
//   scatter: 16 rounds of 256 elements; the stable rank of an element among
//            equal digits of its round comes from 8 wave ballots (wave64),
//            per-wave digit counts in LDS give the cross-wave prefix.
#include <cmath>

#include "common.h"

namespace xm {
namespace {

constexpr int kBlock = 256;
constexpr int kRounds = 16;
constexpr int kTile = kBlock * kRounds;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                            int64_t n, int shift, int num_tiles,
                                                            uint32_t* __restrict__ counts) {
  __shared__ uint32_t hist[256];
  const int t = threadIdx.x;
  hist[t] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
  for (int q = 0; q < kRounds; ++q) {
    const int64_t e = base + q * kBlock + t;
    if (e < n) atomicAdd(&hist[(keys[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  counts[static_cast<int64_t>(t) * num_tiles + blockIdx.x] = hist[t];
}

__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint64_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint64_t* __restrict__ vout, int64_t n, int shift, int num_tiles,
    const uint32_t* __restrict__ offsets) {
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcnt[4][256];
  const int t = threadIdx.x, wid = t >> 6;
  running[t] = offsets[static_cast<int64_t>(t) * num_tiles + blockIdx.x];
  wcnt[0][t] = wcnt[1][t] = wcnt[2][t] = wcnt[3][t] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
  const uint64_t lt = __lanemask_lt();
  for (int q = 0; q < kRounds; ++q) {
    const int64_t e = base + q * kBlock + t;
    const bool valid = e < n;
    const uint32_t key = valid ? kin[e] : 0u;
    const uint64_t val = valid ? vin[e] : 0ull;
    const uint32_t d = (key >> shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const int on = (d >> bit) & 1u;
      const uint64_t b = __ballot(on);
      m &= on ? b : ~b;
    }
    const uint32_t rank = __popcll(m & lt);
    if (valid && rank == 0) wcnt[wid][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = running[d] + rank;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    running[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    wcnt[0][t] = wcnt[1][t] = wcnt[2][t] = wcnt[3][t] = 0;
    __syncthreads();
  }
}

// ---- exclusive scan (generic over the element type) -------------------------
template <typename T>
__device__ T block_exclusive_scan(T v, T* lds, T* total) {
  // Hillis-Steele over 256 thread totals in LDS.
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    T add = (t >= off) ? lds[t - off] : T(0);
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  T incl = lds[t];
  *total = lds[kBlock - 1];
  __syncthreads();
  return incl - v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scan_tiles_kernel(const T* __restrict__ in, T* out, int64_t n,
                                                           T* __restrict__ tile_sums) {
  __shared__ T lds[kBlock];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  T loc[kScanItems];
  T sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t e = base + i;
    loc[i] = (e < n) ? in[e] : T(0);
    sum += loc[i];
  }
  T total;
  T pre = block_exclusive_scan<T>(sum, lds, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t e = base + i;
    if (e < n) out[e] = pre;
    pre += loc[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scan_sums_kernel(T* sums, int64_t m) {
  // single block: exclusive scan of sums[0..m) in place, total -> sums[m]
  __shared__ T lds[kBlock];
  T carry = 0;
  for (int64_t c0 = 0; c0 < m; c0 += kBlock) {
    const int64_t e = c0 + threadIdx.x;
    T v = (e < m) ? sums[e] : T(0);
    T total;
    T pre = block_exclusive_scan<T>(v, lds, &total);
    if (e < m) sums[e] = carry + pre;
    carry += total;
  }
  if (threadIdx.x == 0) sums[m] = carry;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scan_add_kernel(T* out, int64_t n, const T* __restrict__ sums) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e < n) out[e] += sums[e / kScanTile];
}

template <typename T>
void exclusive_scan(const T* in, T* out, int64_t n, T* tile_sums, hipStream_t s) {
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(scan_tiles_kernel<T>, dim3(static_cast<unsigned>(tiles)), dim3(kBlock), 0, s, in,
                     out, n, tile_sums);
  XM_LAUNCH_CHECK("scan_tiles_kernel");
  hipLaunchKernelGGL(scan_sums_kernel<T>, dim3(1), dim3(kBlock), 0, s, tile_sums, tiles);
  XM_LAUNCH_CHECK("scan_sums_kernel");
  hipLaunchKernelGGL(scan_add_kernel<T>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, out, n,
                     static_cast<const T*>(tile_sums));
  XM_LAUNCH_CHECK("scan_add_kernel");
}

__global__ void write_total_kernel(const int64_t* tile_sums, int64_t tiles, int64_t* out_n) {
  *out_n = tile_sums[tiles];
}

// Sort keys of a score: the bit pattern of a finite double >= 0 grows with its
// value, so its complement sorts the largest first; split into the low and high
// 32-bit words (two stable passes give the order of the whole 64-bit key).
// flag[0] = 1 for a NaN, infinite or negative score.
__global__ void score_keys_kernel(const double* __restrict__ score, int64_t n, uint32_t* __restrict__ lo,
                                  uint32_t* __restrict__ hi, uint64_t* __restrict__ idx, int* flag) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= n) return;
  const double v = score[e];
  if (!(v >= 0.0) || isinf(v)) flag[0] = 1;
  const uint64_t k = ~static_cast<uint64_t>(__double_as_longlong(v >= 0.0 ? v : 0.0));
  lo[e] = static_cast<uint32_t>(k);
  hi[e] = static_cast<uint32_t>(k >> 32);
  idx[e] = static_cast<uint64_t>(e);
}

// high key words in the order of the first pass
__global__ void gather_hi_kernel(const uint64_t* __restrict__ idx, int64_t n, const uint32_t* __restrict__ hi,
                                 uint32_t* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e < n) out[e] = hi[idx[e]];
}

// keep[o] = 0 for the first k entries of the sorted order, 1 for the rest
__global__ void keep_mask_kernel(const uint64_t* __restrict__ idx, int64_t n, int64_t k, uint8_t* __restrict__ keep) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e < n) keep[idx[e]] = (e < k) ? 0 : 1;
}

// Frame guard of the XM^2 deletion.  cnt[k] = kept observations of landmark k;
// flag[0] = 1 for a frame or landmark index out of range.
__global__ void guard_count_kernel(const int32_t* __restrict__ frame, const int32_t* __restrict__ landmark,
                                   const uint8_t* __restrict__ keep, int64_t n, int32_t N, int32_t M,
                                   int32_t* __restrict__ cnt, int* flag) {
  const int64_t o = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (o >= n) return;
  const int32_t i = frame[o], k = landmark[o];
  if (i < 0 || i >= N || k < 0 || k >= M) {
    flag[0] = 1;
    return;
  }
  if (keep[o]) atomicAdd(cnt + k, 1);
}

// links[i] = kept observations of frame i whose landmark keeps >= 2
__global__ void guard_links_kernel(const int32_t* __restrict__ frame, const int32_t* __restrict__ landmark,
                                   const uint8_t* __restrict__ keep, int64_t n,
                                   const int32_t* __restrict__ cnt, int32_t* __restrict__ links) {
  const int64_t o = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (o >= n) return;
  if (keep[o] && cnt[landmark[o]] >= 2) atomicAdd(links + frame[o], 1);
}

// rescued[k] = 1 for every landmark seen by a frame with fewer than min_links
// links (every writer stores the same value)
__global__ void guard_rescue_kernel(const int32_t* __restrict__ frame, const int32_t* __restrict__ landmark,
                                    int64_t n, const int32_t* __restrict__ links, int32_t min_links,
                                    uint8_t* __restrict__ rescued) {
  const int64_t o = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (o >= n) return;
  if (links[frame[o]] < min_links) rescued[landmark[o]] = 1;
}

// keep[o] = 1 again when o's frame is starved or its landmark rescued;
// restored[0] counts the flips
__global__ void guard_restore_kernel(const int32_t* __restrict__ frame, const int32_t* __restrict__ landmark,
                                     int64_t n, const int32_t* __restrict__ links, int32_t min_links,
                                     const uint8_t* __restrict__ rescued, uint8_t* __restrict__ keep,
                                     unsigned long long* restored) {
  const int64_t o = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (o >= n) return;
  if (!keep[o] && (links[frame[o]] < min_links || rescued[landmark[o]])) {
    keep[o] = 1;
    atomicAdd(restored, 1ull);
  }
}

}  // namespace

void radix_sort_pairs(uint32_t* keys, uint64_t* vals, uint32_t* keys_tmp, uint64_t* vals_tmp,
                      int64_t n, int key_bits, hipStream_t s) {
  if (n <= 1) return;
  require(n < (int64_t(1) << 31), XM_EINVAL, "radix sort: too many elements");
  const int num_tiles = static_cast<int>((n + kTile - 1) / kTile);
  const int64_t ncount = static_cast<int64_t>(num_tiles) * 256;
  DevBuf<uint32_t> counts(ncount);
  DevBuf<uint32_t> tile_sums((ncount + kScanTile - 1) / kScanTile + 1);
  uint32_t *ka = keys, *kb = keys_tmp;
  uint64_t *va = vals, *vb = vals_tmp;
  const int passes = (key_bits + 7) / 8;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(num_tiles), dim3(kBlock), 0, s, ka, n, shift,
                       num_tiles, counts.ptr);
    XM_LAUNCH_CHECK("radix_hist_kernel");
    exclusive_scan<uint32_t>(counts.ptr, counts.ptr, ncount, tile_sums.ptr, s);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(num_tiles), dim3(kBlock), 0, s, ka, va, kb, vb, n,
                       shift, num_tiles, counts.ptr);
    XM_LAUNCH_CHECK("radix_scatter_kernel");
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    XM_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    XM_HIP(hipMemcpyAsync(vals, va, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
  }
  // scratch buffers are freed at scope exit: make sure the kernels are done with them
  XM_HIP(hipStreamSynchronize(s));
}

int64_t drop_largest(const double* score, int64_t n, double frac, uint8_t* keep, hipStream_t s) {
  require(score && keep, XM_EINVAL, "score and keep must be non-NULL");
  require(n >= 1 && n < (int64_t(1) << 31), XM_EINVAL, "n must be in [1, 2^31)");
  require(frac >= 0.0 && frac <= 1.0, XM_EINVAL, "frac must be in [0, 1]");
  const int64_t k = static_cast<int64_t>(std::floor(frac * static_cast<double>(n)));
  DevBuf<uint32_t> lo(n), hi(n), tmpk(n);
  DevBuf<uint64_t> idx(n), tmpv(n);
  DevBuf<int> flag(1);
  XM_HIP(hipMemsetAsync(flag.ptr, 0, sizeof(int), s));
  const unsigned g = static_cast<unsigned>((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(score_keys_kernel, dim3(g), dim3(kBlock), 0, s, score, n, lo.ptr, hi.ptr, idx.ptr, flag.ptr);
  XM_LAUNCH_CHECK("score_keys_kernel");
  int hflag = 0;
  XM_HIP(hipMemcpyAsync(&hflag, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  require(!hflag, XM_EINVAL, "scores must be finite and >= 0");
  // stable LSD over the 64-bit key: low word first, then the high word; equal
  // keys keep index order, so ties drop the lower index first
  radix_sort_pairs(lo.ptr, idx.ptr, tmpk.ptr, tmpv.ptr, n, 32, s);
  hipLaunchKernelGGL(gather_hi_kernel, dim3(g), dim3(kBlock), 0, s, idx.ptr, n, hi.ptr, lo.ptr);
  XM_LAUNCH_CHECK("gather_hi_kernel");
  radix_sort_pairs(lo.ptr, idx.ptr, tmpk.ptr, tmpv.ptr, n, 32, s);
  hipLaunchKernelGGL(keep_mask_kernel, dim3(g), dim3(kBlock), 0, s, idx.ptr, n, k, keep);
  XM_LAUNCH_CHECK("keep_mask_kernel");
  XM_HIP(hipStreamSynchronize(s));
  return k;
}

int64_t guard_frames(int32_t N, int32_t M, int64_t n, const int32_t* frame, const int32_t* landmark,
                     int32_t min_links, uint8_t* keep, hipStream_t s) {
  require(frame && landmark && keep, XM_EINVAL, "frame, landmark and keep must be non-NULL");
  require(N >= 1 && M >= 1, XM_EINVAL, "N and M must be >= 1");
  require(n >= 1 && n < (int64_t(1) << 31), XM_EINVAL, "n must be in [1, 2^31)");
  require(min_links >= 0, XM_EINVAL, "min_links must be >= 0");
  DevBuf<int32_t> cnt(M), links(N);
  DevBuf<uint8_t> rescued(M);
  DevBuf<int> flag(1);
  DevBuf<unsigned long long> restored(1);
  XM_HIP(hipMemsetAsync(cnt.ptr, 0, M * sizeof(int32_t), s));
  XM_HIP(hipMemsetAsync(links.ptr, 0, N * sizeof(int32_t), s));
  XM_HIP(hipMemsetAsync(rescued.ptr, 0, M * sizeof(uint8_t), s));
  XM_HIP(hipMemsetAsync(flag.ptr, 0, sizeof(int), s));
  XM_HIP(hipMemsetAsync(restored.ptr, 0, sizeof(unsigned long long), s));
  const unsigned g = static_cast<unsigned>((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(guard_count_kernel, dim3(g), dim3(kBlock), 0, s, frame, landmark,
                     static_cast<const uint8_t*>(keep), n, N, M, cnt.ptr, flag.ptr);
  XM_LAUNCH_CHECK("guard_count_kernel");
  int hflag = 0;
  XM_HIP(hipMemcpyAsync(&hflag, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  require(!hflag, XM_EINVAL, "frame or landmark index out of range");
  hipLaunchKernelGGL(guard_links_kernel, dim3(g), dim3(kBlock), 0, s, frame, landmark,
                     static_cast<const uint8_t*>(keep), n, static_cast<const int32_t*>(cnt.ptr), links.ptr);
  XM_LAUNCH_CHECK("guard_links_kernel");
  hipLaunchKernelGGL(guard_rescue_kernel, dim3(g), dim3(kBlock), 0, s, frame, landmark, n,
                     static_cast<const int32_t*>(links.ptr), min_links, rescued.ptr);
  XM_LAUNCH_CHECK("guard_rescue_kernel");
  hipLaunchKernelGGL(guard_restore_kernel, dim3(g), dim3(kBlock), 0, s, frame, landmark, n,
                     static_cast<const int32_t*>(links.ptr), min_links, static_cast<const uint8_t*>(rescued.ptr),
                     keep, restored.ptr);
  XM_LAUNCH_CHECK("guard_restore_kernel");
  unsigned long long hr = 0;
  XM_HIP(hipMemcpyAsync(&hr, restored.ptr, sizeof(hr), hipMemcpyDeviceToHost, s));
  XM_HIP(hipStreamSynchronize(s));
  return static_cast<int64_t>(hr);
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) {
    XM_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
    XM_HIP(hipStreamSynchronize(s));
    return;
  }
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  DevBuf<int64_t> tile_sums(tiles + 1);
  exclusive_scan<int64_t>(in, out, n, tile_sums.ptr, s);
  hipLaunchKernelGGL(write_total_kernel, dim3(1), dim3(1), 0, s, static_cast<const int64_t*>(tile_sums.ptr),
                     tiles, out + n);
  XM_LAUNCH_CHECK("write_total_kernel");
  XM_HIP(hipStreamSynchronize(s));
}

}  // namespace xm
