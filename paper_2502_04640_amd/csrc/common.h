// Internal definitions shared by the HIP sources of libxm (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/xm.h"

namespace xm {

// ---------------------------------------------------------------------------
// Errors: C++ exceptions inside the library, converted to xm_status at the ABI.
struct Error : public std::runtime_error {
  xm_status code;
  Error(xm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(XM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define XM_HIP(expr) ::xm::hip_check((expr), #expr)
#define XM_LAUNCH_CHECK(name) ::xm::hip_check(hipGetLastError(), name)

inline void require(bool ok, xm_status code, const std::string& msg) {
  if (!ok) throw Error(code, msg);
}

// ---------------------------------------------------------------------------
// Device memory of the library (pool.cpp).  Freed blocks are kept per device
// and handed out again to requests of about their size, so that repeated
// builds and solves of one problem shape allocate nothing from the runtime
// once the first has run.  pool_free waits for the device to go idle before
// it recycles the block (the same ordering hipFree gives), so a block is never
// handed out while a kernel may still use it.  pool_alloc throws XM_ENOMEM
// (after releasing the cached blocks and retrying once).
void* pool_alloc(size_t bytes);
void pool_free(void* ptr);
// Return every cached (free) block of every device to the runtime; the
// number of bytes released.
size_t pool_trim();
// Bytes held in live blocks and in cached blocks, over all devices.
void pool_usage(size_t* live, size_t* cached);

// ---------------------------------------------------------------------------
// Owning device buffer (memory from the pool above).
template <typename T>
struct DevBuf {
  T* ptr = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), n(o.n) { o.ptr = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); ptr = o.ptr; n = o.n; o.ptr = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    ptr = static_cast<T*>(pool_alloc(count * sizeof(T)));
    n = count;
  }
  // grow-only reallocation (contents are not kept)
  void ensure(size_t count) {
    if (count > n) alloc(count);
  }
  void release() {
    if (ptr) pool_free(ptr);
    ptr = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Pinned host scratch for scalars read back after a stream sync.
struct HostScalars {
  double* p = nullptr;
  size_t n = 0;
  explicit HostScalars(size_t count = 64) {
    XM_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), count * sizeof(double), hipHostMallocDefault));
    n = count;
  }
  HostScalars(const HostScalars&) = delete;
  HostScalars& operator=(const HostScalars&) = delete;
  ~HostScalars() { if (p) (void)hipHostFree(p); }
};

inline unsigned cdiv(size_t a, size_t b) { return static_cast<unsigned>((a + b - 1) / b); }
inline size_t round_up(size_t a, size_t b) { return ((a + b - 1) / b) * b; }

// ---------------------------------------------------------------------------
// Device helpers.
#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NV>
struct Pow2Up {  // smallest power of two >= NV
  static constexpr int v = NV <= 1 ? 1 : 2 * Pow2Up<(NV + 1) / 2>::v;
};
template <>
struct Pow2Up<1> {
  static constexpr int v = 1;
};
template <int P>
struct Log2 {  // log2 of a power of two
  static constexpr int v = 1 + Log2<P / 2>::v;
};
template <>
struct Log2<1> {
  static constexpr int v = 0;
};

// Sums each of NP per-lane values (NP a power of two, at most W) over aligned
// groups of W lanes by recursive halving: at the exchange over lane distance o
// a lane keeps the half of its values that its partner sends away and adds
// the partner's copy of it, so the NP sums take NP - 1 exchanges, plus
// log2(W / NP) for the last value, instead of NP log2(W).  `lane` is the
// index within the group; it returns the total of value
// group_split_index<NP, W>(lane), and the lanes whose bits below W / NP are
// zero hold each index once.  Every total is summed over the lane bits from
// the highest down, as wave_sum does, so the results are bitwise those of NP
// separate wave_sum calls.
template <int NP, int W, typename T>
__device__ __forceinline__ T group_split_sum(T (&v)[NP], int lane) {
  static_assert(NP >= 1 && (NP & (NP - 1)) == 0 && NP <= W && W <= 64 && (W & (W - 1)) == 0,
                "NP and W: powers of two, NP <= W <= 64");
  constexpr int kSteps = Log2<NP>::v, kAll = Log2<W>::v;
#pragma unroll
  for (int st = 0; st < kSteps; ++st) {
    const int o = (W / 2) >> st, h = NP >> (st + 1);
    const bool b = (lane & o) != 0;
#pragma unroll
    for (int k = 0; k < NP / 2; ++k) {
      if (k < h) {
        // the empty asm hands the two values over as opaque registers, so the
        // selects stay selects of values (not of an index into v, which the
        // compiler would expand into a select chain over the whole array)
        T lo = v[k], hi = v[k + h];
        asm("" : "+v"(lo), "+v"(hi));
        const T send = b ? lo : hi;
        const T keep = b ? hi : lo;
        v[k] = keep + __shfl_xor(send, o, W);
      }
    }
  }
  T t = v[0];
#pragma unroll
  for (int st = kSteps; st < kAll; ++st) t += __shfl_xor(t, (W / 2) >> st, W);
  return t;
}
template <int NP, int W>
__device__ __forceinline__ int group_split_index(int lane) {
  int idx = 0;
#pragma unroll
  for (int st = 0; st < Log2<NP>::v; ++st) idx += (lane & ((W / 2) >> st)) ? (NP >> (st + 1)) : 0;
  return idx;
}

// Deterministic block reduction of NQ doubles per thread (fixed tree order).
// `lds` must hold NQ * (blockDim.x / 64) doubles.  Result valid in thread 0.
template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ], double* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0)
    for (int q = 0; q < NQ; ++q) lds[q * nw + wid] = v[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[q * nw + w];
      v[q] = s;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}
#endif

// ---------------------------------------------------------------------------
// Launchers implemented in the .hip files (host-callable).

// sort.hip ------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs by the low `key_bits` bits.
// keys/vals are sorted in place using the scratch buffers.
void radix_sort_pairs(uint32_t* keys, uint64_t* vals, uint32_t* keys_tmp, uint64_t* vals_tmp,
                      int64_t n, int key_bits, hipStream_t s);
// Exclusive prefix sum of int64 values (in -> out, may alias).  Returns nothing;
// the total is written to out[n] (out must hold n + 1 entries).
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
// keep[o] = 0 for the floor(frac n) largest scores (ties: lower index first),
// 1 otherwise; scores must be finite and >= 0.  Returns the number dropped.
int64_t drop_largest(const double* score, int64_t n, double frac, uint8_t* keep, hipStream_t s);
// Frame guard of the deletion: a kept observation of landmark k links its
// frame when k keeps >= 2 observations; for a frame with < min_links links,
// every observation of it and of the landmarks it sees is kept again.  Frame
// and landmark indices are range-checked.  Returns the number restored.
int64_t guard_frames(int32_t N, int32_t M, int64_t n, const int32_t* frame, const int32_t* landmark,
                     int32_t min_links, uint8_t* keep, hipStream_t s);

// reduce.hip ----------------------------------------------------------------
// Deterministic sum of `parts` rows of `nq` doubles laid out [parts][nq] into out[nq].
void sum_partials(const double* partials, int parts, int nq, double* out, hipStream_t s);

}  // namespace xm
