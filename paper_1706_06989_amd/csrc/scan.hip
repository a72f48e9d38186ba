// Device-wide exclusive prefix sums (reduce -> scan of block sums -> down-sweep).
// Deterministic: integer sums in a fixed tree order.  In place is allowed.
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;  // threads per block (4 waves of 64)
constexpr int kIT = 8;    // consecutive items per thread
constexpr int kChunk = kBS * kIT;

template <typename T>
__device__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// exclusive scan of one value per thread across the block; block total in *tot
template <typename T>
__device__ T block_excl_scan(T v, T* tot) {
  __shared__ T wsum[kBS / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  T off = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kBS / 64; ++i) {
    if (i < w) off += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *tot = all;
  return off + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(kBS) k_reduce(const T* __restrict__ in, int64_t n, T* __restrict__ bsum) {
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  T s = 0;
#pragma unroll
  for (int i = 0; i < kIT; ++i) {
    int64_t idx = base + i * kBS + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  T tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// scans one chunk per block; offs (may be null) holds each block's exclusive prefix;
// writes out[0..n) and out[n] = total
template <typename T>
__global__ void __launch_bounds__(kBS) k_scan_chunk(const T* in, T* out, int64_t n,
                                                     const T* __restrict__ offs) {
  __shared__ T tile[kChunk];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
#pragma unroll
  for (int i = 0; i < kIT; ++i) {
    int64_t idx = base + i * kBS + threadIdx.x;
    tile[i * kBS + threadIdx.x] = idx < n ? in[idx] : T(0);
  }
  __syncthreads();
  T v[kIT];
  T s = 0;
#pragma unroll
  for (int i = 0; i < kIT; ++i) {
    v[i] = tile[threadIdx.x * kIT + i];
    s += v[i];
  }
  T tot;
  T ex = block_excl_scan(s, &tot);
  if (offs) ex += offs[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kIT; ++i) {
    tile[threadIdx.x * kIT + i] = ex;
    if (base + threadIdx.x * kIT + i == n - 1) out[n] = ex + v[i];
    ex += v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kIT; ++i) {
    int64_t idx = base + i * kBS + threadIdx.x;
    if (idx < n) out[idx] = tile[i * kBS + threadIdx.x];
  }
}

template <typename T>
__global__ void k_zero_one(T* out) {
  out[0] = 0;
}

template <typename T>
void scan_impl(Ctx& c, const T* in, T* out, int64_t n, DevBuf& tmpbuf) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_zero_one<T>, dim3(1), dim3(1), 0, c.stream, out);
    AMFMM_HIP(hipGetLastError());
    return;
  }
  // block-sum arrays of every recursion level, carved from one buffer
  std::vector<int64_t> sizes;
  for (int64_t m = n; m > kChunk;) {
    m = (m + kChunk - 1) / kChunk;
    sizes.push_back(m);
  }
  size_t total = 0;
  for (int64_t s : sizes) total += (size_t)(s + 1);
  T* tmp = (T*)ensure(c, tmpbuf, sizeof(T) * (total + 1));
  std::vector<T*> lev;
  size_t off = 0;
  for (int64_t s : sizes) {
    lev.push_back(tmp + off);
    off += (size_t)(s + 1);
  }
  // up-sweep
  const T* src = in;
  int64_t m = n;
  for (size_t l = 0; l < sizes.size(); ++l) {
    hipLaunchKernelGGL(k_reduce<T>, dim3((unsigned)sizes[l]), dim3(kBS), 0, c.stream, src, m, lev[l]);
    AMFMM_HIP(hipGetLastError());
    src = lev[l];
    m = sizes[l];
  }
  // top level in one block (in place), then down-sweeps
  if (!sizes.empty()) {
    T* top = lev.back();
    hipLaunchKernelGGL(k_scan_chunk<T>, dim3(1), dim3(kBS), 0, c.stream, top, top, sizes.back(),
                       (const T*)nullptr);
    AMFMM_HIP(hipGetLastError());
    for (int l = (int)sizes.size() - 2; l >= 0; --l) {
      hipLaunchKernelGGL(k_scan_chunk<T>, dim3((unsigned)sizes[l + 1]), dim3(kBS), 0, c.stream,
                         lev[l], lev[l], sizes[l], (const T*)lev[l + 1]);
      AMFMM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_scan_chunk<T>, dim3((unsigned)sizes[0]), dim3(kBS), 0, c.stream, in, out, n,
                       (const T*)lev[0]);
  } else {
    hipLaunchKernelGGL(k_scan_chunk<T>, dim3(1), dim3(kBS), 0, c.stream, in, out, n, (const T*)nullptr);
  }
  AMFMM_HIP(hipGetLastError());
}

}  // namespace

void scan_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n) { scan_impl<int32_t>(c, in, out, n, c.scratch); }
void scan_i64(Ctx& c, const int64_t* in, int64_t* out, int64_t n) { scan_impl<int64_t>(c, in, out, n, c.scratch); }

}  // namespace amfmm
