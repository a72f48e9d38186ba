// Stable LSD radix sort of (uint64 key, int32 value) pairs, 8-bit digits.
//
// Per pass: per-tile digit histograms (LDS atomics; counts are order-free),
// a device-wide exclusive scan of the digit-major histogram, and a stable
// scatter in which each wave ranks equal digits with 8 ballots (match mask)
// and the block combines waves and item slices in element order.
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;
constexpr int kItems = 16;
constexpr int kTile = kBS * kItems;
constexpr int kBins = 256;

__global__ void __launch_bounds__(kBS) k_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                              int32_t* __restrict__ hist, int nblk) {
  __shared__ int32_t h[kBins];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
  for (int j = 0; j < kItems; ++j) {
    int64_t e = base + j * kBS + threadIdx.x;
    if (e < n) atomicAdd(&h[(keys[e] >> shift) & 0xFF], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kBS) k_scatter(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                 uint64_t* __restrict__ kout, int32_t* __restrict__ vout,
                                                 int64_t n, int shift, const int32_t* __restrict__ offs,
                                                 int nblk) {
  __shared__ int32_t run[kBins];
  __shared__ int32_t cnt[kBS / 64][kBins];
  __shared__ int32_t base_off[kBins];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  run[tid] = 0;
  base_off[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
#pragma unroll
  for (int q = 0; q < kBS / 64; ++q) cnt[q][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int j = 0; j < kItems; ++j) {
    int64_t e = base + j * kBS + tid;
    bool valid = e < n;
    uint64_t key = valid ? kin[e] : 0;
    int32_t val = valid ? vin[e] : 0;
    int d = (int)((key >> shift) & 0xFF);
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1;
      uint64_t bb = __ballot(bit);
      mask &= bit ? bb : ~bb;
    }
    int wrank = __popcll(mask & lt);
    if (valid && wrank == 0) cnt[w][d] = __popcll(mask);
    __syncthreads();
    if (valid) {
      int r = run[d] + wrank;
      for (int q = 0; q < w; ++q) r += cnt[q][d];
      int64_t dst = (int64_t)base_off[d] + r;
      kout[dst] = key;
      vout[dst] = val;
    }
    __syncthreads();
    {
      int s = 0;
#pragma unroll
      for (int q = 0; q < kBS / 64; ++q) {
        s += cnt[q][tid];
        cnt[q][tid] = 0;
      }
      run[tid] += s;
    }
    __syncthreads();
  }
}

}  // namespace

void radix_sort(Ctx& c, uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt,
                int64_t n, int bits) {
  if (n <= 1) return;
  const int nblk = (int)((n + kTile - 1) / kTile);
  const int64_t nh = (int64_t)kBins * nblk;
  int32_t* hist = (int32_t*)ensure(c, c.hist, sizeof(int32_t) * (nh + 1));
  int passes = (bits + 7) / 8;
  if (passes & 1) ++passes;  // even count: result lands back in keys/vals
  uint64_t* ka = keys;
  int32_t* va = vals;
  uint64_t* kb = keys_alt;
  int32_t* vb = vals_alt;
  for (int p = 0; p < passes; ++p) {
    int shift = 8 * p;
    hipLaunchKernelGGL(k_hist, dim3(nblk), dim3(kBS), 0, c.stream, ka, n, shift, hist, nblk);
    AMFMM_HIP(hipGetLastError());
    scan_i32(c, hist, hist, nh);
    hipLaunchKernelGGL(k_scatter, dim3(nblk), dim3(kBS), 0, c.stream, ka, va, kb, vb, n, shift,
                       hist, nblk);
    AMFMM_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
  }
}

}  // namespace amfmm
