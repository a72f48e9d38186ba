// Octree build (Sec. 2): validation + bounding cube, Morton keys, stable sort,
// gather into sorted double4 particles, and cells level by level.
//
// Cells are numbered in (level, first particle) order: cells of one level are
// contiguous and sorted by their key prefix, children of a cell are
// contiguous and in octant order.  A cell splits into its non-empty octants
// iff it holds more than n_crit particles and sits above level 21.
//
// Compiled with -ffp-contract=off: the key arithmetic must round exactly as
// written so that keys (and hence the tree) are reproducible bit for bit.
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;
constexpr int kBBoxBlocks = 1024;

__device__ inline bool finite(double v) { return __builtin_isfinite(v); }

// per-block min of (x, y, z, -x, -y, -z) over the finite particles
__global__ void __launch_bounds__(kBS) k_bbox_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                      const double* __restrict__ z, const double* __restrict__ m,
                                                      int64_t n, double* __restrict__ part) {
  double v6[6] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
    double v[3] = {x[i], y[i], z[i]};
    if (!(finite(v[0]) && finite(v[1]) && finite(v[2]) && finite(m[i]))) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v6[d] = fmin(v6[d], v[d]);
      v6[3 + d] = fmin(v6[3 + d], -v[d]);
    }
  }
  __shared__ double s[6][kBS];
  for (int q = 0; q < 6; ++q) s[q][threadIdx.x] = v6[q];
  __syncthreads();
  for (int w = kBS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 6; ++q) s[q][threadIdx.x] = fmin(s[q][threadIdx.x], s[q][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) part[(int64_t)blockIdx.x * 8 + q] = s[q][0];
}

__global__ void __launch_bounds__(kBS) k_flags_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                       const double* __restrict__ z, const double* __restrict__ m,
                                                       int64_t n, int* __restrict__ flags) {
  int bv = 0, bm = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
    bool ok = finite(x[i]) && finite(y[i]) && finite(z[i]) && finite(m[i]);
    if (!ok) bv = 1;
    else if (!(m[i] > 0.0)) bm = 1;
  }
  if (__any(bv)) {
    if ((threadIdx.x & 63) == 0) atomicOr(&flags[0], 1);
  }
  if (__any(bm)) {
    if ((threadIdx.x & 63) == 0) atomicOr(&flags[1], 1);
  }
}

__global__ void __launch_bounds__(kBS) k_bbox_final(const double* __restrict__ part, int nb, double* __restrict__ box) {
  __shared__ double s[6][kBS];
  double v[6] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
  for (int b = threadIdx.x; b < nb; b += kBS)
    for (int q = 0; q < 6; ++q) v[q] = fmin(v[q], part[(int64_t)b * 8 + q]);
  for (int q = 0; q < 6; ++q) s[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = kBS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 6; ++q) s[q][threadIdx.x] = fmin(s[q][threadIdx.x], s[q][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) {
      box[d] = s[d][0];
      box[3 + d] = -s[3 + d][0];
    }
  }
}

__global__ void k_zero_int(int* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// spread the low 21 bits of v so that bit b lands on bit 3b
__device__ inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__global__ void __launch_bounds__(kBS) k_keys(const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, int64_t n, const double* __restrict__ box,
                                              uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (i >= n) return;
  const double lo[3] = {box[0], box[1], box[2]};
  double side = 0.0;
  for (int d = 0; d < 3; ++d) side = fmax(side, box[3 + d] - lo[d]);
  if (side == 0.0) side = 1.0;
  const double scale = (double)(1ull << kMaxLevel) / side;
  const uint64_t qmax = (1ull << kMaxLevel) - 1;
  const double v[3] = {x[i], y[i], z[i]};
  uint64_t q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double f = floor((v[d] - lo[d]) * scale);
    uint64_t qi = f <= 0.0 ? 0ull : (uint64_t)f;
    q[d] = qi > qmax ? qmax : qi;
  }
  keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  idx[i] = (int32_t)i;
}

__global__ void __launch_bounds__(kBS) k_gather(const double* __restrict__ x, const double* __restrict__ y,
                                                const double* __restrict__ z, const double* __restrict__ m,
                                                int64_t n, const int32_t* __restrict__ perm, double4* __restrict__ pos) {
  int64_t s = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (s >= n) return;
  int32_t i = perm[s];
  pos[s] = make_double4(x[i], y[i], z[i], m[i]);
}

__global__ void k_root(int32_t* beg, int32_t* cnt, int32_t* par, int32_t* ch0, int32_t* nch, int32_t n) {
  beg[0] = 0;
  cnt[0] = n;
  par[0] = -1;
  ch0[0] = -1;
  nch[0] = 0;
}

__device__ inline int32_t lower_bound_key(const uint64_t* __restrict__ keys, int32_t b, int32_t e, uint64_t v) {
  while (b < e) {
    int32_t mid = b + ((e - b) >> 1);
    if (keys[mid] < v) b = mid + 1;
    else e = mid;
  }
  return b;
}

// octant boundaries of the cell [b, b+cnt) at level lev: bounds[0..8]
__device__ inline void octant_bounds(const uint64_t* __restrict__ keys, int32_t b, int32_t cnt, int lev,
                                     int32_t bounds[9]) {
  const int shift = 3 * (kMaxLevel - lev);
  const int cshift = shift - 3;
  const uint64_t prefix = keys[b] >> shift;
  bounds[0] = b;
  bounds[8] = b + cnt;
#pragma unroll
  for (int o = 1; o < 8; ++o) bounds[o] = lower_bound_key(keys, bounds[o - 1], b + cnt, ((prefix << 3) | (uint64_t)o) << cshift);
}

__global__ void __launch_bounds__(kBS) k_split_count(const uint64_t* __restrict__ keys, const int32_t* __restrict__ beg,
                                                     const int32_t* __restrict__ cnt, int32_t c0, int32_t nl, int lev,
                                                     int n_crit, int32_t* __restrict__ nch_out) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  int32_t c = c0 + i;
  int32_t k = 0;
  if (cnt[c] > n_crit && lev < kMaxLevel) {
    int32_t bd[9];
    octant_bounds(keys, beg[c], cnt[c], lev, bd);
#pragma unroll
    for (int o = 0; o < 8; ++o) k += bd[o + 1] > bd[o];
  }
  nch_out[i] = k;
}

__global__ void __launch_bounds__(kBS) k_split_emit(const uint64_t* __restrict__ keys, int32_t* beg, int32_t* cnt,
                                                    int32_t* par, int32_t* ch0, int32_t* nch, int32_t c0, int32_t nl,
                                                    int lev, const int32_t* __restrict__ nchild,
                                                    const int32_t* __restrict__ off, int32_t next0) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  int32_t c = c0 + i;
  int32_t k = nchild[i];
  if (k == 0) return;
  int32_t bd[9];
  octant_bounds(keys, beg[c], cnt[c], lev, bd);
  int32_t first = next0 + off[i];
  int32_t q = first;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    if (bd[o + 1] > bd[o]) {
      beg[q] = bd[o];
      cnt[q] = bd[o + 1] - bd[o];
      par[q] = c;
      ch0[q] = -1;
      nch[q] = 0;
      ++q;
    }
  }
  ch0[c] = first;
  nch[c] = k;
}

__global__ void __launch_bounds__(kBS) k_leaf_flags(const int32_t* __restrict__ nch, int32_t nc, int32_t* __restrict__ f) {
  int32_t c = blockIdx.x * kBS + threadIdx.x;
  if (c < nc) f[c] = nch[c] == 0;
}

__global__ void __launch_bounds__(kBS) k_leaf_compact(const int32_t* __restrict__ nch, int32_t nc,
                                                      const int32_t* __restrict__ off, int32_t* __restrict__ leaves) {
  int32_t c = blockIdx.x * kBS + threadIdx.x;
  if (c < nc && nch[c] == 0) leaves[off[c]] = c;
}

}  // namespace

int bbox_validate(Ctx& c, const double* x, const double* y, const double* z, const double* m,
                  int64_t n) {
  int nb = (int)std::min<int64_t>(kBBoxBlocks, (n + kBS - 1) / kBS);
  double* part = (double*)ensure(c, c.scratch2, sizeof(double) * 8 * (size_t)nb + 64);
  double* box = (double*)ensure(c, c.bbox, sizeof(double) * 8);
  int* flags = (int*)(part + 8 * (size_t)nb);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, c.stream, flags, 2);
  hipLaunchKernelGGL(k_flags_partial, dim3(nb), dim3(kBS), 0, c.stream, x, y, z, m, n, flags);
  hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kBS), 0, c.stream, x, y, z, m, n, part);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBS), 0, c.stream, part, nb, box);
  AMFMM_HIP(hipGetLastError());
  int hf[2];
  AMFMM_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
  if (hf[0]) return AMFMM_E_NONFINITE;
  if (hf[1]) return AMFMM_E_INVALID;
  return AMFMM_OK;
}

void build_keys_sort(Ctx& c, const double* x, const double* y, const double* z, const double* m,
                     int64_t n) {
  uint64_t* keys = (uint64_t*)ensure(c, c.keys, sizeof(uint64_t) * n);
  int32_t* perm = (int32_t*)ensure(c, c.perm, sizeof(int32_t) * n);
  uint64_t* k2 = (uint64_t*)ensure(c, c.keys2, sizeof(uint64_t) * n);
  int32_t* p2 = (int32_t*)ensure(c, c.perm2, sizeof(int32_t) * n);
  double4* pos = (double4*)ensure(c, c.pos4, sizeof(double4) * n);
  hipLaunchKernelGGL(k_keys, dim3(blocks_for(n, kBS)), dim3(kBS), 0, c.stream, x, y, z, n,
                     (const double*)c.bbox.p, keys, perm);
  AMFMM_HIP(hipGetLastError());
  radix_sort(c, keys, perm, k2, p2, n, 3 * kMaxLevel);
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, kBS)), dim3(kBS), 0, c.stream, x, y, z, m, n,
                     perm, pos);
  AMFMM_HIP(hipGetLastError());
  c.n = n;
}

void build_levels(Ctx& c) {
  const int32_t n = (int32_t)c.n;
  int64_t cap = std::max<int64_t>(1024, c.n / 4);
  auto grow = [&](int64_t need, int64_t have_cells) {
    if (need <= cap && c.c_begin.cap >= sizeof(int32_t) * (size_t)need) return;
    while (cap < need) cap *= 2;
    size_t keep = sizeof(int32_t) * (size_t)have_cells;
    ensure_keep(c, c.c_begin, sizeof(int32_t) * cap, keep);
    ensure_keep(c, c.c_count, sizeof(int32_t) * cap, keep);
    ensure_keep(c, c.c_parent, sizeof(int32_t) * cap, keep);
    ensure_keep(c, c.c_child0, sizeof(int32_t) * cap, keep);
    ensure_keep(c, c.c_nchild, sizeof(int32_t) * cap, keep);
  };
  grow(cap, 0);
  hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, c.stream, as<int32_t>(c.c_begin), as<int32_t>(c.c_count),
                     as<int32_t>(c.c_parent), as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild), n);
  AMFMM_HIP(hipGetLastError());
  c.level_start.assign({0, 1});
  int32_t ncells = 1;
  const uint64_t* keys = as<uint64_t>(c.keys);
  for (int lev = 0;; ++lev) {
    int32_t c0 = c.level_start[lev], nl = c.level_start[lev + 1] - c0;
    int32_t* nchbuf = (int32_t*)ensure(c, c.fcnt, sizeof(int32_t) * (2 * (size_t)nl + 2));
    int32_t* off = nchbuf + nl + 1;
    hipLaunchKernelGGL(k_split_count, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, keys,
                       as<int32_t>(c.c_begin), as<int32_t>(c.c_count), c0, nl, lev, c.opt.n_crit, nchbuf);
    AMFMM_HIP(hipGetLastError());
    scan_i32(c, nchbuf, off, nl);
    int32_t total = 0;
    AMFMM_HIP(hipMemcpyAsync(&total, off + nl, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    AMFMM_HIP(hipStreamSynchronize(c.stream));
    if (total == 0) break;
    grow((int64_t)ncells + total, ncells);
    hipLaunchKernelGGL(k_split_emit, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, keys,
                       as<int32_t>(c.c_begin), as<int32_t>(c.c_count), as<int32_t>(c.c_parent),
                       as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild), c0, nl, lev,
                       (const int32_t*)nchbuf, (const int32_t*)off, ncells);
    AMFMM_HIP(hipGetLastError());
    ncells += total;
    c.level_start.push_back(ncells);
  }
  c.ncells = ncells;
  c.depth = (int32_t)c.level_start.size() - 2;
  // leaf list
  int32_t* f = (int32_t*)ensure(c, c.fcnt, sizeof(int32_t) * (2 * (size_t)ncells + 2));
  int32_t* off = f + ncells + 1;
  hipLaunchKernelGGL(k_leaf_flags, dim3(blocks_for(ncells, kBS)), dim3(kBS), 0, c.stream,
                     as<int32_t>(c.c_nchild), ncells, f);
  AMFMM_HIP(hipGetLastError());
  scan_i32(c, f, off, ncells);
  int32_t nleaves = 0;
  AMFMM_HIP(hipMemcpyAsync(&nleaves, off + ncells, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
  int32_t* leaves = (int32_t*)ensure(c, c.leaves, sizeof(int32_t) * (size_t)nleaves);
  hipLaunchKernelGGL(k_leaf_compact, dim3(blocks_for(ncells, kBS)), dim3(kBS), 0, c.stream,
                     as<int32_t>(c.c_nchild), ncells, (const int32_t*)off, leaves);
  AMFMM_HIP(hipGetLastError());
  c.nleaves = nleaves;
}

}  // namespace amfmm
