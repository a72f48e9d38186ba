// Upward pass (Sec. 2): mass M (eq. 1), centre of mass Z, quadrupole M_ij
// (eq. quad) and octupole M_ijk about Z, and R_max.
//
//  * leaves: one thread per leaf, sequential over its particles in key order;
//  * parents: one thread per cell per level, bottom-up, summing the children in
//    octant order (mass and first moment), then shifting the children's M_ij,
//    M_ijk to the parent's centre (exact for moments about a centre of mass);
//  * R_max: exact largest distance to Z over the cell's particles; every
//    particle visits its ancestors level by level, lanes holding the same
//    ancestor reduce within the wave first, and a wave carries the run at
//    the end of one 64-particle slab into the next before its atomic max.
//
// Compiled with -ffp-contract=off: the centres of mass and R_max must round
// exactly as written (they decide the walk, which is reproduced bit for bit).
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;

// packed mom layout: [0]=M, [1..6]=M_ij (xx xy xz yy yz zz), [7..16]=M_ijk
// (xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz), [17] pad
__device__ inline void add_about(double* M2, double* M3, double mu, double x, double y, double z) {
  // mu x_i x_j and mu x_i x_j x_k, multiplied left to right
  double mx = mu * x, my = mu * y, mz = mu * z;
  M2[0] += mx * x;
  M2[1] += mx * y;
  M2[2] += mx * z;
  M2[3] += my * y;
  M2[4] += my * z;
  M2[5] += mz * z;
  M3[0] += mx * x * x;
  M3[1] += mx * x * y;
  M3[2] += mx * x * z;
  M3[3] += mx * y * y;
  M3[4] += mx * y * z;
  M3[5] += mx * z * z;
  M3[6] += my * y * y;
  M3[7] += my * y * z;
  M3[8] += my * z * z;
  M3[9] += mz * z * z;
}

__global__ void __launch_bounds__(kBS) k_leaf_moments(const double4* __restrict__ pos, const int32_t* __restrict__ leaves,
                                                      int32_t nleaves, const int32_t* __restrict__ beg,
                                                      const int32_t* __restrict__ cnt, double4* __restrict__ geo,
                                                      double* __restrict__ mom, double4* __restrict__ msum) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nleaves) return;
  int32_t c = leaves[i];
  int32_t b = beg[c], e = b + cnt[c];
  double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
  for (int32_t p = b; p < e; ++p) {
    double4 q = pos[p];
    M += q.w;
    Sx += q.w * q.x;
    Sy += q.w * q.y;
    Sz += q.w * q.z;
  }
  double Zx = Sx / M, Zy = Sy / M, Zz = Sz / M;
  double M2[6] = {}, M3[10] = {};
  for (int32_t p = b; p < e; ++p) {
    double4 q = pos[p];
    add_about(M2, M3, q.w, q.x - Zx, q.y - Zy, q.z - Zz);
  }
  geo[c] = make_double4(Zx, Zy, Zz, 0.0);
  msum[c] = make_double4(Sx, Sy, Sz, M);
  double* o = mom + (int64_t)c * kMom;
  o[0] = M;
  for (int q = 0; q < 6; ++q) o[1 + q] = M2[q];
  for (int q = 0; q < 10; ++q) o[7 + q] = M3[q];
  o[17] = 0.0;
}

__global__ void __launch_bounds__(kBS) k_m2m(int32_t c0, int32_t nl, const int32_t* __restrict__ ch0,
                                             const int32_t* __restrict__ nch, double4* __restrict__ geo,
                                             double* __restrict__ mom, double4* __restrict__ msum) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  int32_t c = c0 + i;
  int32_t k = nch[c];
  if (k == 0) return;
  int32_t f = ch0[c];
  double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
  for (int32_t q = f; q < f + k; ++q) {
    double4 s = msum[q];
    M += s.w;
    Sx += s.x;
    Sy += s.y;
    Sz += s.z;
  }
  double Zx = Sx / M, Zy = Sy / M, Zz = Sz / M;
  double M2[6] = {}, M3[10] = {};
  for (int32_t q = f; q < f + k; ++q) {
    double4 g = geo[q];
    const double* cm = mom + (int64_t)q * kMom;
    double mc = cm[0];
    double d[3] = {g.x - Zx, g.y - Zy, g.z - Zz};
    const double* a = cm + 1;  // child M_ij
    const double* t = cm + 7;  // child M_ijk
    // M_ij += Mc_ij + Mc d_i d_j
    const int I2[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
    for (int u = 0; u < 6; ++u) M2[u] += a[u] + mc * d[I2[u][0]] * d[I2[u][1]];
    // M_ijk += Mc_ijk + Mc_ij d_k + Mc_jk d_i + Mc_ik d_j + Mc d_i d_j d_k
    const int I3[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                           {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
    auto p2 = [&](int x, int y) {
      int lo = x < y ? x : y, hi = x < y ? y : x;
      return a[lo == 0 ? hi : (lo == 1 ? 2 + hi : 5)];
    };
#pragma unroll
    for (int u = 0; u < 10; ++u) {
      int ii = I3[u][0], jj = I3[u][1], kk = I3[u][2];
      M3[u] += t[u] + p2(ii, jj) * d[kk] + p2(jj, kk) * d[ii] + p2(ii, kk) * d[jj] +
               mc * d[ii] * d[jj] * d[kk];
    }
  }
  geo[c] = make_double4(Zx, Zy, Zz, 0.0);
  msum[c] = make_double4(Sx, Sy, Sz, M);
  double* o = mom + (int64_t)c * kMom;
  o[0] = M;
  for (int q = 0; q < 6; ++q) o[1 + q] = M2[q];
  for (int q = 0; q < 10; ++q) o[7 + q] = M3[q];
  o[17] = 0.0;
}

__global__ void __launch_bounds__(kBS) k_leaf_of(const int32_t* __restrict__ leaves, int32_t nleaves,
                                                 const int32_t* __restrict__ beg, const int32_t* __restrict__ cnt,
                                                 int32_t* __restrict__ leafof) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nleaves) return;
  int32_t c = leaves[i];
  for (int32_t p = beg[c]; p < beg[c] + cnt[c]; ++p) leafof[p] = c;
}

__global__ void k_cell_level(const int32_t* __restrict__ level_start, int nlev, int32_t nc, int8_t* __restrict__ lev) {
  int32_t c = blockIdx.x * kBS + threadIdx.x;
  if (c >= nc) return;
  int l = 0;
  while (l + 1 < nlev && level_start[l + 1] <= c) ++l;
  lev[c] = (int8_t)l;
}

__global__ void __launch_bounds__(kBS) k_zero_u64(unsigned long long* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// 64-particle slabs one wave of k_rmax takes, in key order
constexpr int kRmaxSlabs = 32;

// R_max^2 of every ancestor of every particle, by atomic max on the bit
// pattern (order-preserving for non-negative doubles).  A wave takes
// kRmaxSlabs consecutive slabs of 64 particles; on each level, lanes with
// the same ancestor (contiguous, as cells are) reduce to the run's first
// lane, and the run that reaches the slab's end stays pending in the wave
// and joins the next slab's first run when that has the same cell.  A cell
// of many particles so gets one atomic per wave that touches it rather than
// one per slab (all waves otherwise meet on the same few top cells).
__global__ void __launch_bounds__(kBS) k_rmax(const double4* __restrict__ pos, int64_t n,
                                              const int32_t* __restrict__ leafof, const int32_t* __restrict__ par,
                                              const int8_t* __restrict__ lev, const double4* __restrict__ geo,
                                              unsigned long long* __restrict__ r2max) {
  const int lane = threadIdx.x & 63;
  const int64_t p0 = (((int64_t)blockIdx.x * kBS + threadIdx.x) >> 6) * (64 * kRmaxSlabs);
  // per level, the pending run (wave-uniform): its cell (-1: none) and max
  int32_t pend_id[kMaxLevel + 1];
  double pend_r2[kMaxLevel + 1];
#pragma unroll
  for (int l = 0; l <= kMaxLevel; ++l) {
    pend_id[l] = -1;
    pend_r2[l] = -1.0;
  }
  for (int s = 0; s < kRmaxSlabs; ++s) {
    const int64_t p = p0 + (int64_t)s * 64 + lane;
    if (p0 + (int64_t)s * 64 >= n) break;  // wave-uniform
    const bool valid = p < n;
    int32_t anc[kMaxLevel + 1];
    const double4 q = valid ? pos[p] : make_double4(0, 0, 0, 0);
    {
      int32_t a = valid ? leafof[p] : -1;
      int L = valid ? (int)lev[a] : -1;
#pragma unroll
      for (int l = kMaxLevel; l >= 0; --l) {
        if (l > L) {
          anc[l] = -1;
        } else {
          anc[l] = a;
          a = par[a];
        }
      }
    }
#pragma unroll
    for (int l = 0; l <= kMaxLevel; ++l) {
      const int32_t id = anc[l];
      // no particle of the slab below this level: deeper runs stay pending
      if (!__any(id >= 0)) break;
      double r2 = -1.0;
      if (id >= 0) {
        const double4 g = geo[id];
        const double dx = q.x - g.x, dy = q.y - g.y, dz = q.z - g.z;
        r2 = (dx * dx + dy * dy) + dz * dz;
      }
      // segmented max over contiguous lanes with the same ancestor
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_down(r2, off, 64);
        const int32_t oid = __shfl_down(id, off, 64);
        if (lane + off < 64 && oid == id && o > r2) r2 = o;
      }
      const int32_t prev = __shfl_up(id, 1, 64);
      const bool head = id >= 0 && (lane == 0 || prev != id);
      const unsigned long long hm = __ballot(head);  // nonzero: some lane has an ancestor here
      const int last = 63 - __clzll(hm);
      const bool joins = __shfl(id, 0, 64) == pend_id[l];
      if (lane == 0 && joins) r2 = fmax(r2, pend_r2[l]);
      if (lane == 0 && !joins && pend_id[l] >= 0)
        atomicMax(&r2max[pend_id[l]], (unsigned long long)__double_as_longlong(pend_r2[l]));
      if (head && lane != last) atomicMax(&r2max[id], (unsigned long long)__double_as_longlong(r2));
      pend_id[l] = __shfl(id, last, 64);
      pend_r2[l] = __shfl(r2, last, 64);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int l = 0; l <= kMaxLevel; ++l)
      if (pend_id[l] >= 0) atomicMax(&r2max[pend_id[l]], (unsigned long long)__double_as_longlong(pend_r2[l]));
  }
}

__global__ void __launch_bounds__(kBS) k_rmax_final(int32_t nc, const unsigned long long* __restrict__ r2max,
                                                    double4* __restrict__ geo) {
  int32_t c = blockIdx.x * kBS + threadIdx.x;
  if (c >= nc) return;
  geo[c].w = sqrt(__longlong_as_double((long long)r2max[c]));
}

}  // namespace

void upward_pass(Ctx& c) {
  const int32_t nc = c.ncells;
  double4* geo = (double4*)ensure(c, c.geo, sizeof(double4) * nc);
  double* mom = (double*)ensure(c, c.mom, sizeof(double) * kMom * (size_t)nc);
  double4* msum = (double4*)ensure(c, c.msum, sizeof(double4) * nc);
  const int32_t* beg = as<int32_t>(c.c_begin);
  const int32_t* cnt = as<int32_t>(c.c_count);
  hipLaunchKernelGGL(k_leaf_moments, dim3(blocks_for(c.nleaves, kBS)), dim3(kBS), 0, c.stream,
                     (const double4*)c.pos4.p, as<int32_t>(c.leaves), c.nleaves, beg, cnt, geo, mom, msum);
  AMFMM_HIP(hipGetLastError());
  for (int l = c.depth - 1; l >= 0; --l) {
    int32_t c0 = c.level_start[l], nl = c.level_start[l + 1] - c0;
    hipLaunchKernelGGL(k_m2m, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, c0, nl,
                       as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild), geo, mom, msum);
    AMFMM_HIP(hipGetLastError());
  }
  // R_max: scratch = leafof (int32 n) + level (int8 nc) + r2max (u64 nc) + level_start
  size_t nlev = c.level_start.size();
  size_t bytes = sizeof(int32_t) * c.n + sizeof(unsigned long long) * nc + nc + 64 + sizeof(int32_t) * nlev;
  char* s = (char*)ensure(c, c.scratch2, bytes);
  int32_t* leafof = (int32_t*)s;
  unsigned long long* r2 = (unsigned long long*)(s + ((sizeof(int32_t) * c.n + 7) & ~size_t(7)));
  int32_t* ls = (int32_t*)(r2 + nc);
  int8_t* lev = (int8_t*)(ls + nlev);
  AMFMM_HIP(hipMemcpyAsync(ls, c.level_start.data(), sizeof(int32_t) * nlev, hipMemcpyHostToDevice, c.stream));
  hipLaunchKernelGGL(k_cell_level, dim3(blocks_for(nc, kBS)), dim3(kBS), 0, c.stream, (const int32_t*)ls,
                     (int)nlev, nc, lev);
  hipLaunchKernelGGL(k_leaf_of, dim3(blocks_for(c.nleaves, kBS)), dim3(kBS), 0, c.stream,
                     as<int32_t>(c.leaves), c.nleaves, beg, cnt, leafof);
  hipLaunchKernelGGL(k_zero_u64, dim3(blocks_for(nc, kBS)), dim3(kBS), 0, c.stream, r2, (int64_t)nc);
  const int64_t rmax_waves = (c.n + 64 * kRmaxSlabs - 1) / (64 * kRmaxSlabs);
  hipLaunchKernelGGL(k_rmax, dim3(blocks_for(rmax_waves * 64, kBS)), dim3(kBS), 0, c.stream, (const double4*)c.pos4.p,
                     c.n, (const int32_t*)leafof, as<int32_t>(c.c_parent), (const int8_t*)lev,
                     (const double4*)geo, r2);
  hipLaunchKernelGGL(k_rmax_final, dim3(blocks_for(nc, kBS)), dim3(kBS), 0, c.stream, nc,
                     (const unsigned long long*)r2, geo);
  AMFMM_HIP(hipGetLastError());
  // keep the cell levels for the walk and the getters
  c.have_moments = true;
}

}  // namespace amfmm
