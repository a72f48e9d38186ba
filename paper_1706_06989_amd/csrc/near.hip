// Near field (direct summation between particles of non-accepted leaf pairs),
// fused with the evaluation of the far-field coefficients at each particle and
// the scatter back to caller order.
//
// One wave per target leaf.  Each lane holds four targets in registers
// (register blocking: one source load feeds four interactions) and a slice of
// the sources; lanes = (target group g, slice s), slices a power of two so
// that the partial sums of a group reduce with a fixed xor butterfly
// (deterministic).  Source leaves that follow each other in particle order
// are merged into one run; runs are read straight from the key-sorted double4
// particle array (consecutive lanes read consecutive particles).
#include "device_math.h"
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / 64;
constexpr int kTG = 4;    // targets per lane
constexpr int kCap = 384; // source particles per wave staged in LDS

// make this wave's LDS writes visible to its other lanes before they read
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int pow2floor(int v) { return 1 << (31 - __builtin_clz(v)); }

// interactions of this lane's kTG targets with sources buf[s], buf[s+nsl], ...
__device__ inline void near_tile(const double4* buf, int fill, int s, int nsl, const double* tx, const double* ty,
                                 const double* tz, double* fx, double* fy, double* fz, double* ph) {
  for (int j = s; j < fill; j += nsl) {
    const double4 q = buf[j];
#pragma unroll
    for (int u = 0; u < kTG; ++u) {
      const double dx = q.x - tx[u], dy = q.y - ty[u], dz = q.z - tz[u];
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      double y = rsqrt_f64_1nr(r2);
      y = r2 > 0.0 ? y : 0.0;
      const double my = q.w * y;
      const double my3 = my * (y * y);
      fx[u] = fma(my3, dx, fx[u]);
      fy[u] = fma(my3, dy, fy[u]);
      fz[u] = fma(my3, dz, fz[u]);
      ph[u] -= my;
    }
  }
}

// leaves == nullptr: the targets are the leaves among cells [c_lo, c_lo + nleaves)
__global__ void __launch_bounds__(kBS) k_near(int32_t nleaves, const int32_t* __restrict__ leaves, int32_t c_lo,
                                              const int32_t* __restrict__ nch,
                                              const int32_t* __restrict__ beg, const int32_t* __restrict__ cnt,
                                              const double4* __restrict__ pos, const double4* __restrict__ geo,
                                              const double* __restrict__ loc, const int64_t* __restrict__ nstart,
                                              const int32_t* __restrict__ ncount, const int32_t* __restrict__ nsrc,
                                              const int32_t* __restrict__ perm, double G, double* __restrict__ ax,
                                              double* __restrict__ ay, double* __restrict__ az, double* __restrict__ pot,
                                              unsigned long long* __restrict__ inter) {
  const int lane = threadIdx.x & 63;
  const int32_t li = uniform((int32_t)(blockIdx.x * kWaves + (threadIdx.x >> 6)));
  if (li >= nleaves) return;
  const int32_t X = uniform(leaves ? leaves[li] : c_lo + li);
  if (!leaves && uniform(nch[X]) != 0) return;
  const int32_t b = uniform(beg[X]), nt = uniform(cnt[X]);
  const int64_t st = nstart[X];
  const int32_t nsc = uniform(ncount[X]);
  const double4 gx = geo[X];
  const double* L = loc + (int64_t)X * kLoc;
  __shared__ double4 lds[kWaves][kCap];
  double4* buf = lds[threadIdx.x >> 6];
  int64_t nsrc_particles = 0;  // source particles of this leaf's list (lane 0)
  for (int32_t tb = b; tb < b + nt; tb += 64) {
    const int ntc = min(64, b + nt - tb);
    const int ng = (ntc + kTG - 1) / kTG;
    const int nsl = pow2floor(64 / ng);
    const int g = lane / nsl, s = lane % nsl;
    const bool active = g < ng;
    double tx[kTG], ty[kTG], tz[kTG];
    double fx[kTG], fy[kTG], fz[kTG], ph[kTG];
#pragma unroll
    for (int q = 0; q < kTG; ++q) {
      const int t = g * kTG + q;
      const double4 p = pos[tb + ((active && t < ntc) ? t : 0)];
      tx[q] = p.x;
      ty[q] = p.y;
      tz[q] = p.z;
      fx[q] = fy[q] = fz[q] = ph[q] = 0.0;
    }
    // The near list is consumed 64 entries at a time: every lane fetches one
    // source leaf (index, first particle, count) with independent loads, an
    // in-wave prefix sum places each leaf in this wave's LDS buffer, and
    // every lane copies its own leaf.  Leaves are taken while they fit.
    int32_t k = 0;
    while (k < nsc) {
      const int32_t kk = k + lane;
      const int32_t Yl = kk < nsc ? nsrc[st + kk] : -1;
      const int32_t bl = Yl >= 0 ? beg[Yl] : 0;
      const int32_t cl = Yl >= 0 ? cnt[Yl] : 0;
      int32_t inc = cl;  // inclusive prefix over lanes
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
      }
      const uint64_t fits = __ballot(Yl >= 0 && inc <= kCap);
      const int take = __popcll(fits);  // prefix is monotone: leading lanes fit
      int fill;
      if (take > 0) {
        if (lane < take)
          for (int32_t j = 0; j < cl; ++j) buf[inc - cl + j] = pos[bl + j];
        fill = __shfl(inc, take - 1, 64);
        if (tb == b) nsrc_particles += fill;
        k += take;
      } else {
        // a single leaf larger than the buffer (coincident points at the
        // deepest level): stream it in buffer-sized pieces
        const int32_t b0 = __shfl(bl, 0, 64), c0 = __shfl(cl, 0, 64);
        for (int32_t off = 0; off < c0; off += kCap) {
          const int part = min(kCap, c0 - off);
          for (int i = lane; i < part; i += 64) buf[i] = pos[b0 + off + i];
          wave_sync();
          if (active) near_tile(buf, part, s, nsl, tx, ty, tz, fx, fy, fz, ph);
          wave_sync();
        }
        if (tb == b) nsrc_particles += c0;
        k += 1;
        continue;
      }
      wave_sync();
      if (active) near_tile(buf, fill, s, nsl, tx, ty, tz, fx, fy, fz, ph);
      wave_sync();
    }
    // sum the slices of each group (fixed butterfly)
    for (int off = nsl >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int u = 0; u < kTG; ++u) {
        fx[u] += __shfl_xor(fx[u], off, 64);
        fy[u] += __shfl_xor(fy[u], off, 64);
        fz[u] += __shfl_xor(fz[u], off, 64);
        ph[u] += __shfl_xor(ph[u], off, 64);
      }
    }
    // lane s < 4 of group g finishes target g*4 + s
    const int t = g * kTG + s;
    if (active && s < kTG && t < ntc) {
      double px = tx[0], py = ty[0], pz = tz[0], sx = fx[0], sy = fy[0], sz = fz[0], sp = ph[0];
#pragma unroll
      for (int u = 1; u < kTG; ++u) {
        if (s == u) {
          px = tx[u];
          py = ty[u];
          pz = tz[u];
          sx = fx[u];
          sy = fy[u];
          sz = fz[u];
          sp = ph[u];
        }
      }
      const double x[3] = {px - gx.x, py - gx.y, pz - gx.z};
      double gl[3], phi;
      eval_local(L, x, gl, phi);
      const int32_t o = perm[tb + t];
      ax[o] = G * (sx + gl[0]);
      ay[o] = G * (sy + gl[1]);
      az[o] = G * (sz + gl[2]);
      if (pot) pot[o] = G * (sp + phi);
    }
  }
  if (lane == 0) atomicAdd(inter, (unsigned long long)((int64_t)nt * nsrc_particles - nt));
}

}  // namespace

void near_field(Ctx& c, const int32_t* leaves, int32_t c_lo, int32_t count, double* ax, double* ay, double* az,
                double* pot) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_near, dim3(blocks_for(count, kWaves)), dim3(kBS), 0, c.stream, count, leaves, c_lo,
                     as<int32_t>(c.c_nchild), as<int32_t>(c.c_begin), as<int32_t>(c.c_count), (const double4*)c.pos4.p,
                     (const double4*)c.geo.p, (const double*)c.loc.p, (const int64_t*)c.near_start.p,
                     (const int32_t*)c.near_count.p, (const int32_t*)c.near_src.p, as<int32_t>(c.perm), c.opt.G, ax,
                     ay, az, pot, (unsigned long long*)c.counters.p);
  AMFMM_HIP(hipGetLastError());
}

}  // namespace amfmm
