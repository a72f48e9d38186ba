// Near field (direct summation between particles of non-accepted leaf pairs),
// fused with the evaluation of the far-field coefficients at each particle and
// the scatter back to caller order.
//
// One wave per target leaf.  Each lane holds K targets in registers
// (register blocking: one source load feeds K interactions) and a slice of
// the sources; lanes = (target group g, slice s), 64 / groups slices per group
// (any count: the partial sums of a group reduce over a fixed tree into its
// first lane, deterministic).  K is 1, 2 or 4, chosen per leaf to waste the
// fewest lanes (leaves hold a few particles: 7 on average at n_crit = 25).
// The leaf's source entries are staged in LDS a bufferful at a time,
// consecutive lanes copying consecutive particles.
//
// Mixed precision: targets and staged sources are FP32 offsets from the
// target leaf's centre of mass (each difference taken in FP64, then rounded),
// the pair terms are FP32 (hardware reciprocal square root), and each lane's
// FP32 sums run over at most kFlush sources before they are flushed into a
// compensated FP64 sum per target and component: an FP64 accumulator plus the
// rounding error of every addition to it (TwoSum, Knuth), collected in an
// FP32 compensation term (the errors are below 2^-53 of the sum, so FP32
// holds them to far below FP64 resolution).  The slices of a target are
// reduced the same way; the compensation is added back once, before L2P.
// L2P and the output stay FP64.
#include "device_math.h"
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / 64;
constexpr int kTGMax = 4; // targets per lane: 1, 2 or 4
constexpr int kCap = 320; // source particles per wave staged in LDS (4 workgroups per CU)

// make this wave's LDS writes visible to its other lanes before they read
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int pow2floor(int v) { return 1 << (31 - __builtin_clz(v)); }

constexpr int kFlush = 32;  // FP32 terms per lane and target before an FP64 flush

// s + b = s' + e exactly (TwoSum: six operations, no condition on the
// magnitudes; the library is built without contraction, so no step fuses);
// s <- s', the rounding error e goes to the compensation term c
__device__ inline void comp_add(double& s, float& c, double b) {
  const double t = s + b;
  const double bp = t - s;
  const double e = (s - (t - bp)) + (b - bp);
  s = t;
  c += (float)e;
}

// FP32 interactions of this lane's targets (offsets t*) with sources
// buf[s], buf[s+nsl], ...; partial sums flushed into the compensated FP64
// sums (f*, compensation terms c*).  SOFT: the softened kernel, 1/(r^2 +
// eps2)^{1/2} and ^{3/2} (Sec. 4); pairs at r = 0 are skipped either way.
template <int kTG, bool SOFT>
__device__ inline void near_tile_f32(const float4* buf, int fill, int s, int nsl, const float* tx, const float* ty,
                                     const float* tz, double* fx, double* fy, double* fz, double* ph, float* cx,
                                     float* cy, float* cz, float* cp, float eps2) {
  for (int j0 = s; j0 < fill; j0 += kFlush * nsl) {
    const int j1 = min(fill, j0 + kFlush * nsl);
    float gx[kTG], gy[kTG], gz[kTG], gp[kTG];
#pragma unroll
    for (int u = 0; u < kTG; ++u) gx[u] = gy[u] = gz[u] = gp[u] = 0.0f;
    for (int j = j0; j < j1; j += nsl) {
      const float4 q = buf[j];
#pragma unroll
      for (int u = 0; u < kTG; ++u) {
        const float dx = q.x - tx[u], dy = q.y - ty[u], dz = q.z - tz[u];
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        float y = __builtin_amdgcn_rsqf(SOFT ? r2 + eps2 : r2);
        y = r2 > 0.0f ? y : 0.0f;
        const float my = q.w * y;
        const float my3 = my * (y * y);
        gx[u] = fmaf(my3, dx, gx[u]);
        gy[u] = fmaf(my3, dy, gy[u]);
        gz[u] = fmaf(my3, dz, gz[u]);
        gp[u] -= my;
      }
    }
#pragma unroll
    for (int u = 0; u < kTG; ++u) {
      comp_add(fx[u], cx[u], (double)gx[u]);
      comp_add(fy[u], cy[u], (double)gy[u]);
      comp_add(fz[u], cz[u], (double)gz[u]);
      comp_add(ph[u], cp[u], (double)gp[u]);
    }
  }
}

// interactions of this lane's kTG targets with sources buf[s], buf[s+nsl], ...
template <int kTG, bool SOFT>
__device__ inline void near_tile(const double4* buf, int fill, int s, int nsl, const double* tx, const double* ty,
                                 const double* tz, double* fx, double* fy, double* fz, double* ph, double eps2) {
  for (int j = s; j < fill; j += nsl) {
    const double4 q = buf[j];
#pragma unroll
    for (int u = 0; u < kTG; ++u) {
      const double dx = q.x - tx[u], dy = q.y - ty[u], dz = q.z - tz[u];
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      double y = rsqrt_f64_1nr(SOFT ? r2 + eps2 : r2);
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

// FP32 offset of a particle from a centre (difference in FP64, then rounded)
__device__ inline float4 offset32(const double4 p, const double4 c) {
  return make_float4((float)(p.x - c.x), (float)(p.y - c.y), (float)(p.z - c.z), (float)p.w);
}

// Targets per lane (1, 2 or 4) for a block of ntc <= 64 targets: the fewest
// lane steps, a step over one source costing about 19 operations per target
// and 3 of its own (ties: more targets per lane).
__device__ inline int targets_per_lane(int ntc) {
  int best = kTGMax, bnsl = 64 / ((ntc + kTGMax - 1) / kTGMax);
  for (int k = 2; k >= 1; k >>= 1) {
    const int nsl = 64 / ((ntc + k - 1) / k);
    if ((19 * k + 3) * bnsl < (19 * best + 3) * nsl) {
      best = k;
      bnsl = nsl;
    }
  }
  return best;
}

// One block of ntc <= 64 targets starting at tb, kTG per lane, against the
// leaf's whole near list; returns the source particles of the list.
template <int kTG, bool MIXED, bool SOFT>
__device__ __forceinline__ int64_t near_block(int lane, int32_t tb, int ntc, int64_t st, int32_t nsc, const double4 gx,
                                     const double* L, double4* buf, const int32_t* __restrict__ nsrc,
                                     const int32_t* __restrict__ beg, const int32_t* __restrict__ cnt,
                                     const double4* __restrict__ pos, const int32_t* __restrict__ perm, double G,
                                     double* __restrict__ ax, double* __restrict__ ay, double* __restrict__ az,
                                     double* __restrict__ pot, double eps2) {
  float4* buf32 = reinterpret_cast<float4*>(buf);
  constexpr int cap = MIXED ? 2 * kCap : kCap;
  int64_t nsp = 0;
  const int ng = (ntc + kTG - 1) / kTG;
  const int nsl = 64 / ng;  // slices per group: as many lanes as the groups leave
  const int g = lane / nsl, s = lane % nsl;
  const bool active = g < ng;
  double tx[kTG], ty[kTG], tz[kTG];
  float ux[kTG], uy[kTG], uz[kTG];  // mixed: FP32 offsets from the leaf centre
  double fx[kTG], fy[kTG], fz[kTG], ph[kTG];
  float cx[kTG], cy[kTG], cz[kTG], cp[kTG];  // mixed: compensation terms
#pragma unroll
  for (int q = 0; q < kTG; ++q) {
    cx[q] = cy[q] = cz[q] = cp[q] = 0.0f;
    const int t = g * kTG + q;
    const double4 p = pos[tb + ((active && t < ntc) ? t : 0)];
    tx[q] = p.x;
    ty[q] = p.y;
    tz[q] = p.z;
    ux[q] = (float)(p.x - gx.x);
    uy[q] = (float)(p.y - gx.y);
    uz[q] = (float)(p.z - gx.z);
    fx[q] = fy[q] = fz[q] = ph[q] = 0.0;
  }
  // The near list is consumed 64 entries at a time: every lane fetches one
  // source leaf (index, first particle, count), an in-wave prefix sum places
  // each leaf in this wave's LDS buffer, and the wave copies them.  Leaves are
  // taken while they fit.  The next round's entries are fetched while this
  // round copies and computes.
  int32_t k = 0;
  int32_t Yl = lane < nsc ? nsrc[st + lane] : -1;
  int32_t bl = Yl >= 0 ? beg[Yl] : 0;
  int32_t cl = Yl >= 0 ? cnt[Yl] : 0;
  while (k < nsc) {
    const int32_t inc = wave_incl_scan(cl);  // inclusive prefix over lanes
    const uint64_t fits = __ballot(Yl >= 0 && inc <= cap);
    const int take = __popcll(fits);  // prefix is monotone: leading lanes fit
    const int adv = take > 0 ? take : 1;
    const int32_t kn = k + adv + lane;
    const int32_t Yn = kn < nsc ? nsrc[st + kn] : -1;
    int fill = 0;
    if (take > 0) {
      fill = __shfl(inc, take - 1, 64);
      // Cooperative copy: buffer slot v belongs to the entry e with
      // end[e-1] <= v < end[e] (binary search over the lanes' prefix ends),
      // so consecutive lanes copy consecutive particles of an entry; two
      // slots per lane and iteration, both loads in flight together.
      const int32_t endx = lane < take ? inc : INT32_MAX;
      const int32_t startx = inc - cl;
      for (int32_t v0 = 0; v0 < fill; v0 += 128) {
        const int32_t va = v0 + lane, vb = va + 64;
        int ea = 0, eb = 0;
#pragma unroll
        for (int sp = 32; sp >= 1; sp >>= 1) {
          if (__shfl(endx, ea + sp - 1, 64) <= va) ea += sp;
          if (__shfl(endx, eb + sp - 1, 64) <= vb) eb += sp;
        }
        const int32_t sa = __shfl(startx, ea, 64), ba = __shfl(bl, ea, 64);
        const int32_t sb = __shfl(startx, eb, 64), bb = __shfl(bl, eb, 64);
        double4 pa = make_double4(0.0, 0.0, 0.0, 0.0), pb = pa;
        if (va < fill) pa = pos[ba + va - sa];
        if (vb < fill) pb = pos[bb + vb - sb];
        if (va < fill) {
          if (MIXED) buf32[va] = offset32(pa, gx);
          else buf[va] = pa;
        }
        if (vb < fill) {
          if (MIXED) buf32[vb] = offset32(pb, gx);
          else buf[vb] = pb;
        }
      }
      nsp += fill;
    } else {
      // a single leaf larger than the buffer (coincident points at the
      // deepest level): stream it in buffer-sized pieces
      const int32_t b0 = __shfl(bl, 0, 64), c0 = __shfl(cl, 0, 64);
      for (int32_t off = 0; off < c0; off += cap) {
        const int part = min(cap, c0 - off);
        if (MIXED) {
          for (int i = lane; i < part; i += 64) buf32[i] = offset32(pos[b0 + off + i], gx);
        } else {
          for (int i = lane; i < part; i += 64) buf[i] = pos[b0 + off + i];
        }
        wave_sync();
        if (active) {
          if (MIXED) near_tile_f32<kTG, SOFT>(buf32, part, s, nsl, ux, uy, uz, fx, fy, fz, ph, cx, cy, cz, cp, (float)eps2);
          else near_tile<kTG, SOFT>(buf, part, s, nsl, tx, ty, tz, fx, fy, fz, ph, eps2);
        }
        wave_sync();
      }
      nsp += c0;
    }
    // the next round's extents load while this round computes
    const int32_t bn = Yn >= 0 ? beg[Yn] : 0;
    const int32_t cn = Yn >= 0 ? cnt[Yn] : 0;
    if (take > 0) {
      wave_sync();
      if (active) {
        if (MIXED) near_tile_f32<kTG, SOFT>(buf32, fill, s, nsl, ux, uy, uz, fx, fy, fz, ph, cx, cy, cz, cp, (float)eps2);
        else near_tile<kTG, SOFT>(buf, fill, s, nsl, tx, ty, tz, fx, fy, fz, ph, eps2);
      }
      wave_sync();
    }
    Yl = Yn;
    bl = bn;
    cl = cn;
    k += adv;
  }
  // sum the slices of each group into its first lane (a fixed tree: at
  // step off, slice s adds slice s + off of its own group)
  for (int off = nsl > 1 ? pow2floor(nsl - 1) : 0; off > 0; off >>= 1) {
    const bool take = s + off < nsl;
#pragma unroll
    for (int u = 0; u < kTG; ++u) {
      const double vx = __shfl(fx[u], lane + off, 64), vy = __shfl(fy[u], lane + off, 64);
      const double vz = __shfl(fz[u], lane + off, 64), vp = __shfl(ph[u], lane + off, 64);
      if (MIXED) {
        const float wx = __shfl(cx[u], lane + off, 64), wy = __shfl(cy[u], lane + off, 64);
        const float wz = __shfl(cz[u], lane + off, 64), wp = __shfl(cp[u], lane + off, 64);
        if (take) {
          comp_add(fx[u], cx[u], vx);
          comp_add(fy[u], cy[u], vy);
          comp_add(fz[u], cz[u], vz);
          comp_add(ph[u], cp[u], vp);
          cx[u] += wx;
          cy[u] += wy;
          cz[u] += wz;
          cp[u] += wp;
        }
      } else if (take) {
        fx[u] += vx;
        fy[u] += vy;
        fz[u] += vz;
        ph[u] += vp;
      }
    }
  }
  if (MIXED) {
    // the compensated sums, rounded once to FP64
#pragma unroll
    for (int u = 0; u < kTG; ++u) {
      fx[u] += (double)cx[u];
      fy[u] += (double)cy[u];
      fz[u] += (double)cz[u];
      ph[u] += (double)cp[u];
    }
  }
  // lane s < 4 of group g finishes target g*4 + s with the sums of the
  // group's first lane
  const int t = g * kTG + s;
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
#pragma unroll
  for (int u = 0; u < kTG; ++u) {
    const double vx = __shfl(fx[u], g * nsl, 64), vy = __shfl(fy[u], g * nsl, 64);
    const double vz = __shfl(fz[u], g * nsl, 64), vp = __shfl(ph[u], g * nsl, 64);
    if (s == u) {
      sx = vx;
      sy = vy;
      sz = vz;
      sp = vp;
    }
  }
  if (active && s < kTG && t < ntc) {
    const double4 pt = pos[tb + t];  // reloaded: the mixed path keeps no FP64 copy
    const double x[3] = {pt.x - gx.x, pt.y - gx.y, pt.z - gx.z};
    double gl[3], phi;
    eval_local(L, x, gl, phi);
    const int32_t o = perm[tb + t];
    ax[o] = G * (sx + gl[0]);
    ay[o] = G * (sy + gl[1]);
    az[o] = G * (sz + gl[2]);
    if (pot) pot[o] = G * (sp + phi);
  }
  return nsp;
}

// leaves == nullptr: the targets are the leaves among cells [c_lo, c_lo + nleaves)
template <bool MIXED, bool SOFT>
__global__ void __launch_bounds__(kBS) __attribute__((amdgpu_waves_per_eu(4))) k_near(int32_t nleaves, const int32_t* __restrict__ leaves, int32_t c_lo,
                                              const int32_t* __restrict__ nch,
                                              const int32_t* __restrict__ beg, const int32_t* __restrict__ cnt,
                                              const double4* __restrict__ pos, const double4* __restrict__ geo,
                                              const double* __restrict__ loc, const int64_t* __restrict__ nstart,
                                              const int32_t* __restrict__ ncount, const int32_t* __restrict__ nsrc,
                                              const int32_t* __restrict__ perm, double G, double* __restrict__ ax,
                                              double* __restrict__ ay, double* __restrict__ az, double* __restrict__ pot,
                                              unsigned long long* __restrict__ inter, double eps2) {
  const int lane = threadIdx.x & 63;
  const int32_t li = uniform((int32_t)(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6)));
  if (li >= nleaves) return;
  const int32_t X = uniform(leaves ? leaves[li] : c_lo + li);
  if (!leaves && uniform(nch[X]) != 0) return;
  const int32_t b = uniform(beg[X]), nt = uniform(cnt[X]);
  const int64_t st = nstart[X];
  const int32_t nsc = uniform(ncount[X]);
  const double4 gx = geo[X];
  const double* L = loc + (int64_t)X * kLoc;
  // FP64 staging holds kCap double4 per wave; the mixed path puts 2 kCap
  // float4 offsets in the same bytes
  __shared__ double4 lds[kWaves][kCap];
  double4* buf = lds[threadIdx.x >> 6];
  int64_t nsrc_particles = 0;  // source particles of this leaf's list (lane 0)
  for (int32_t tb = b; tb < b + nt; tb += 64) {
    const int ntc = min(64, b + nt - tb);
    const int K = targets_per_lane(ntc);
    int64_t nsp;
    if (K == 1)
      nsp = near_block<1, MIXED, SOFT>(lane, tb, ntc, st, nsc, gx, L, buf, nsrc, beg, cnt, pos, perm, G, ax, ay, az,
                                       pot, eps2);
    else if (K == 2)
      nsp = near_block<2, MIXED, SOFT>(lane, tb, ntc, st, nsc, gx, L, buf, nsrc, beg, cnt, pos, perm, G, ax, ay, az,
                                       pot, eps2);
    else
      nsp = near_block<kTGMax, MIXED, SOFT>(lane, tb, ntc, st, nsc, gx, L, buf, nsrc, beg, cnt, pos, perm, G, ax, ay,
                                            az, pot, eps2);
    if (tb == b) nsrc_particles = nsp;
  }
  if (lane == 0) atomicAdd(inter, (unsigned long long)((int64_t)nt * nsrc_particles - nt));
}

}  // namespace

void near_field(Ctx& c, const int32_t* leaves, int32_t c_lo, int32_t count, double* ax, double* ay, double* az,
                double* pot) {
  if (count <= 0) return;
  ++c.near_launches;
  const bool mixed = c.opt.precision == AMFMM_MIXED, soft = c.opt.softening > 0.0;
  auto kern = mixed ? (soft ? k_near<true, true> : k_near<true, false>)
                    : (soft ? k_near<false, true> : k_near<false, false>);
  hipLaunchKernelGGL(kern, dim3(blocks_for(count, kWaves)), dim3(kBS), 0, c.stream, count, leaves, c_lo,
                     as<int32_t>(c.c_nchild), as<int32_t>(c.c_begin), as<int32_t>(c.c_count), (const double4*)c.pos4.p,
                     (const double4*)c.geo.p, (const double*)c.loc.p, (const int64_t*)c.near_start.p,
                     (const int32_t*)c.near_count.p, (const int32_t*)c.near_src.p, as<int32_t>(c.perm), c.opt.G, ax,
                     ay, az, pot, (unsigned long long*)c.counters.p, c.opt.softening * c.opt.softening);
  AMFMM_HIP(hipGetLastError());
  if (c.opt.order != 3) order_l2p(c, leaves, c_lo, count, ax, ay, az, pot);
}

}  // namespace amfmm
