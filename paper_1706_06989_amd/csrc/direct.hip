// Direct summation (the exact g_PP of Sec. 3) at a set of targets, and the
// net force / torque balance metric of Sec. 3 with compensated sums.
#include "device_math.h"
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;


// one thread per target and source chunk, sources staged through LDS in index
// order; partial sums per chunk are added in chunk order by k_direct_sum
__global__ void __launch_bounds__(kBS) k_direct(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                                const double* __restrict__ z, const double* __restrict__ m,
                                                int64_t nt, const int64_t* __restrict__ tg, int64_t chunk,
                                                double* __restrict__ part, double eps2) {
  __shared__ double4 tile[kBS];
  const int64_t q = (int64_t)blockIdx.x * kBS + threadIdx.x;
  int64_t i = q < nt ? (tg ? tg[q] : q) : 0;
  if (i < 0 || i >= n) i = 0;  // out-of-range targets are flagged by k_direct_sum
  const double xi = x[i], yi = y[i], zi = z[i];
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0, sa = 0.0;
  const int64_t j0 = (int64_t)blockIdx.y * chunk, j1 = min(n, j0 + chunk);
  for (int64_t t0 = j0; t0 < j1; t0 += kBS) {
    const int64_t j = t0 + threadIdx.x;
    tile[threadIdx.x] = j < j1 ? make_double4(x[j], y[j], z[j], m[j]) : make_double4(0, 0, 0, 0);
    __syncthreads();
    const int lim = (int)min<int64_t>(kBS, j1 - t0);
    for (int k = 0; k < lim; ++k) {
      const double4 s = tile[k];
      const double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      double w = rsqrt_f64(r2 + eps2);  // softened for eps2 > 0 (Sec. 4)
      w = r2 > 0.0 ? w : 0.0;
      const double mw = s.w * w;
      const double mw3 = mw * w * w;
      sx = fma(mw3, dx, sx);
      sy = fma(mw3, dy, sy);
      sz = fma(mw3, dz, sz);
      sp -= mw;
      sa = fma(mw, w, sa);
    }
    __syncthreads();
  }
  if (q < nt) {
    double* o = part + ((int64_t)blockIdx.y * nt + q) * 5;
    o[0] = sx;
    o[1] = sy;
    o[2] = sz;
    o[3] = sp;
    o[4] = sa;
  }
}

__global__ void __launch_bounds__(kBS) k_direct_sum(int64_t n, int64_t nt, const int64_t* __restrict__ tg, int nchunk,
                                                    const double* __restrict__ part, double G, double* __restrict__ ax,
                                                    double* __restrict__ ay, double* __restrict__ az,
                                                    double* __restrict__ pot, double* __restrict__ gabs) {
  const int64_t q = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (q >= nt) return;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < nchunk; ++c)
    for (int k = 0; k < 5; ++k) s[k] += part[((int64_t)c * nt + q) * 5 + k];
  const int64_t i = tg ? tg[q] : q;
  if (i < 0 || i >= n)
    for (int k = 0; k < 5; ++k) s[k] = __builtin_nan("");
  ax[q] = G * s[0];
  ay[q] = G * s[1];
  az[q] = G * s[2];
  if (pot) pot[q] = G * s[3];
  if (gabs) gabs[q] = G * s[4];
}

struct KS {  // compensated running sum (Neumaier)
  double s = 0.0, c = 0.0;
  __device__ void add(double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  __device__ void add(const KS& o) {
    add(o.s);
    c += o.c;
  }
};

constexpr int kNSum = 12;

__global__ void __launch_bounds__(kBS) k_balance_partial(int64_t n, const double* __restrict__ x,
                                                         const double* __restrict__ y, const double* __restrict__ z,
                                                         const double* __restrict__ m, const double* __restrict__ gx,
                                                         const double* __restrict__ gy, const double* __restrict__ gz,
                                                         double* __restrict__ part) {
  KS acc[kNSum];
  for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
    const double g[3] = {gx[i], gy[i], gz[i]};
    const double X[3] = {x[i], y[i], z[i]};
    const double t[3] = {X[1] * g[2] - X[2] * g[1], X[2] * g[0] - X[0] * g[2], X[0] * g[1] - X[1] * g[0]};
    const double mi = m[i];
    for (int d = 0; d < 3; ++d) {
      acc[d].add(mi * g[d]);
      acc[3 + d].add(mi * fabs(g[d]));
      acc[6 + d].add(mi * t[d]);
      acc[9 + d].add(mi * fabs(t[d]));
    }
  }
  __shared__ double ss[kNSum][kBS], sc[kNSum][kBS];
  for (int q = 0; q < kNSum; ++q) {
    ss[q][threadIdx.x] = acc[q].s;
    sc[q][threadIdx.x] = acc[q].c;
  }
  __syncthreads();
  if (threadIdx.x < kNSum) {
    KS k;
    for (int t = 0; t < kBS; ++t) {
      KS o;
      o.s = ss[threadIdx.x][t];
      o.c = sc[threadIdx.x][t];
      k.add(o);
    }
    part[(int64_t)blockIdx.x * 2 * kNSum + 2 * threadIdx.x] = k.s;
    part[(int64_t)blockIdx.x * 2 * kNSum + 2 * threadIdx.x + 1] = k.c;
  }
}

__global__ void k_balance_final(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double tot[kNSum];
  if (threadIdx.x < kNSum) {
    KS k;
    for (int b = 0; b < nb; ++b) {
      KS o;
      o.s = part[(int64_t)b * 2 * kNSum + 2 * threadIdx.x];
      o.c = part[(int64_t)b * 2 * kNSum + 2 * threadIdx.x + 1];
      k.add(o);
    }
    tot[threadIdx.x] = k.s + k.c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double num = 0.0, den = 0.0, tnum = 0.0, tden = 0.0;
    for (int d = 0; d < 3; ++d) {
      num += tot[d] * tot[d];
      den += tot[3 + d] * tot[3 + d];
      tnum += tot[6 + d] * tot[6 + d];
      tden += tot[9 + d] * tot[9 + d];
    }
    out[0] = sqrt(num / den);
    out[1] = sqrt(tnum / tden);
  }
}

}  // namespace

void direct_sum(Ctx& c, int64_t n, const double* x, const double* y, const double* z, const double* m,
                int64_t ntarget, const int64_t* targets, double* ax, double* ay, double* az, double* pot,
                double* gabs) {
  if (ntarget <= 0) return;
  // split the sources so that the launch has enough blocks to fill the chip
  const int64_t tblocks = (ntarget + kBS - 1) / kBS;
  int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>((4096 + tblocks - 1) / tblocks, (n + 4095) / 4096));
  nchunk = std::min<int64_t>(nchunk, 65535);
  int64_t chunk = (n + nchunk - 1) / nchunk;
  chunk = (chunk + kBS - 1) / kBS * kBS;
  nchunk = (n + chunk - 1) / chunk;
  double* part = (double*)ensure(c, c.scratch2, sizeof(double) * 5 * (size_t)(nchunk * ntarget));
  hipLaunchKernelGGL(k_direct, dim3((unsigned)tblocks, (unsigned)nchunk), dim3(kBS), 0, c.stream, n, x, y, z, m,
                     ntarget, targets, chunk, part, c.opt.softening * c.opt.softening);
  hipLaunchKernelGGL(k_direct_sum, dim3((unsigned)tblocks), dim3(kBS), 0, c.stream, n, ntarget, targets,
                     (int)nchunk, (const double*)part, c.opt.G, ax, ay, az, pot, gabs);
  AMFMM_HIP(hipGetLastError());
}

void balance(Ctx& c, int64_t n, const double* x, const double* y, const double* z, const double* m,
             const double* ax, const double* ay, const double* az, double* out) {
  const int nb = (int)std::min<int64_t>(512, (n + kBS - 1) / kBS);
  double* part = (double*)ensure(c, c.scratch2, sizeof(double) * (2 * kNSum * (size_t)nb + 2));
  double* res = part + 2 * kNSum * (size_t)nb;
  hipLaunchKernelGGL(k_balance_partial, dim3(nb), dim3(kBS), 0, c.stream, n, x, y, z, m, ax, ay, az, part);
  hipLaunchKernelGGL(k_balance_final, dim3(1), dim3(64), 0, c.stream, nb, (const double*)part, res);
  AMFMM_HIP(hipGetLastError());
  AMFMM_HIP(hipMemcpyAsync(out, res, sizeof(double) * 2, hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
}

}  // namespace amfmm
