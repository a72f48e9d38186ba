// Evaluation: far field per target cell, push-down to the leaves, and the
// near field fused with the evaluation at the particles and the unsort.
//
// Far field (eqs. 2-4, dipoles dropped, octupole constant dropped): for the
// target X and a source Y with R = Z_X - Z_Y, the Taylor coefficients of the
// potential about Z_X are
//   C    += M_Y D + 1/2 M_Y,lm D_lm          C_k   += M_Y D_k + 1/2 M_Y,lm D_klm
//   C_kl += M_Y D_kl                          C_klm += M_Y D_klm
// (eq. 2 read as a polynomial in x; eq. 4 for the other cell of a pair is the
// same expression with R -> -R, so directed evaluation per target reproduces
// the symmetric pair exactly up to summation order).  The correction of eq. 7
// (prefactor 1/6, see the appendix at P = 3) adds F_c/M_X to X with
//   F_c,i = -(1/6) Q_jkl D_ijkl,  Q = M_X,jkl M_Y - M_X M_Y,jkl,
// contracted in closed form: Q_jkl D_ijkl = t4 R_i (Q.RRR) + 3 t3 (Q_ikl R_k
// R_l + R_i Q_jkk R_j) + 3 t2 Q_ikk with t2 = -3/R^5, t3 = 15/R^7, t4 =
// -105/R^9.  Eq. 8 keeps only 3 t3 Q_ikl R_k R_l + 3 t2 Q_ikk.
//
// One wave per target cell, lanes over its sources, fixed-order butterfly
// reduction (deterministic).  Mixed precision: R = Z_X - Z_Y is formed in FP64
// and rounded, the coefficient terms are FP32 and each lane adds at most
// kFarFlush of them in FP32 before an FP64 flush; the correction (which
// cancels M_X,jkl M_Y against M_X M_Y,jkl) stays FP64.  For UC and TC the
// mixed path reads each source from one 128-byte record (one cache line
// instead of three): Z and M in FP64, the traceless octupole (7 components,
// FP64; D_ijkl is traceless, so the correction needs no more) and the
// quadrupole in FP32.
#include "device_math.h"
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sources per lane summed in FP32 before an FP64 flush (mixed path)
constexpr int kFarFlush = 8;

// far-field source record of the mixed UC/TC path: 128 bytes, one cache line
struct alignas(128) FarRec {
  double z[3], m;
  double o[7];  // traceless octupole: xxx xxy xxz xyy xyz yyy yyz (xzz, yzz, zzz follow)
  float q[6];   // quadrupole xx xy xz yy yz zz
  float pad[4];
};
static_assert(sizeof(FarRec) == 128, "far record");

__global__ void __launch_bounds__(kBS) k_pack_far(int32_t nc, const double4* __restrict__ geo,
                                                  const double* __restrict__ mom, FarRec* __restrict__ rec) {
  const int32_t c = blockIdx.x * kBS + threadIdx.x;
  if (c >= nc) return;
  const double4 g = geo[c];
  const double* mo = mom + (int64_t)c * kMom;
  double T[10];
  octupole_traceless(mo + 7, T);
  FarRec r;
  r.z[0] = g.x;
  r.z[1] = g.y;
  r.z[2] = g.z;
  r.m = mo[0];
  r.o[0] = T[0];
  r.o[1] = T[1];
  r.o[2] = T[2];
  r.o[3] = T[3];
  r.o[4] = T[4];
  r.o[5] = T[6];
  r.o[6] = T[7];
#pragma unroll
  for (int u = 0; u < 6; ++u) r.q[u] = (float)mo[1 + u];
#pragma unroll
  for (int u = 0; u < 4; ++u) r.pad[u] = 0.0f;
  rec[c] = r;
}

// the full traceless octupole of a record
__device__ inline void record_octupole(const double o[7], double T[10]) {
  T[0] = o[0];
  T[1] = o[1];
  T[2] = o[2];
  T[3] = o[3];
  T[4] = o[4];
  T[5] = -o[0] - o[3];
  T[6] = o[5];
  T[7] = o[6];
  T[8] = -o[1] - o[5];
  T[9] = -o[2] - o[6];
}

// Mixed UC/TC far field from the records (see k_far)
template <int VARIANT>
__global__ void __launch_bounds__(kBS) k_far_rec(int32_t c_lo, int32_t nc, const FarRec* __restrict__ rec,
                                                 const int64_t* __restrict__ fstart,
                                                 const int32_t* __restrict__ fcount,
                                                 const int32_t* __restrict__ fsrc, double* __restrict__ loc) {
  const int lane = threadIdx.x & 63;
  const int32_t Xi = uniform((int32_t)(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6)));
  if (Xi >= nc) return;
  const int32_t X = c_lo + Xi;
  const int32_t cnt = fcount[X];
  const int64_t st = fstart[X];
  const FarRec& rx = rec[X];
  const double gx[3] = {rx.z[0], rx.z[1], rx.z[2]};
  const double MX = rx.m;
  double OX[10];
  if (VARIANT) record_octupole(rx.o, OX);
  double acc[20], F[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 20; ++u) acc[u] = 0.0;
  for (int64_t j0 = lane; j0 < cnt; j0 += 64 * kFarFlush) {
    float a32[20];
#pragma unroll
    for (int u = 0; u < 20; ++u) a32[u] = 0.0f;
    const int64_t j1 = j0 + 64 * kFarFlush < cnt ? j0 + 64 * kFarFlush : cnt;
    for (int64_t j = j0; j < j1; j += 64) {
      const FarRec& ry = rec[fsrc[st + j]];
      const double R[3] = {gx[0] - ry.z[0], gx[1] - ry.z[1], gx[2] - ry.z[2]};
      const double M = ry.m;
      const float Rf[3] = {(float)R[0], (float)R[1], (float)R[2]};
      float Q2f[6];
#pragma unroll
      for (int u = 0; u < 6; ++u) Q2f[u] = ry.q[u];
      far_coeffs<float>(Rf, (float)M, Q2f, a32, 0.0f);
      if (VARIANT) {
        double O3[10];
        record_octupole(ry.o, O3);
        far_correction_traceless(R, MX, OX, M, O3, F);
      }
    }
#pragma unroll
    for (int u = 0; u < 20; ++u) acc[u] += (double)a32[u];
  }
#pragma unroll
  for (int u = 0; u < 20; ++u) acc[u] = wave_sum(acc[u]);
#pragma unroll
  for (int i = 0; i < 3; ++i) F[i] = wave_sum(F[i]);
  if (lane == 0) {
    double* o = loc + (int64_t)X * kLoc;
    const double cf = -1.0 / (6.0 * MX);
#pragma unroll
    for (int u = 0; u < 20; ++u) o[u] = acc[u];
#pragma unroll
    for (int i = 0; i < 3; ++i) o[20 + i] = VARIANT ? cf * F[i] : 0.0;
    o[23] = 0.0;
  }
}

template <int VARIANT, bool MIXED>
__global__ void __launch_bounds__(kBS) k_far(int32_t c_lo, int32_t nc, const double4* __restrict__ geo, const double* __restrict__ mom,
                                             const int64_t* __restrict__ fstart, const int32_t* __restrict__ fcount,
                                             const int32_t* __restrict__ fsrc, double* __restrict__ loc, double eps2) {
  const int lane = threadIdx.x & 63;
  const int32_t Xi = uniform((int32_t)(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6)));
  if (Xi >= nc) return;
  const int32_t X = c_lo + Xi;
  const int32_t cnt = fcount[X];
  const int64_t st = fstart[X];
  const double4 gx = geo[X];
  const double* mx = mom + (int64_t)X * kMom;
  const double MX = mx[0];
  double OX[10];
#pragma unroll
  for (int u = 0; u < 10; ++u) OX[u] = VARIANT ? mx[7 + u] : 0.0;
  double acc[20], F[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 20; ++u) acc[u] = 0.0;
  const int64_t step = MIXED ? 64 * kFarFlush : (int64_t)cnt + 64;
  for (int64_t j0 = lane; j0 < cnt; j0 += step) {
    float a32[20];
#pragma unroll
    for (int u = 0; u < 20; ++u) a32[u] = 0.0f;
    const int64_t j1 = j0 + step < cnt ? j0 + step : cnt;
    for (int64_t j = j0; j < j1; j += 64) {
      const int32_t Y = fsrc[st + j];
      const double4 gy = geo[Y];
      const double* my = mom + (int64_t)Y * kMom;
      const double M = my[0];
      const double R[3] = {gx.x - gy.x, gx.y - gy.y, gx.z - gy.z};
      if (MIXED) {
        const float Rf[3] = {(float)R[0], (float)R[1], (float)R[2]};
        float Q2f[6];
#pragma unroll
        for (int u = 0; u < 6; ++u) Q2f[u] = (float)my[1 + u];
        far_coeffs<float>(Rf, (float)M, Q2f, a32, (float)eps2);
      } else {
        double Q2[6];
#pragma unroll
        for (int u = 0; u < 6; ++u) Q2[u] = my[1 + u];
        far_coeffs<double>(R, M, Q2, acc, eps2);
      }
      if (VARIANT) {
        double O3[10];
#pragma unroll
        for (int u = 0; u < 10; ++u) O3[u] = my[7 + u];
        far_correction<VARIANT>(R, MX, OX, M, O3, F, eps2);
      }
    }
    if (MIXED) {
#pragma unroll
      for (int u = 0; u < 20; ++u) acc[u] += (double)a32[u];
    }
  }
#pragma unroll
  for (int u = 0; u < 20; ++u) acc[u] = wave_sum(acc[u]);
#pragma unroll
  for (int i = 0; i < 3; ++i) F[i] = wave_sum(F[i]);
  if (lane == 0) {
    double* o = loc + (int64_t)X * kLoc;
    const double cf = -1.0 / (6.0 * MX);
#pragma unroll
    for (int u = 0; u < 20; ++u) o[u] = acc[u];
#pragma unroll
    for (int i = 0; i < 3; ++i) o[20 + i] = VARIANT ? cf * F[i] : 0.0;
    o[23] = 0.0;
  }
}

// loc[child] += Taylor shift of loc[parent] to the child's centre
__global__ void __launch_bounds__(kBS) k_l2l(int32_t c0, int32_t nl, const int32_t* __restrict__ par,
                                             const double4* __restrict__ geo, double* __restrict__ loc) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  const int32_t c = c0 + i;
  const int32_t P = par[c];
  const double4 gc = geo[c], gp = geo[P];
  const double d[3] = {gc.x - gp.x, gc.y - gp.y, gc.z - gp.z};
  const double* L = loc + (int64_t)P * kLoc;
  double* o = loc + (int64_t)c * kLoc;
  double C1[3] = {L[1], L[2], L[3]};
  double C2[6], C3[10];
#pragma unroll
  for (int u = 0; u < 6; ++u) C2[u] = L[4 + u];
#pragma unroll
  for (int u = 0; u < 10; ++u) C3[u] = L[10 + u];
  const double dd[6] = {d[0] * d[0], d[0] * d[1], d[0] * d[2], d[1] * d[1], d[1] * d[2], d[2] * d[2]};
  const double mult[6] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0};
  // (C3 dd)_k and (C2 d)_k
  double C3dd[3], C2d[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) s = fma(mult[p] * C3[kT3[p][k]], dd[p], s);
    C3dd[k] = s;
  }
  C2d[0] = fma(C2[0], d[0], fma(C2[1], d[1], C2[2] * d[2]));
  C2d[1] = fma(C2[1], d[0], fma(C2[3], d[1], C2[4] * d[2]));
  C2d[2] = fma(C2[2], d[0], fma(C2[4], d[1], C2[5] * d[2]));
  double c0v = L[0];
#pragma unroll
  for (int k = 0; k < 3; ++k) c0v += d[k] * (C1[k] + 0.5 * C2d[k] + (1.0 / 6.0) * C3dd[k]);
  o[0] += c0v;
#pragma unroll
  for (int k = 0; k < 3; ++k) o[1 + k] += C1[k] + C2d[k] + 0.5 * C3dd[k];
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    double s = C2[p];
#pragma unroll
    for (int m = 0; m < 3; ++m) s = fma(C3[kT3[p][m]], d[m], s);
    o[4 + p] += s;
  }
#pragma unroll
  for (int u = 0; u < 10; ++u) o[10 + u] += C3[u];
#pragma unroll
  for (int i2 = 0; i2 < 3; ++i2) o[20 + i2] += L[20 + i2];
}

__global__ void k_zero_u64_n(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

}  // namespace

void zero_u64(Ctx& c, unsigned long long* p, int n) {
  hipLaunchKernelGGL(k_zero_u64_n, dim3(1), dim3(64), 0, c.stream, p, n);
  AMFMM_HIP(hipGetLastError());
}

// the 128-byte records carry traceless octupoles, enough for the correction
// of the plain -1/R only (mixed UC and TC)
static bool use_records(const Ctx& c) {
  return c.opt.precision == AMFMM_MIXED && c.opt.variant != AMFMM_TCO && c.opt.softening == 0.0 && c.opt.order == 3;
}

void far_prepare(Ctx& c) {
  if (!use_records(c) || c.ncells <= 0) return;
  FarRec* rec = (FarRec*)ensure(c, c.farrec, sizeof(FarRec) * (size_t)c.ncells);
  hipLaunchKernelGGL(k_pack_far, dim3(blocks_for(c.ncells, kBS)), dim3(kBS), 0, c.stream, c.ncells,
                     (const double4*)c.geo.p, (const double*)c.mom.p, rec);
  AMFMM_HIP(hipGetLastError());
}

void far_field(Ctx& c, int32_t c_lo, int32_t c_hi) {
  const int32_t nc = c_hi - c_lo;
  if (nc <= 0) return;
  double* loc = (double*)ensure_keep(c, c.loc, sizeof(double) * kLoc * (size_t)c.ncells,
                                     sizeof(double) * kLoc * (size_t)c.ncells);
  if (c.opt.order != 3) {
    ++c.far_launches;
    order_far(c, c_lo, c_hi, loc);
    return;
  }
  dim3 grid(blocks_for(nc, kWaves));
  if (use_records(c)) {
    ++c.far_launches;
    hipLaunchKernelGGL(c.opt.variant == AMFMM_TC ? k_far_rec<AMFMM_TC> : k_far_rec<AMFMM_UC>, grid, dim3(kBS), 0,
                       c.stream, c_lo, nc, (const FarRec*)c.farrec.p, (const int64_t*)c.far_start.p,
                       (const int32_t*)c.far_count.p, (const int32_t*)c.far_src.p, loc);
    AMFMM_HIP(hipGetLastError());
    return;
  }
  auto args = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(kBS), 0, c.stream, c_lo, nc, (const double4*)c.geo.p, (const double*)c.mom.p,
                       (const int64_t*)c.far_start.p, (const int32_t*)c.far_count.p, (const int32_t*)c.far_src.p, loc,
                       c.opt.softening * c.opt.softening);
  };
  ++c.far_launches;
  const bool mixed = c.opt.precision == AMFMM_MIXED;
  switch (c.opt.variant) {
    case AMFMM_UC: mixed ? args(k_far<AMFMM_UC, true>) : args(k_far<AMFMM_UC, false>); break;
    case AMFMM_TC: mixed ? args(k_far<AMFMM_TC, true>) : args(k_far<AMFMM_TC, false>); break;
    default: mixed ? args(k_far<AMFMM_TCO, true>) : args(k_far<AMFMM_TCO, false>); break;
  }
  AMFMM_HIP(hipGetLastError());
}

void push_down(Ctx& c, int32_t c_lo, int32_t c_hi) {
  const int32_t nl = c_hi - c_lo;
  if (nl <= 0) return;
  if (c.opt.order != 3) {  // the order-3 records hold zeros
    order_push_down(c, c_lo, c_hi);
    return;
  }
  hipLaunchKernelGGL(k_l2l, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, c_lo, nl, as<int32_t>(c.c_parent),
                     (const double4*)c.geo.p, as<double>(c.loc));
  AMFMM_HIP(hipGetLastError());
}

}  // namespace amfmm
