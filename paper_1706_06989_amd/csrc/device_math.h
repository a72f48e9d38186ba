// Small device helpers shared by the evaluation kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "amfmm.h"

namespace amfmm {

// T[p][m]: packed triple index of sorted(pair p, m) with pairs xx xy xz yy yz zz
// and triples xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
__device__ constexpr int kT3[6][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}, {3, 6, 7}, {4, 7, 8}, {5, 8, 9}};
// multiplicity of each packed pair in a full 3x3 contraction
__device__ constexpr double kMult2[6] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0};

// 1/sqrt(r2): hardware estimate refined by two Newton steps (full FP64)
__device__ inline double rsqrt_f64(double r2) {
  double y = __builtin_amdgcn_rsq(r2);
  const double h = 0.5 * r2;
  y = y * fma(-h, y * y, 1.5);
  y = y * fma(-h, y * y, 1.5);
  return y;
}

// 1/sqrt(r2) with one Newton step: relative error below 3e-14 (the hardware
// estimate is good to about 2^-23); used by the near field, where it sits far
// below both the method's error and the 1e-12 agreement with plain FP64
__device__ inline double rsqrt_f64_1nr(double r2) {
  double y = __builtin_amdgcn_rsq(r2);
  const double h = 0.5 * r2;
  return y * fma(-h, y * y, 1.5);
}

// Far-field coefficients of one source (moments M, quadrupole Q2) at R:
// acc[0] C, acc[1..3] C_k, acc[4..9] C_kl, acc[10..19] C_klm (packed).
// T = double (FP64 path) or float (mixed path).  The D tensors are written as
// sums over index pairings of the radial factors t_k = (1/R d/dR)^k g, which
// holds for any g of the distance alone: eps2 > 0 gives the softened g =
// -1/sqrt(R^2 + eps2) (Sec. 4), eps2 = 0 the plain -1/R (adding zero is exact).
template <typename T>
__device__ inline void far_coeffs(const T R[3], T M, const T Q2[6], T* acc, T eps2) {
  const T r2 = fma(R[0], R[0], fma(R[1], R[1], R[2] * R[2])) + eps2;
  T ri;
  if constexpr (sizeof(T) == 8) ri = rsqrt_f64(r2);
  else ri = __builtin_amdgcn_rsqf(r2);
  const T ri2 = ri * ri;
  const T t1 = ri * ri2;
  const T t2 = T(-3) * t1 * ri2;
  const T t3 = T(-5) * t2 * ri2;
  const T RR[6] = {R[0] * R[0], R[0] * R[1], R[0] * R[2], R[1] * R[1], R[1] * R[2], R[2] * R[2]};
  // D_kl and D_klm (packed)
  T D2[6], D3[10];
#pragma unroll
  for (int u = 0; u < 6; ++u) D2[u] = t2 * RR[u];
  D2[0] += t1;
  D2[3] += t1;
  D2[5] += t1;
  D3[0] = fma(t3 * RR[0], R[0], T(3) * t2 * R[0]);
  D3[1] = fma(t3 * RR[0], R[1], t2 * R[1]);
  D3[2] = fma(t3 * RR[0], R[2], t2 * R[2]);
  D3[3] = fma(t3 * RR[3], R[0], t2 * R[0]);
  D3[4] = t3 * RR[1] * R[2];
  D3[5] = fma(t3 * RR[5], R[0], t2 * R[0]);
  D3[6] = fma(t3 * RR[3], R[1], T(3) * t2 * R[1]);
  D3[7] = fma(t3 * RR[3], R[2], t2 * R[2]);
  D3[8] = fma(t3 * RR[5], R[1], t2 * R[1]);
  D3[9] = fma(t3 * RR[5], R[2], T(3) * t2 * R[2]);
  // contractions of the source quadrupole
  const T trQ = Q2[0] + Q2[3] + Q2[5];
  const T QR[3] = {fma(Q2[0], R[0], fma(Q2[1], R[1], Q2[2] * R[2])),
                   fma(Q2[1], R[0], fma(Q2[3], R[1], Q2[4] * R[2])),
                   fma(Q2[2], R[0], fma(Q2[4], R[1], Q2[5] * R[2]))};
  const T RQR = fma(R[0], QR[0], fma(R[1], QR[1], R[2] * QR[2]));
  acc[0] += fma(-M, ri, T(0.5) * fma(t2, RQR, t1 * trQ));
  const T a1 = fma(M, t1, T(0.5) * fma(t3, RQR, t2 * trQ));
#pragma unroll
  for (int k = 0; k < 3; ++k) acc[1 + k] += fma(a1, R[k], t2 * QR[k]);
#pragma unroll
  for (int u = 0; u < 6; ++u) acc[4 + u] = fma(M, D2[u], acc[4 + u]);
#pragma unroll
  for (int u = 0; u < 10; ++u) acc[10 + u] = fma(M, D3[u], acc[10 + u]);
}

// Q_jkl D_ijkl (TC) or Q_jkl D'_ijkl (TCO) of the correction, FP64, with
// Q = M_X,jkl M_Y - M_X M_Y,jkl; adds to F[3].  In the radial-factor form of
// far_coeffs (softened for eps2 > 0).
template <int VARIANT>
__device__ inline void far_correction(const double R[3], double MX, const double OX[10], double M, const double O3[10],
                                      double F[3], double eps2) {
  const double r2 = fma(R[0], R[0], fma(R[1], R[1], R[2] * R[2])) + eps2;
  const double ri = rsqrt_f64(r2);
  const double ri2 = ri * ri;
  const double t2 = -3.0 * (ri * ri2) * ri2;
  const double t3 = -5.0 * t2 * ri2;
  const double RR[6] = {R[0] * R[0], R[0] * R[1], R[0] * R[2], R[1] * R[1], R[1] * R[2], R[2] * R[2]};
  double Q[10];
#pragma unroll
  for (int u = 0; u < 10; ++u) Q[u] = fma(OX[u], M, -MX * O3[u]);
  const double mult[6] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0};
  double v[3], w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) s = fma(mult[p] * Q[kT3[p][i]], RR[p], s);
    v[i] = s;
  }
  w[0] = Q[0] + Q[3] + Q[5];
  w[1] = Q[1] + Q[6] + Q[8];
  w[2] = Q[2] + Q[7] + Q[9];
  if (VARIANT == AMFMM_TC) {
    const double t4 = -7.0 * t3 * ri2;
    const double s = fma(R[0], v[0], fma(R[1], v[1], R[2] * v[2]));
    const double wR = fma(R[0], w[0], fma(R[1], w[1], R[2] * w[2]));
#pragma unroll
    for (int i = 0; i < 3; ++i) F[i] += fma(t4 * s, R[i], 3.0 * fma(t3, fma(R[i], wR, v[i]), t2 * w[i]));
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) F[i] += 3.0 * fma(t3, v[i], t2 * w[i]);
  }
}

// The correction of eq. 7 (TC) from traceless octupoles (plain -1/R only: the
// softened D_ijkl is not traceless): D_ijkl is traceless
// in every pair of indices, so only the traceless part of Q = M_X,jkl M_Y -
// M_X M_Y,jkl contributes, and with a traceless Q the closed form reduces to
// t4 R_i (Q.RRR) + 3 t3 Q_ikl R_k R_l.  OXt, O3t: traceless octupoles (10
// packed components); adds to F[3].
__device__ inline void far_correction_traceless(const double R[3], double MX, const double OXt[10], double M,
                                                const double O3t[10], double F[3]) {
  const double r2 = fma(R[0], R[0], fma(R[1], R[1], R[2] * R[2]));
  const double ri = rsqrt_f64(r2);
  const double ri2 = ri * ri;
  const double t3 = 15.0 * ((ri * ri2) * ri2) * ri2;
  const double t4 = -7.0 * t3 * ri2;
  const double RR[6] = {R[0] * R[0], R[0] * R[1], R[0] * R[2], R[1] * R[1], R[1] * R[2], R[2] * R[2]};
  double Q[10];
#pragma unroll
  for (int u = 0; u < 10; ++u) Q[u] = fma(OXt[u], M, -MX * O3t[u]);
  const double mult[6] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0};
  double v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) s = fma(mult[p] * Q[kT3[p][i]], RR[p], s);
    v[i] = s;
  }
  const double s = fma(R[0], v[0], fma(R[1], v[1], R[2] * v[2]));
#pragma unroll
  for (int i = 0; i < 3; ++i) F[i] += fma(t4 * s, R[i], 3.0 * t3 * v[i]);
}

// traceless part of a packed symmetric octupole (xxx xxy xxz xyy xyz xzz yyy
// yyz yzz zzz): T_jkl - (delta_jk u_l + delta_jl u_k + delta_kl u_j)/5, u_l = T_jjl
__device__ inline void octupole_traceless(const double O[10], double T[10]) {
  const double ux = O[0] + O[3] + O[5], uy = O[1] + O[6] + O[8], uz = O[2] + O[7] + O[9];
  T[0] = O[0] - 0.6 * ux;
  T[1] = O[1] - 0.2 * uy;
  T[2] = O[2] - 0.2 * uz;
  T[3] = O[3] - 0.2 * ux;
  T[4] = O[4];
  T[5] = O[5] - 0.2 * ux;
  T[6] = O[6] - 0.6 * uy;
  T[7] = O[7] - 0.2 * uz;
  T[8] = O[8] - 0.2 * uy;
  T[9] = O[9] - 0.6 * uz;
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (all lanes active): four shifts within each row of 16, then row
// 0's total into row 1 and row 2's into row 3, then row 1's into rows 2, 3.
__device__ inline int32_t wave_incl_scan(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b on XCD
// b mod 8), each with its own L2.  This bijection on [0, nb) gives each XCD
// runs of kRun consecutive work blocks (runs dealt round-robin, so the load
// stays balanced), so that neighbouring cells, which share sources, are
// served by the same L2.  Blocks past the last full round keep their index.
constexpr uint32_t kXcds = 8, kRun = 32;
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t full = nb / (kXcds * kRun) * (kXcds * kRun);
  if (b >= full) return b;
  const uint32_t x = b % kXcds, q = b / kXcds;
  return ((q / kRun) * kXcds + x) * kRun + q % kRun;
}

template <typename T>
__device__ inline T uniform(T v) {
  return (T)__builtin_amdgcn_readfirstlane((int)v);
}

// Taylor polynomial of a cell's coefficients (kLoc layout) at offset x:
// acceleration g (including the constant correction g_c) and potential phi
__device__ inline void eval_local(const double* L, const double x[3], double g[3], double& phi) {
  const double xx[6] = {x[0] * x[0], x[0] * x[1], x[0] * x[2], x[1] * x[1], x[1] * x[2], x[2] * x[2]};
  double C3xx[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double v = 0.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) v = fma(kMult2[p] * L[10 + kT3[p][k]], xx[p], v);
    C3xx[k] = v;
  }
  const double C2x[3] = {fma(L[4], x[0], fma(L[5], x[1], L[6] * x[2])),
                         fma(L[5], x[0], fma(L[7], x[1], L[8] * x[2])),
                         fma(L[6], x[0], fma(L[8], x[1], L[9] * x[2]))};
  phi = L[0];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g[k] = L[20 + k] - (L[1 + k] + C2x[k] + 0.5 * C3xx[k]);
    phi += x[k] * (L[1 + k] + 0.5 * C2x[k] + (1.0 / 6.0) * C3xx[k]);
  }
}

}  // namespace amfmm
