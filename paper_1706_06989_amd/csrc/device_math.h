// Small device helpers shared by the evaluation kernels.
#pragma once
#include <hip/hip_runtime.h>

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
