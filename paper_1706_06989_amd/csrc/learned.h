// Learned pair selection: pair features, the network's FP32 inference and the
// accept rule.  Not in the paper: a network predicts the force error of an
// accepted pair, taking the role of the error-estimating pair selection that
// Sec. 2 cites.  Everything here is defined so that the decision is a
// function of the unordered pair, reproducible bit for bit: features use
// IEEE-rounded operations on centres, radii, masses and counts (bit-exact
// across implementations) and a quadrupole norm quantised to 1/64 of
// M R_max^2; the network runs in FP32 with fused multiply-adds in a fixed
// order on BF16-rounded weights.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "amfmm.h"

namespace amfmm {

constexpr int kFeat = 8, kHid = 64;
// model layout (floats): W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3,
// normalisation a[8], b[8] (x = fma(f, a, b)), training range lo[8], hi[8]
constexpr int kW1 = 0, kB1 = 512, kW2 = 576, kB2 = 4672, kW3 = 4736, kB3 = 4800;
constexpr int kNA = 4801, kNB = 4809, kLo = 4817, kHi = 4825;
static_assert(kHi + kFeat == AMFMM_MLP_MODEL, "model layout");
static_assert(kB3 + 1 == AMFMM_MLP_PARAMS, "parameter layout");

// analytic error factor q^3 against the allowed factor u: below u/4 accept,
// above 16 u open, in between the network decides
constexpr double kGateLo = 0.25, kGateHi = 16.0;
constexpr int32_t kCountCap = 1024;  // particle counts saturate here in the features

// nearest BF16 value (ties to even), as float
__host__ __device__ inline float bf16r(float v) {
  uint32_t u = __builtin_bit_cast(uint32_t, v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  return __builtin_bit_cast(float, u);
}

// piecewise-linear log2: x = 2^e (1 + f), f in [0, 1) -> e + f
__device__ inline double plog2(double x) {
  if (!(x > 0.0)) return -2048.0;
  if (__builtin_isinf(x)) return 2048.0;
  int e;
  const double m = frexp(x, &e);  // x = m 2^e, m in [0.5, 1)
  return (double)(e - 1) + (2.0 * m - 1.0);
}

// ||M_ij||_F / (M R_max^2) in [0, 1] to the nearest multiple of 1/64, from
// packed xx xy xz yy yz zz (exact values such as 1, two equal masses, sit
// mid-bin, away from the boundaries where rounding could move them)
__device__ inline int quad_level(double M, double R, const double* Q2) {
  const double s = Q2[0] * Q2[0] + Q2[3] * Q2[3] + Q2[5] * Q2[5] +
                   2.0 * (Q2[1] * Q2[1] + Q2[2] * Q2[2] + Q2[4] * Q2[4]);
  const double den = M * (R * R);
  if (!(den > 0.0)) return 0;
  const double k = floor(64.0 * (sqrt(s) / den) + 0.5);
  return k < 0.0 ? 0 : (k > 64.0 ? 64 : (int)k);
}

struct PairSide {
  double R, M;
  int q;
  int32_t n;
};

// the eight features of an unordered pair at centre distance d > 0
__device__ inline void pair_features(double d, const PairSide& A, const PairSide& B, float f[kFeat]) {
  const double r = A.R + B.R;
  f[0] = (float)(r / d);
  f[1] = (float)plog2(r / d);
  f[2] = (float)(r > 0.0 ? fabs(A.R - B.R) / r : 0.0);
  f[3] = (float)(fabs(A.M - B.M) / (A.M + B.M));
  f[4] = (float)((double)(A.q + B.q) / 128.0);
  f[5] = (float)((double)abs(A.q - B.q) / 64.0);
  // counts saturate at kCountCap (a larger cell behaves as a continuum)
  const double ca = (double)(A.n < kCountCap ? A.n : kCountCap), cb = (double)(B.n < kCountCap ? B.n : kCountCap);
  f[6] = (float)plog2(ca * cb);
  f[7] = (float)fabs(plog2(ca) - plog2(cb));
}

// FP32 inference; P holds BF16-rounded weights (biases and normalisation as
// given) and is the same for every lane: the weight reads become scalar
// loads.  Kept out of line so that the walk kernels calling it keep their
// own register budget.
__device__ __noinline__ float mlp_infer8(const float* __restrict__ Pin, float f0, float f1, float f2, float f3,
                                         float f4, float f5, float f6, float f7) {
  const uint64_t pu = (uint64_t)Pin;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pu);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(pu >> 32));
  const float* __restrict__ P = (const float*)(((uint64_t)hi << 32) | lo);
  const float f[kFeat] = {f0, f1, f2, f3, f4, f5, f6, f7};
  float x[kFeat];
#pragma unroll
  for (int i = 0; i < kFeat; ++i) x[i] = bf16r(fmaf(f[i], P[kNA + i], P[kNB + i]));
  // Layer 2 in two halves of its outputs; the hidden layer 1 is recomputed
  // per half (j outer), so only 32 accumulators are live.  Every output k
  // still sums its inputs j = 0..63 in order: the result is the same as with
  // the layers evaluated one after the other.
  float y = P[kB3];
  for (int half = 0; half < 2; ++half) {
    float s2[kHid / 2];
#pragma unroll
    for (int k = 0; k < kHid / 2; ++k) s2[k] = P[kB2 + half * (kHid / 2) + k];
    for (int j = 0; j < kHid; ++j) {
      float s = P[kB1 + j];
#pragma unroll
      for (int i = 0; i < kFeat; ++i) s = fmaf(P[kW1 + kFeat * j + i], x[i], s);
      const float h = bf16r(s > 0.0f ? s : 0.0f);
#pragma unroll
      for (int k = 0; k < kHid / 2; ++k) s2[k] = fmaf(P[kW2 + kHid * (half * (kHid / 2) + k) + j], h, s2[k]);
    }
#pragma unroll
    for (int k = 0; k < kHid / 2; ++k) y = fmaf(P[kW3 + half * (kHid / 2) + k], bf16r(s2[k] > 0.0f ? s2[k] : 0.0f), y);
  }
  return y;
}

__device__ inline float mlp_infer(const float* __restrict__ P, const float f[kFeat]) {
  return mlp_infer8(P, f[0], f[1], f[2], f[3], f[4], f[5], f[6], f[7]);
}

// Learned accept decision of a pair with d > 0 and R_A + R_B <= theta_max d;
// s = field scales, eps = accepted error relative to them, min_work = least
// N_A N_B for which the network is asked; smaller pairs and pairs with
// features outside the training range take the analytic factor q^3
__device__ inline bool learned_accept(const float* __restrict__ P, double eps, int64_t min_work,
                                      double d, const PairSide& A, double sA, const PairSide& B, double sB) {
  const double r = A.R + B.R;
  const double q = r / d;
  const double uA = (eps * sA) * (d * d) / B.M, uB = (eps * sB) * (d * d) / A.M;
  const double u = uB < uA ? uB : uA;
  const double q3 = q * q * q;
  if (q3 <= kGateLo * u) return true;
  if (q3 > kGateHi * u) return false;
  if ((int64_t)A.n * (int64_t)B.n < min_work) return q3 <= u;
  float f[kFeat];
  pair_features(d, A, B, f);
  bool in = true;
#pragma unroll
  for (int i = 0; i < kFeat; ++i) in = in && (f[i] >= P[kLo + i] && f[i] <= P[kHi + i]);
  if (!in) return q3 <= u;
  return mlp_infer(P, f) <= (float)plog2(u);
}

}  // namespace amfmm
