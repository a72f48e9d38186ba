// The multipole error estimate and the learned pair selection built on it.
// Neither is in the paper: both take the role of the error-based pair
// selection Sec. 2 cites.  The estimate bounds the error of an accepted pair
// from the terms a third-order expansion drops; the network predicts, from
// eight features of the pair, how far the error the method actually makes
// lies from that estimate.  Everything here is defined so that the decision
// is a function of the unordered pair, reproducible bit for bit: features use
// IEEE-rounded operations on centres, radii, masses and counts and the
// traceless norm levels (quantised to 1/128); the network runs in FP32 with
// fused multiply-adds in a fixed order on BF16-rounded weights.
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

// The network is asked where the multipole estimate sits near the allowed
// error (rho in (1/4, 2]); below the band the pair is accepted, above it
// opened.  The method's error stays within a factor of about 2 of the
// estimate on the training pairs (log2 ratio 0.04 to 0.98 between the 10th
// and 90th percentiles), so predictions rarely reach beyond the band.
// Powers of two: scaling eps by them is exact.
constexpr double kGateLo = 0.25, kGateHi = 2.0;
constexpr int32_t kCountCap = 1024;  // particle counts saturate here in the features

// The multipole estimate of the error of an accepted pair on field cell T
// from source S (Sec. 2's error-based selection, built from the parts a
// third-order expansion drops: S's traceless octupole, S's traceless
// quadrupole over T's extent, and the truncation of S's field over T; the next
// order adds R^4/d terms), per unit mass of S and times d^6:
//   P d + Q,  P = w3 k3_S R_S^3 + w2 k2_S R_S^2 R_T + w1 R_T^3,  Q = w4 R_S^4 + w5 R_T^4
// with k2, k3 the traceless norms in units of M R^2, M R^3.  The weights are a
// least-squares fit in log space to the largest error this method makes from
// each accepted pair of geometric walks of a 65536-particle Plummer sphere
// (opening angles 0.4, 0.6, 0.8); w1 >= 1 is used by the subtree rule of the
// walk.
constexpr double kMw1 = 1.326, kMw2 = 4.095, kMw3 = 0.285, kMw4 = 0.1416, kMw5 = 1.618;
constexpr double kMq = 128.0;  // the norm ratios are held to the nearest 1/128

__device__ inline double multipole_bracket(double rt, double rs, int k2s, int k3s, double d) {
  const double rt2 = rt * rt, rs2 = rs * rs;
  const double P = ((kMw3 * (k3s / kMq)) * (rs2 * rs) + (kMw2 * (k2s / kMq)) * (rs2 * rt)) + kMw1 * (rt2 * rt);
  const double Q = kMw4 * (rs2 * rs2) + kMw5 * (rt2 * rt2);
  return P * d + Q;
}

// Frobenius norms of the traceless parts of M_ij (packed xx xy xz yy yz zz)
// and of M_ijk (packed xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz): M_ij -
// delta_ij tr/3 and M_ijk - (v_i delta_jk + v_j delta_ik + v_k delta_ij)/5,
// v_i = M_ijj.  Squares are summed over all index tuples in row-major order
// (the order of the plain definition, so the result rounds the same way).
__device__ inline double traceless_norm2(const double* Q) {
  const double m[3][3] = {{Q[0], Q[1], Q[2]}, {Q[1], Q[3], Q[4]}, {Q[2], Q[4], Q[5]}};
  const double tr = m[0][0] + m[1][1] + m[2][2];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double v = m[i][j] - (i == j ? tr / 3.0 : 0.0);
      s += v * v;
    }
  return sqrt(s);
}

// packed position of M_ijk (symmetric: any order of i, j, k)
__device__ inline int oct_index(int i, int j, int k) {
  constexpr int idx[27] = {0, 1, 2, 1, 3, 4, 2, 4, 5, 1, 3, 4, 3, 6, 7, 4, 7, 8, 2, 4, 5, 4, 7, 8, 5, 8, 9};
  return idx[9 * i + 3 * j + k];
}

__device__ inline double traceless_norm3(const double* O) {
  double v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = O[oct_index(i, 0, 0)] + O[oct_index(i, 1, 1)] + O[oct_index(i, 2, 2)];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double dij = i == j ? 1.0 : 0.0, dik = i == k ? 1.0 : 0.0, djk = j == k ? 1.0 : 0.0;
        const double w = O[oct_index(i, j, k)] - (v[i] * djk + v[j] * dik + v[k] * dij) / 5.0;
        s += w * w;
      }
  return sqrt(s);
}

// norm / (M R^p) to the nearest 1/kMq, in [0, kMq] (0 where M R^p = 0)
__device__ inline int norm_level(double norm, double M, double R, int p) {
  const double den = M * (p == 2 ? R * R : R * R * R);
  if (!(den > 0.0)) return 0;
  const double k = floor(kMq * (norm / den) + 0.5);
  return k < 0.0 ? 0 : (k > kMq ? (int)kMq : (int)k);
}

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

// one cell of a pair: radius, mass, traceless norm levels, particles, field scale
struct PairSide {
  double R, M;
  int k2, k3;
  int32_t n;
  double s;
};

// the eight features of an unordered pair at centre distance d > 0, each
// symmetric in the two cells
__device__ inline void pair_features(double d, const PairSide& A, const PairSide& B, float f[kFeat]) {
  const double r = A.R + B.R;
  f[0] = (float)(r / d);
  f[1] = (float)(r > 0.0 ? fabs(A.R - B.R) / r : 0.0);
  f[2] = (float)((double)(A.k2 + B.k2) / (2.0 * kMq));
  f[3] = (float)((double)abs(A.k2 - B.k2) / kMq);
  f[4] = (float)((double)(A.k3 + B.k3) / (2.0 * kMq));
  f[5] = (float)((double)abs(A.k3 - B.k3) / kMq);
  f[6] = (float)(fabs(A.M - B.M) / (A.M + B.M));
  // counts saturate at kCountCap (a larger cell behaves as a continuum)
  const double ca = (double)(A.n < kCountCap ? A.n : kCountCap), cb = (double)(B.n < kCountCap ? B.n : kCountCap);
  f[7] = (float)plog2(ca * cb);
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

// The model as the walk keeps it in LDS: the same layout, but W2 transposed
// (entry kW2 + kHid j + k holds W2[k][j]), so that the weights of one input j
// to the 64 units of layer 2 are contiguous.
__device__ inline int lds_model_index(int i) {
  if (i < kW2 || i >= kB2) return i;
  const int k = (i - kW2) / kHid, j = (i - kW2) % kHid;
  return kW2 + kHid * j + k;
}

__device__ inline float mlp_infer(const float* __restrict__ P, const float f[kFeat]) {
  return mlp_infer8(P, f[0], f[1], f[2], f[3], f[4], f[5], f[6], f[7]);
}

// What lane j of a wave holds of the network for cooperative inference:
// hidden unit j of layer 1 (row j of W1, b1[j]) and of layer 2 (b2[j]), and
// its output weight w3[j].  P: the LDS copy.
struct MlpLane {
  float w1[kFeat];
  float b1, b2, w3;
};

__device__ inline MlpLane mlp_lane(const float* P) {
  const int j = threadIdx.x & 63;
  MlpLane L;
#pragma unroll
  for (int i = 0; i < kFeat; ++i) L.w1[i] = P[kW1 + kFeat * j + i];
  L.b1 = P[kB1 + j];
  L.b2 = P[kB2 + j];
  L.w3 = P[kW3 + j];
  return L;
}

__device__ inline float lane_value(float v, int j) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
}

// The network's output for one pair's features f (the same in every lane),
// computed by the whole wave (all 64 lanes active): lane j evaluates unit j of
// each hidden layer, the inputs of a layer come from the lanes holding the
// layer below, and the output sums the units in order.  The operations and
// their order are those of mlp_infer8: the result is bit-identical.  P: the
// LDS copy (lane k reads W2[k][j] at kW2 + kHid j + k, conflict-free).
__device__ inline float mlp_infer_wave(const float* P, const MlpLane& L, const float f[kFeat]) {
  const int k = threadIdx.x & 63;
  float s = L.b1;
#pragma unroll
  for (int i = 0; i < kFeat; ++i) s = fmaf(L.w1[i], bf16r(fmaf(f[i], P[kNA + i], P[kNB + i])), s);
  const float h = bf16r(s > 0.0f ? s : 0.0f);
  float s2 = L.b2;
#pragma unroll 8
  for (int j = 0; j < kHid; ++j) s2 = fmaf(P[kW2 + kHid * j + k], lane_value(h, j), s2);
  const float h2 = bf16r(s2 > 0.0f ? s2 : 0.0f);
  float y = P[kB3];
#pragma unroll 8
  for (int j = 0; j < kHid; ++j) y = fmaf(lane_value(L.w3, j), lane_value(h2, j), y);
  return y;
}

// The learned rule up to the network, for a pair at distance d (d2 = d^2 >
// 0) with R_A + R_B <= theta_max d.  e_A, e_B are the multipole estimates
// (times d^6), rho the larger of e/(eps s d^6) over the two cells.  rho <= 1/4
// accepts, rho > 2 opens (both in the product form of the multipole walk,
// eps scaled by a power of two).  In between, for pairs with N_A N_B >=
// min_work whose features lie in the training range [lo, hi], the network
// decides: it predicts log2 of the ratio of the method's error to the
// estimate, and the pair is accepted when rho times that ratio is at most 1
// (prediction <= thr = -plog2 rho).  Other pairs in the band take the
// multipole decision rho <= 1.
// Returns 1 (accept), 0 (open) or 2 (ask the network, with f and thr set).
enum : int { kLrnOpen = 0, kLrnAccept = 1, kLrnAsk = 2 };

__device__ inline int learned_gate(const float* P, double eps, int64_t min_work, double d, double d2,
                                   const PairSide& A, const PairSide& B, float f[kFeat], float* thr) {
  const double d6 = (d2 * d2) * d2;
  const double ea = multipole_bracket(A.R, B.R, B.k2, B.k3, d) * B.M;
  const double eb = multipole_bracket(B.R, A.R, A.k2, A.k3, d) * A.M;
  const double lo = kGateLo * eps, hi = kGateHi * eps;
  if (ea <= (lo * A.s) * d6 && eb <= (lo * B.s) * d6) return kLrnAccept;
  if (!(ea <= (hi * A.s) * d6 && eb <= (hi * B.s) * d6)) return kLrnOpen;
  const int plain = ea <= (eps * A.s) * d6 && eb <= (eps * B.s) * d6 ? kLrnAccept : kLrnOpen;
  if ((int64_t)A.n * (int64_t)B.n < min_work) return plain;
  pair_features(d, A, B, f);
  bool in = true;
#pragma unroll
  for (int i = 0; i < kFeat; ++i) in = in && (f[i] >= P[kLo + i] && f[i] <= P[kHi + i]);
  if (!in) return plain;
  const double ra = ea / ((eps * A.s) * d6), rb = eb / ((eps * B.s) * d6);
  const double rho = ra > rb ? ra : rb;
  *thr = (float)(-plog2(rho));
  return kLrnAsk;
}

}  // namespace amfmm
