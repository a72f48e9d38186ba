// Learned pair selection on the GPU: pair features and error labels from the
// method's own pair evaluation against direct sums, FP32 inference, and
// training (forward and backward of the pinball loss, Adam).
//
// Training runs 64 rows per workgroup (four waves, 16 rows each).  The hidden
// layer product H1 W2^T is a BF16 matrix-core product with FP32 accumulation
// (v_mfma_f32_16x16x16bf16); the two backward products (dH1 = dZ2 W2 and the
// weight gradient dZ2^T H1) are FP32 matrix-core products
// (v_mfma_f32_16x16x4f32), so gradients carry FP32 precision.  The small
// layers (8 inputs, 1 output) run on the vector units.  Each workgroup
// writes its partial gradient; a second kernel sums the partials in a fixed
// order, so results do not depend on scheduling.
#include <cmath>

#include "device_math.h"
#include "internal.h"
#include "learned.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;
constexpr int kLabelSample = 64;  // sampled particles per cell for a label
constexpr int kRows = 64;         // training rows per workgroup
constexpr int kLd = kHid + 1;     // LDS row stride (floats) of the 64-wide tiles

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double centre_distance(const double4& a, const double4& b) {
  const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return sqrt((dx * dx + dy * dy) + dz * dz);
}

// a cell's side of a pair (no field scale: features and labels do not use it)
__device__ inline PairSide side_of(const double4& g, const double* mo, int32_t n) {
  return PairSide{g.w, mo[0], norm_level(traceless_norm2(mo + 1), mo[0], g.w, 2),
                  norm_level(traceless_norm3(mo + 7), mo[0], g.w, 3), n, 0.0};
}

__global__ void __launch_bounds__(kBS) k_pair_features(int64_t np, const int32_t* __restrict__ pairs, int32_t nc,
                                                       const double4* __restrict__ geo, const double* __restrict__ mom,
                                                       const int32_t* __restrict__ cnt, float* __restrict__ feats) {
  const int64_t k = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (k >= np) return;
  const int32_t a = pairs[2 * k], b = pairs[2 * k + 1];
  if (a < 0 || a >= nc || b < 0 || b >= nc) {  // not a cell of the tree
#pragma unroll
    for (int i = 0; i < kFeat; ++i) feats[kFeat * k + i] = __builtin_nanf("");
    return;
  }
  const double4 ga = geo[a], gb = geo[b];
  const PairSide A = side_of(ga, mom + (int64_t)a * kMom, cnt[a]);
  const PairSide B = side_of(gb, mom + (int64_t)b * kMom, cnt[b]);
  float f[kFeat];
  pair_features(centre_distance(ga, gb), A, B, f);
#pragma unroll
  for (int i = 0; i < kFeat; ++i) feats[kFeat * k + i] = f[i];
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// One wave per pair.  For each cell T of the pair (the other S): the local
// coefficients of the pair alone about Z_T (as the far field computes them,
// with the correction of the variant), evaluated at up to 64 particles of T,
// against the direct sum over S's particles; the largest error over those
// particles, divided by the multipole estimate of the error on T.  The
// label is log2 of the larger ratio of the two cells (cells whose estimate
// is zero, point masses, are exact and left out; -inf when both are).
template <int VARIANT>
__global__ void __launch_bounds__(kBS) k_pair_labels(int64_t np, const int32_t* __restrict__ pairs, int32_t nc,
                                                     const double4* __restrict__ geo, const double* __restrict__ mom,
                                                     const int32_t* __restrict__ beg, const int32_t* __restrict__ cnt,
                                                     const double4* __restrict__ pos, double* __restrict__ labels) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (kBS / 64) + (threadIdx.x >> 6);
  if (k >= np) return;
  const int32_t pa = pairs[2 * k], pb = pairs[2 * k + 1];
  if (pa < 0 || pa >= nc || pb < 0 || pb >= nc) {  // not a cell of the tree (wave-uniform)
    if (lane == 0) labels[k] = __builtin_nan("");
    return;
  }
  const double d = centre_distance(geo[pa], geo[pb]);
  const double d2 = d * d, d6 = (d2 * d2) * d2;
  double worst = -INFINITY;
  for (int side = 0; side < 2; ++side) {
    const int32_t T = side ? pb : pa, Sc = side ? pa : pb;
    const double4 gt = geo[T], gs = geo[Sc];
    const double* mt = mom + (int64_t)T * kMom;
    const double* ms = mom + (int64_t)Sc * kMom;
    const double R[3] = {gt.x - gs.x, gt.y - gs.y, gt.z - gs.z};
    double L[kLoc];
#pragma unroll
    for (int u = 0; u < kLoc; ++u) L[u] = 0.0;
    const double Q2[6] = {ms[1], ms[2], ms[3], ms[4], ms[5], ms[6]};
    far_coeffs<double>(R, ms[0], Q2, L, 0.0);
    if (VARIANT != AMFMM_UC) {
      double OX[10], O3[10], F[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 10; ++u) {
        OX[u] = mt[7 + u];
        O3[u] = ms[7 + u];
      }
      far_correction<VARIANT>(R, mt[0], OX, ms[0], O3, F, 0.0);
      const double cf = -1.0 / (6.0 * mt[0]);
#pragma unroll
      for (int i = 0; i < 3; ++i) L[20 + i] = cf * F[i];
    }
    const int32_t nT = cnt[T], bS = beg[Sc], nS = cnt[Sc];
    const int ns = nT < kLabelSample ? nT : kLabelSample;
    double E = 0.0;
    if (lane < ns) {
      const int64_t p = beg[T] + ((int64_t)lane * nT) / ns;
      const double4 P = pos[p];
      const double x[3] = {P.x - gt.x, P.y - gt.y, P.z - gt.z};
      double g[3], phi;
      eval_local(L, x, g, phi);
      double gd[3] = {0.0, 0.0, 0.0};
      for (int32_t j = bS; j < bS + nS; ++j) {
        const double4 q = pos[j];
        const double dx = q.x - P.x, dy = q.y - P.y, dz = q.z - P.z;
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const double r3 = r2 * sqrt(r2);
        gd[0] += q.w * dx / r3;
        gd[1] += q.w * dy / r3;
        gd[2] += q.w * dz / r3;
      }
      const double ex = g[0] - gd[0], ey = g[1] - gd[1], ez = g[2] - gd[2];
      E = sqrt((ex * ex + ey * ey) + ez * ez);
    }
    E = wave_max(E);
    const PairSide pt = side_of(gt, mt, nT), ps = side_of(gs, ms, nS);
    const double est = multipole_bracket(pt.R, ps.R, ps.k2, ps.k3, d) * ps.M / d6;
    if (est > 0.0) worst = fmax(worst, E / est);
  }
  if (lane == 0) labels[k] = worst > 0.0 ? log2(worst) : -INFINITY;
}

// weights (W1, W2, w3) rounded to BF16; biases, normalisation, range copied
__global__ void __launch_bounds__(kBS) k_round_model(const float* __restrict__ in, float* __restrict__ out) {
  const int i = blockIdx.x * kBS + threadIdx.x;
  if (i >= AMFMM_MLP_MODEL) return;
  const bool weight = (i >= kW1 && i < kB1) || (i >= kW2 && i < kB2) || (i >= kW3 && i < kB3);
  out[i] = weight ? bf16r(in[i]) : in[i];
}

__global__ void __launch_bounds__(kBS) k_mlp_predict(int64_t n, const float* __restrict__ P,
                                                     const float* __restrict__ feats, float* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (r >= n) return;
  float f[kFeat];
#pragma unroll
  for (int i = 0; i < kFeat; ++i) f[i] = feats[kFeat * r + i];
  y[r] = mlp_infer(P, f);
}

__device__ inline short bf16_bits(float v) { return (short)(__builtin_bit_cast(uint32_t, v) >> 16); }

// Forward and backward of rows [blk*64, blk*64+64) of a batch of B rows; batch
// row i is data row (off + i) mod n.  Writes this workgroup's partial
// gradient (AMFMM_MLP_PARAMS floats) and partial loss.  LDS tiles are reused:
// dL/dz2 overwrites H2 and dL/dz1 overwrites H1 once they are no longer read.
__global__ void __launch_bounds__(kBS) k_mlp_step(int64_t n, int64_t off, int64_t B, const float* __restrict__ feats,
                                                  const float* __restrict__ labels, const float* __restrict__ P,
                                                  float tau, float invB, float* __restrict__ part,
                                                  float* __restrict__ lpart) {
  __shared__ float Xs[kRows][kFeat];
  __shared__ float H1[kRows][kLd];  // hidden 1, later dL/dz1
  __shared__ float H2[kRows][kLd];  // hidden 2, later dL/dz2
  __shared__ float W2[kHid][kLd];   // BF16-rounded, W2[k][j]
  __shared__ float dys[kRows], ls[kRows];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  float* g = part + (int64_t)blockIdx.x * AMFMM_MLP_PARAMS;
  for (int idx = t; idx < kRows * kFeat; idx += kBS) {
    const int r = idx / kFeat, i = idx % kFeat;
    float f = 0.0f;
    if (r0 + r < B) f = feats[kFeat * ((off + r0 + r) % n) + i];
    Xs[r][i] = bf16r(fmaf(f, P[kNA + i], P[kNB + i]));
  }
  for (int idx = t; idx < kHid * kHid; idx += kBS) W2[idx / kHid][idx % kHid] = bf16r(P[kW2 + idx]);
  __syncthreads();
  // layer 1 (vector units)
  for (int idx = t; idx < kRows * kHid; idx += kBS) {
    const int r = idx / kHid, j = idx % kHid;
    float s = P[kB1 + j];
#pragma unroll
    for (int i = 0; i < kFeat; ++i) s = fmaf(bf16r(P[kW1 + kFeat * j + i]), Xs[r][i], s);
    H1[r][j] = bf16r(s > 0.0f ? s : 0.0f);
  }
  __syncthreads();
  // layer 2: Z2 = H1 W2^T, BF16 products, FP32 accumulation; wave w takes rows
  // 16w..16w+15.  Operand layout of the 16x16x16 product: lane l supplies
  // A[l%16][4(l/16)+v] and B[4(l/16)+v][l%16]; it receives D[4(l/16)+v][l%16].
  for (int ct = 0; ct < 4; ++ct) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int ks = 0; ks < 4; ++ks) {
      bf16x4 a, b;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        a[v] = bf16_bits(H1[16 * w + lr][16 * ks + 4 * lq + v]);
        b[v] = bf16_bits(W2[16 * ct + lr][16 * ks + 4 * lq + v]);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * w + 4 * lq + v, k = 16 * ct + lr;
      const float z = acc[v] + P[kB2 + k];
      H2[r][k] = bf16r(z > 0.0f ? z : 0.0f);
    }
  }
  __syncthreads();
  // output, loss and its derivative
  if (t < kRows) {
    float y = P[kB3];
    for (int k = 0; k < kHid; ++k) y = fmaf(bf16r(P[kW3 + k]), H2[t][k], y);
    float dy = 0.0f, l = 0.0f;
    if (r0 + t < B) {
      const float res = labels[(off + r0 + t) % n] - y;
      l = res < 0.0f ? (tau - 1.0f) * res : tau * res;
      dy = (res < 0.0f ? 1.0f - tau : -tau) * invB;
    }
    dys[t] = dy;
    ls[t] = l;
  }
  __syncthreads();
  // gradients of the output layer (read H2 before it is overwritten)
  if (t >= 128 && t < 192) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s = fmaf(dys[r], H2[r][t - 128], s);
    g[kW3 + t - 128] = s;
  } else if (t == 192) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += dys[r];
    g[kB3] = s;
  } else if (t == 193) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += ls[r];
    lpart[blockIdx.x] = s;
  }
  __syncthreads();
  // dL/dz2 in place of H2 (each element from its own value)
  for (int idx = t; idx < kRows * kHid; idx += kBS) {
    const int r = idx / kHid, k = idx % kHid;
    H2[r][k] = H2[r][k] > 0.0f ? dys[r] * bf16r(P[kW3 + k]) : 0.0f;
  }
  __syncthreads();
  // dW2[k][j] = sum_r dz2[r][k] H1[r][j] (FP32 products); wave w takes k =
  // 16w..16w+15.  Operand layout of the 16x16x4 product: lane l supplies
  // A[l%16][l/16] and B[l/16][l%16]; it receives D[4(l/16)+v][l%16].
  for (int ct = 0; ct < 4; ++ct) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int ks = 0; ks < kRows / 4; ++ks)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(H2[4 * ks + lq][16 * w + lr], H1[4 * ks + lq][16 * ct + lr], acc,
                                                 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) g[kW2 + kHid * (16 * w + 4 * lq + v) + 16 * ct + lr] = acc[v];
  }
  if (t >= 64 && t < 128) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += H2[r][t - 64];
    g[kB2 + t - 64] = s;
  }
  __syncthreads();
  // dz1 = (dz2 W2) masked by the ReLU, in place of H1 (element by element)
  for (int ct = 0; ct < 4; ++ct) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int ks = 0; ks < kHid / 4; ++ks)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(H2[16 * w + lr][4 * ks + lq], W2[4 * ks + lq][16 * ct + lr], acc,
                                                 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * w + 4 * lq + v, j = 16 * ct + lr;
      H1[r][j] = H1[r][j] > 0.0f ? acc[v] : 0.0f;
    }
  }
  __syncthreads();
  // dW1[j][i] = sum_r dz1[r][j] X[r][i]: thread t takes j = t/4, i = 2(t%4), +1
  {
    const int j = t >> 2, i0 = 2 * (t & 3);
    float s0 = 0.0f, s1 = 0.0f;
    for (int r = 0; r < kRows; ++r) {
      s0 = fmaf(H1[r][j], Xs[r][i0], s0);
      s1 = fmaf(H1[r][j], Xs[r][i0 + 1], s1);
    }
    g[kW1 + kFeat * j + i0] = s0;
    g[kW1 + kFeat * j + i0 + 1] = s1;
  }
  if (t < 64) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += H1[r][t];
    g[kB1 + t] = s;
  }
}

// grad[p] = sum over workgroups of the partials, in workgroup order; the
// loss (times invB) in grad[AMFMM_MLP_PARAMS]
__global__ void __launch_bounds__(kBS) k_mlp_reduce(int32_t nblk, const float* __restrict__ part,
                                                    const float* __restrict__ lpart, float invB,
                                                    float* __restrict__ grad) {
  const int p = blockIdx.x * kBS + threadIdx.x;
  if (p > AMFMM_MLP_PARAMS) return;
  float s = 0.0f;
  if (p < AMFMM_MLP_PARAMS) {
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * AMFMM_MLP_PARAMS + p];
  } else {
    for (int b = 0; b < nblk; ++b) s += lpart[b];
    s *= invB;
  }
  grad[p] = s;
}

// Adam (Kingma & Ba 2015) with bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ void __launch_bounds__(kBS) k_mlp_adam(float* __restrict__ P, const float* __restrict__ grad,
                                                  float* __restrict__ m, float* __restrict__ v, double lr, double b1,
                                                  double b2, double eps, double c1, double c2) {
  const int p = blockIdx.x * kBS + threadIdx.x;
  if (p >= AMFMM_MLP_PARAMS) return;
  const double g = grad[p];
  const double mi = b1 * m[p] + (1.0 - b1) * g;
  const double vi = b2 * v[p] + (1.0 - b2) * g * g;
  m[p] = (float)mi;
  v[p] = (float)vi;
  P[p] = (float)(P[p] - lr * (mi / c1) / (sqrt(vi / c2) + eps));
}

void check_pairs(Ctx& c) {
  if (!c.have_moments) throw Error(AMFMM_E_STATE, "pair features and labels need amfmm_compute_moments");
}

// one gradient evaluation over batch rows off .. off+B-1 (mod n); the result
// (AMFMM_MLP_PARAMS gradients, then the loss) in c.mlp_grad
float* mlp_step(Ctx& c, int64_t n, int64_t off, int64_t B, const float* feats, const float* labels, const float* P,
                double tau) {
  const int32_t nblk = (int32_t)((B + kRows - 1) / kRows);
  float* part = (float*)ensure(c, c.mlp_part, sizeof(float) * ((size_t)nblk * AMFMM_MLP_PARAMS + nblk));
  float* lpart = part + (size_t)nblk * AMFMM_MLP_PARAMS;
  float* grad = (float*)ensure(c, c.mlp_grad, sizeof(float) * (AMFMM_MLP_PARAMS + 1));
  const float invB = (float)(1.0 / (double)B);
  hipLaunchKernelGGL(k_mlp_step, dim3(nblk), dim3(kBS), 0, c.stream, n, off, B, feats, labels, P, (float)tau, invB,
                     part, lpart);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks_for(AMFMM_MLP_PARAMS + 1, kBS)), dim3(kBS), 0, c.stream, nblk,
                     (const float*)part, (const float*)lpart, invB, grad);
  AMFMM_HIP(hipGetLastError());
  return grad;
}

}  // namespace

void compute_pair_features(Ctx& c, int64_t np, const int32_t* pairs, float* feats) {
  check_pairs(c);
  if (np <= 0) return;
  hipLaunchKernelGGL(k_pair_features, dim3((unsigned)((np + kBS - 1) / kBS)), dim3(kBS), 0, c.stream, np, pairs,
                     (int32_t)c.ncells, (const double4*)c.geo.p, (const double*)c.mom.p, as<int32_t>(c.c_count), feats);
  AMFMM_HIP(hipGetLastError());
}

void compute_pair_labels(Ctx& c, int variant, int64_t np, const int32_t* pairs, double* labels) {
  check_pairs(c);
  if (np <= 0) return;
  const dim3 grid((unsigned)((np + 3) / 4));
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(kBS), 0, c.stream, np, pairs, (int32_t)c.ncells, (const double4*)c.geo.p,
                       (const double*)c.mom.p, as<int32_t>(c.c_begin), as<int32_t>(c.c_count),
                       (const double4*)c.pos4.p, labels);
  };
  if (variant == AMFMM_UC) launch(k_pair_labels<AMFMM_UC>);
  else if (variant == AMFMM_TC) launch(k_pair_labels<AMFMM_TC>);
  else launch(k_pair_labels<AMFMM_TCO>);
  AMFMM_HIP(hipGetLastError());
}

void round_model(Ctx& c, const float* in, float* out) {
  hipLaunchKernelGGL(k_round_model, dim3(blocks_for(AMFMM_MLP_MODEL, kBS)), dim3(kBS), 0, c.stream, in, out);
  AMFMM_HIP(hipGetLastError());
}

void mlp_predict(Ctx& c, int64_t n, const float* model, const float* feats, float* y) {
  if (n <= 0) return;
  float* P = (float*)ensure(c, c.mlp_tmp, sizeof(float) * AMFMM_MLP_MODEL);
  round_model(c, model, P);
  hipLaunchKernelGGL(k_mlp_predict, dim3((unsigned)((n + kBS - 1) / kBS)), dim3(kBS), 0, c.stream, n,
                     (const float*)P, feats, y);
  AMFMM_HIP(hipGetLastError());
}

double mlp_grad(Ctx& c, int64_t n, const float* model, const float* feats, const float* labels, double tau,
                float* grad) {
  const float* g = mlp_step(c, n, 0, n, feats, labels, model, tau);
  AMFMM_HIP(hipMemcpyAsync(grad, g, sizeof(float) * AMFMM_MLP_PARAMS, hipMemcpyDeviceToDevice, c.stream));
  float loss = 0.0f;
  AMFMM_HIP(hipMemcpyAsync(&loss, g + AMFMM_MLP_PARAMS, sizeof(float), hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
  return loss;
}

double mlp_train(Ctx& c, int64_t n, const float* feats, const float* labels, float* model, float* am, float* av,
                 int64_t step0, int32_t steps, int32_t batch, double lr, double tau) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const float* g = nullptr;
  for (int32_t s = 0; s < steps; ++s) {
    const int64_t st = step0 + s;
    g = mlp_step(c, n, (st * (int64_t)batch) % n, batch, feats, labels, model, tau);
    const double c1 = 1.0 - std::pow(b1, (double)(st + 1)), c2 = 1.0 - std::pow(b2, (double)(st + 1));
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(AMFMM_MLP_PARAMS, kBS)), dim3(kBS), 0, c.stream, model, g, am, av,
                       lr, b1, b2, eps, c1, c2);
    AMFMM_HIP(hipGetLastError());
  }
  float loss = 0.0f;
  if (g) {
    AMFMM_HIP(hipMemcpyAsync(&loss, g + AMFMM_MLP_PARAMS, sizeof(float), hipMemcpyDeviceToHost, c.stream));
    AMFMM_HIP(hipStreamSynchronize(c.stream));
  }
  return loss;
}

}  // namespace amfmm
