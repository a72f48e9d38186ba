// The appendix's general expansion order on the GPU, P = 4, in FP64: the
// Green's function G(R + x - y) (R = Z_X - Z_Y, x and y the offsets from the
// two centres of mass) expanded to order P in both offsets, and the
// corrective force of that order that cancels each pair's torque.
//
// Multi-indices alpha = (a, b, c) stand for index tuples (x^alpha = x^a y^b
// z^c, alpha! = a! b! c!).  Per cell: moments M_alpha = sum mu x^alpha about
// the centre of mass (|alpha| <= P, leaves from their particles, parents by
// shifting their children's); per target cell X the local coefficients
//   L_alpha = sum_Y sum_beta (-1)^|beta| / beta! D_(alpha+beta)(R) M_Y,beta
// over |alpha| + |beta| <= P, dipole terms (|beta| = 1) and the constant
// |alpha| = 0, |beta| = P dropped (as at P = 3), and with the correction
// (TC) the acceleration g_c = F_c / M_X,
//   F_c,k = -sum_n (-1)^n sum_{|alpha| = P-n, |beta| = n} M_X,alpha M_Y,beta
//           D_(alpha+beta+e_k)(R) / (alpha! beta!)
// (evaluated as -sum_gamma Q_gamma D_(gamma+e_k), Q_gamma the sum of the
// moment products with alpha + beta = gamma)
// (at P = 3 this is eq. 7; the mirrored pair gives -F_c, since D of odd order
// changes sign with R).  The derivatives D_gamma of g(R) = -1/sqrt(R^2 +
// eps^2) come from f_k = (1/R d/dR)^k g by pairing equal indices.  Push-down
// shifts L to each child's centre; at a particle the acceleration is minus
// the gradient of sum_alpha x^alpha / alpha! L_alpha, plus g_c.
//
// Evaluated per directed pair (each target its own sources), one wave per
// target cell, lanes over its sources, fixed-order butterfly sums: the same
// organisation as the order-3 far field.
#include "device_math.h"
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / 64;
constexpr int kP = 4;

// multi-indices of order <= n
constexpr int num_mi(int n) { return (n + 1) * (n + 2) * (n + 3) / 6; }
constexpr int kNL = num_mi(kP);      // moments and local coefficients
constexpr int kND = num_mi(kP + 1);  // derivatives (the correction needs order P + 1)
static_assert(kNL + 3 <= kLocGen, "local record");

// graded enumeration: order n, then a from n down, then b from n - a down
struct MITable {
  int a[kND], b[kND], c[kND], n[kND];
  double fact[kND];
};
constexpr MITable make_mi() {
  MITable t{};
  int k = 0;
  for (int n = 0; n <= kP + 1; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b;
        t.a[k] = a;
        t.b[k] = b;
        t.c[k] = c;
        t.n[k] = n;
        double f = 1.0;
        for (int i = 2; i <= a; ++i) f *= i;
        for (int i = 2; i <= b; ++i) f *= i;
        for (int i = 2; i <= c; ++i) f *= i;
        t.fact[k] = f;
        ++k;
      }
  return t;
}
constexpr MITable kMI = make_mi();

__host__ __device__ constexpr int mi_id(int a, int b, int c) {
  return num_mi(a + b + c - 1) + (b + c) * (b + c + 1) / 2 + c;
}
static_assert(mi_id(0, 0, 0) == 0 && mi_id(0, 0, 1) == 3 && mi_id(2, 0, 0) == 4 && mi_id(0, 0, 5) == kND - 1,
              "multi-index numbering");

// ways to pair p of g equal indices: g! / (p! (g - 2p)! 2^p)
constexpr double pair_ways(int g, int p) {
  double v = 1.0;
  for (int i = 2; i <= g; ++i) v *= i;
  for (int i = 2; i <= p; ++i) v /= i;
  for (int i = 2; i <= g - 2 * p; ++i) v /= i;
  for (int i = 0; i < p; ++i) v /= 2.0;
  return v;
}

// binomial coefficient
constexpr double binom(int n, int k) {
  double v = 1.0;
  for (int i = 1; i <= k; ++i) v = v * (n - k + i) / i;
  return v;
}

// The terms of the far field, the correction and the moment shift, listed
// once at compile time (every index a constant after unrolling).
// local coefficients: L[al] += coef D[g] M_source[be], coef = (-1)^|be| / be!
struct Term {
  int al, be, g;
  double coef;
};
constexpr bool local_term(int al, int be) {
  return kMI.n[al] + kMI.n[be] <= kP && kMI.n[be] != 1 && !(kMI.n[al] == 0 && kMI.n[be] == kP);
}
constexpr int count_local() {
  int k = 0;
  for (int al = 0; al < kNL; ++al)
    for (int be = 0; be < kNL; ++be) k += local_term(al, be);
  return k;
}
constexpr int kNLocal = count_local();
struct LocalTerms {
  Term t[kNLocal];
};
// (source moment outer: each is loaded once and used at once)
constexpr LocalTerms make_local() {
  LocalTerms r{};
  int k = 0;
  for (int be = 0; be < kNL; ++be)
    for (int al = 0; al < kNL; ++al)
      if (local_term(al, be)) {
        const int sb = kMI.n[be] % 2 ? -1 : 1;
        r.t[k++] = {al, be, mi_id(kMI.a[al] + kMI.a[be], kMI.b[al] + kMI.b[be], kMI.c[al] + kMI.c[be]),
                    sb / kMI.fact[be]};
      }
  return r;
}
constexpr LocalTerms kLocal = make_local();

// one value per multi-index; kSign: (-1)^|be| / be!, the factor of the source
// moment be in every term above
struct PerIndex {
  double c[kNL];
};
constexpr PerIndex make_signs() {
  PerIndex r{};
  for (int be = 0; be < kNL; ++be) r.c[be] = (kMI.n[be] % 2 ? -1.0 : 1.0) / kMI.fact[be];
  return r;
}
constexpr PerIndex kSign = make_signs();
// 1 / al!
constexpr PerIndex make_inv_fact() {
  PerIndex r{};
  for (int al = 0; al < kNL; ++al) r.c[al] = 1.0 / kMI.fact[al];
  return r;
}
constexpr PerIndex kInvFact = make_inv_fact();
// lanes of the evaluation kernel per leaf
constexpr int kL2PLanes = 8;
constexpr bool local_coef_check() {
  for (int i = 0; i < kNLocal; ++i)
    if (kLocal.t[i].coef != kSign.c[kLocal.t[i].be]) return false;
  return true;
}
static_assert(local_coef_check(), "local term coefficients are (-1)^|be| / be!");

// correction: the moment products gathered into one order-P tensor,
// Q[g] += coef M_target[al] M_source[be] (g = al + be), coef = (-1)^|be| /
// (al! be!), over |al| + |be| = P with neither a dipole; then s_k = sum_g
// Q[g] D[g + e_k]
constexpr bool corr_term(int al, int be) {
  return kMI.n[al] + kMI.n[be] == kP && kMI.n[al] != 1 && kMI.n[be] != 1;
}
constexpr int count_corr() {
  int k = 0;
  for (int al = 0; al < kNL; ++al)
    for (int be = 0; be < kNL; ++be) k += corr_term(al, be);
  return k;
}
constexpr int kNCorr = count_corr();
struct CorrTerm {
  int al, be, q;
  double coef;
};
struct CorrTerms {
  CorrTerm t[kNCorr];
};
// (source moment outer, as for the local terms)
constexpr CorrTerms make_corr() {
  CorrTerms r{};
  int k = 0;
  for (int be = 0; be < kNL; ++be)
    for (int al = 0; al < kNL; ++al)
      if (corr_term(al, be)) {
        const int a = kMI.a[al] + kMI.a[be], b = kMI.b[al] + kMI.b[be], c = kMI.c[al] + kMI.c[be];
        const int sb = kMI.n[be] % 2 ? -1 : 1;
        r.t[k++] = {al, be, mi_id(a, b, c) - num_mi(kP - 1), sb / (kMI.fact[al] * kMI.fact[be])};
      }
  return r;
}
constexpr CorrTerms kCorr = make_corr();

// moment shift: M_parent[be] += coef M_child[ga] s^[d], coef = C(be, ga)
constexpr bool shift_term(int be, int ga) {
  return kMI.a[ga] <= kMI.a[be] && kMI.b[ga] <= kMI.b[be] && kMI.c[ga] <= kMI.c[be];
}
constexpr int count_shift() {
  int k = 0;
  for (int be = 0; be < kNL; ++be)
    for (int ga = 0; ga < kNL; ++ga) k += shift_term(be, ga);
  return k;
}
constexpr int kNShift = count_shift();
struct ShiftTerms {
  Term t[kNShift];  // al: the parent's moment, be: the child's, g: the power of s
};
constexpr ShiftTerms make_shift() {
  ShiftTerms r{};
  int k = 0;
  for (int be = 0; be < kNL; ++be)
    for (int ga = 0; ga < kNL; ++ga)
      if (shift_term(be, ga))
        r.t[k++] = {be, ga, mi_id(kMI.a[be] - kMI.a[ga], kMI.b[be] - kMI.b[ga], kMI.c[be] - kMI.c[ga]),
                    binom(kMI.a[be], kMI.a[ga]) * binom(kMI.b[be], kMI.b[ga]) * binom(kMI.c[be], kMI.c[ga])};
  return r;
}
constexpr ShiftTerms kShift = make_shift();
static_assert(kNLocal == 135 && kNCorr == 66, "term counts at P = 4");

// Derivative terms: D_gamma = sum over the pairings (p, q, r pairs among the
// x, y and z indices of gamma) of f_(|gamma| - p - q - r) times the number of
// such pairings times R^(gamma - 2 (p, q, r)).
struct DerivTerm {
  int g, f, e0, e1, e2;
  double coef;
};
constexpr int count_deriv() {
  int k = 0;
  for (int g = 0; g < kND; ++g) k += (kMI.a[g] / 2 + 1) * (kMI.b[g] / 2 + 1) * (kMI.c[g] / 2 + 1);
  return k;
}
constexpr int kNDeriv = count_deriv();
struct DerivTerms {
  DerivTerm t[kNDeriv];
};
constexpr DerivTerms make_deriv() {
  DerivTerms r{};
  int k = 0;
  for (int g = 0; g < kND; ++g)
    for (int p = 0; 2 * p <= kMI.a[g]; ++p)
      for (int q = 0; 2 * q <= kMI.b[g]; ++q)
        for (int u = 0; 2 * u <= kMI.c[g]; ++u)
          r.t[k++] = {g, kMI.n[g] - p - q - u, kMI.a[g] - 2 * p, kMI.b[g] - 2 * q, kMI.c[g] - 2 * u,
                      pair_ways(kMI.a[g], p) * pair_ways(kMI.b[g], q) * pair_ways(kMI.c[g], u)};
  return r;
}
constexpr DerivTerms kDeriv = make_deriv();

// The radial factors f_k = (1/R d/dR)^k g of g = -1/sqrt(R^2 + eps^2),
// f_0 = -1/sqrt(s), f_(k+1) = -(2k+1) f_k / s (one division, then 1/s =
// f_0^2), and the powers R_i^k, k <= P + 1
__device__ inline void radial_and_powers(const double R[3], double eps2, double f[kP + 2], double pw[3][kP + 2]) {
  const double s = ((R[0] * R[0] + R[1] * R[1]) + R[2] * R[2]) + eps2;
  f[0] = -1.0 / sqrt(s);
  const double is = f[0] * f[0];
#pragma unroll
  for (int k = 0; k <= kP; ++k) f[k + 1] = (-(2.0 * k + 1.0) * f[k]) * is;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    pw[i][0] = 1.0;
#pragma unroll
    for (int k = 0; k <= kP; ++k) pw[i][k + 1] = pw[i][k] * R[i];
  }
}

// D_gamma(R) for LO <= |gamma| <= HI (entries of other orders untouched)
template <int LO, int HI>
__device__ inline void derivatives(const double R[3], double eps2, double D[kND]) {
  double f[kP + 2], pw[3][kP + 2];
  radial_and_powers(R, eps2, f, pw);
#pragma unroll
  for (int g = num_mi(LO - 1); g < num_mi(HI); ++g) D[g] = 0.0;
#pragma unroll
  for (int i = 0; i < kNDeriv; ++i) {
    const DerivTerm& t = kDeriv.t[i];
    if (kMI.n[t.g] < LO || kMI.n[t.g] > HI) continue;
    D[t.g] = fma(f[t.f], t.coef * ((pw[0][t.e0] * pw[1][t.e1]) * pw[2][t.e2]), D[t.g]);
  }
}

// push-down shift: L'[al] += L[g] d^[ga] / ga!, g = al + ga, |al| + |ga| <= P
constexpr int count_l2l() {
  int k = 0;
  for (int al = 0; al < kNL; ++al)
    for (int ga = 0; ga < kNL; ++ga) k += kMI.n[al] + kMI.n[ga] <= kP;
  return k;
}
constexpr int kNL2L = count_l2l();
struct L2LTerms {
  Term t[kNL2L];  // al: the child's coefficient, be: the power of d, g: the parent's coefficient
};
constexpr L2LTerms make_l2l() {
  L2LTerms r{};
  int k = 0;
  for (int al = 0; al < kNL; ++al)
    for (int ga = 0; ga < kNL; ++ga)
      if (kMI.n[al] + kMI.n[ga] <= kP)
        r.t[k++] = {al, ga, mi_id(kMI.a[al] + kMI.a[ga], kMI.b[al] + kMI.b[ga], kMI.c[al] + kMI.c[ga]),
                    1.0 / kMI.fact[ga]};
  return r;
}
constexpr L2LTerms kL2L = make_l2l();

// x^alpha, |alpha| <= P
__device__ inline void monomials(const double x[3], double X[kNL]) {
  double pw[3][kP + 1];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    pw[i][0] = 1.0;
#pragma unroll
    for (int k = 0; k < kP; ++k) pw[i][k + 1] = pw[i][k] * x[i];
  }
#pragma unroll
  for (int g = 0; g < kNL; ++g) X[g] = (pw[0][kMI.a[g]] * pw[1][kMI.b[g]]) * pw[2][kMI.c[g]];
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// leaf moments from the particles, in key order (one thread per leaf)
__global__ void __launch_bounds__(kBS) k_mono_leaves(const double4* __restrict__ pos,
                                                     const int32_t* __restrict__ leaves, int32_t nleaves,
                                                     const int32_t* __restrict__ beg, const int32_t* __restrict__ cnt,
                                                     const double4* __restrict__ geo, double* __restrict__ mono) {
  const int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nleaves) return;
  const int32_t c = leaves[i];
  const double4 z = geo[c];
  double acc[kNL];
#pragma unroll
  for (int g = 0; g < kNL; ++g) acc[g] = 0.0;
  for (int32_t p = beg[c]; p < beg[c] + cnt[c]; ++p) {
    const double4 q = pos[p];
    const double x[3] = {q.x - z.x, q.y - z.y, q.z - z.z};
    double X[kNL];
    monomials(x, X);
#pragma unroll
    for (int g = 0; g < kNL; ++g) acc[g] += q.w * X[g];
  }
  double* o = mono + (int64_t)c * kNL;
#pragma unroll
  for (int g = 0; g < kNL; ++g) o[g] = acc[g];
}

// parent moments: each child's shifted by s = Z_child - Z_parent,
// M_beta += sum_{gamma <= beta} C(beta, gamma) M_child,gamma s^(beta-gamma),
// children in octant order (one thread per parent)
__global__ void __launch_bounds__(kBS) k_mono_up(int32_t c0, int32_t nl, const int32_t* __restrict__ ch0,
                                                 const int32_t* __restrict__ nch, const double4* __restrict__ geo,
                                                 double* __restrict__ mono) {
  const int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  const int32_t c = c0 + i;
  if (nch[c] == 0) return;
  const double4 zp = geo[c];
  double acc[kNL];
#pragma unroll
  for (int g = 0; g < kNL; ++g) acc[g] = 0.0;
  for (int32_t k = ch0[c]; k < ch0[c] + nch[c]; ++k) {
    const double4 zc = geo[k];
    const double s[3] = {zc.x - zp.x, zc.y - zp.y, zc.z - zp.z};
    double S[kNL];
    monomials(s, S);
    const double* m = mono + (int64_t)k * kNL;
    double mc[kNL];
#pragma unroll
    for (int g = 0; g < kNL; ++g) mc[g] = m[g];
#pragma unroll
    for (int i = 0; i < kNShift; ++i) acc[kShift.t[i].al] += kShift.t[i].coef * mc[kShift.t[i].be] * S[kShift.t[i].g];
  }
  double* o = mono + (int64_t)c * kNL;
#pragma unroll
  for (int g = 0; g < kNL; ++g) o[g] = acc[g];
}

// Far field of one target cell per wave: its local coefficients (locg: kNL
// coefficients, then g_c, zero here: k_corr_order sets it for TC) and, for
// the order-3 kernels that run after it, zeros in its loc record (the
// evaluation at the particles adds this expansion separately).
__global__ void __launch_bounds__(kBS) k_far_order(int32_t c_lo, int32_t nc, const double4* __restrict__ geo,
                                                   const double* __restrict__ mono, const int64_t* __restrict__ fstart,
                                                   const int32_t* __restrict__ fcount, const int32_t* __restrict__ fsrc,
                                                   double* __restrict__ locg, double* __restrict__ loc, double eps2) {
  const int lane = threadIdx.x & 63;
  const int32_t Xi = uniform((int32_t)(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6)));
  if (Xi >= nc) return;
  const int32_t X = c_lo + Xi;
  const int32_t cnt = fcount[X];
  const int64_t st = fstart[X];
  const double4 gx = geo[X];
  double L[kNL];
#pragma unroll
  for (int g = 0; g < kNL; ++g) L[g] = 0.0;
  for (int64_t j = lane; j < cnt; j += 64) {
    const int32_t Y = fsrc[st + j];
    const double4 gy = geo[Y];
    const double* my = mono + (int64_t)Y * kNL;
    const double R[3] = {gx.x - gy.x, gx.y - gy.y, gx.z - gy.z};
    double D[kND];
    derivatives<0, kP>(R, eps2, D);
    // each source moment scaled once, then one fma per term
    double cm[kNL];
#pragma unroll
    for (int be = 0; be < kNL; ++be) cm[be] = kSign.c[be] * my[be];
#pragma unroll
    for (int i = 0; i < kNLocal; ++i)
      L[kLocal.t[i].al] = fma(D[kLocal.t[i].g], cm[kLocal.t[i].be], L[kLocal.t[i].al]);
  }
#pragma unroll
  for (int g = 0; g < kNL; ++g) L[g] = wave_sum(L[g]);
  if (lane == 0) {
    double* o = locg + (int64_t)X * kLocGen;
#pragma unroll
    for (int g = 0; g < kNL; ++g) o[g] = L[g];
    for (int u = kNL; u < kLocGen; ++u) o[u] = 0.0;
    double* z = loc + (int64_t)X * kLoc;
    for (int u = 0; u < kLoc; ++u) z[u] = 0.0;
  }
}

// The correction (TC) of one target cell per wave over the same sources:
// g_c = F_c / M_X into locg (after k_far_order).  Only the order-(P+1)
// derivatives and the moments of orders 0, 2 and P enter.
__global__ void __launch_bounds__(kBS) k_corr_order(int32_t c_lo, int32_t nc, const double4* __restrict__ geo,
                                                    const double* __restrict__ mono, const int64_t* __restrict__ fstart,
                                                    const int32_t* __restrict__ fcount, const int32_t* __restrict__ fsrc,
                                                    double* __restrict__ locg, double eps2) {
  constexpr int kNQ = num_mi(kP) - num_mi(kP - 1);  // order-P components
  const int lane = threadIdx.x & 63;
  const int32_t Xi = uniform((int32_t)(xcd_block(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6)));
  if (Xi >= nc) return;
  const int32_t X = c_lo + Xi;
  const int32_t cnt = fcount[X];
  const int64_t st = fstart[X];
  const double4 gx = geo[X];
  const double* mx = mono + (int64_t)X * kNL;
  double F[3] = {0.0, 0.0, 0.0};
  for (int64_t j = lane; j < cnt; j += 64) {
    const int32_t Y = fsrc[st + j];
    const double4 gy = geo[Y];
    const double* my = mono + (int64_t)Y * kNL;
    const double R[3] = {gx.x - gy.x, gx.y - gy.y, gx.z - gy.z};
    double Q[kNQ];
#pragma unroll
    for (int q = 0; q < kNQ; ++q) Q[q] = 0.0;
    // the target's moments stay in scalar registers (wave-uniform loads); the
    // constant goes with the source moment (products shared between terms)
#pragma unroll
    for (int i = 0; i < kNCorr; ++i)
      Q[kCorr.t[i].q] = fma(mx[kCorr.t[i].al], kCorr.t[i].coef * my[kCorr.t[i].be], Q[kCorr.t[i].q]);
    double D[kND];
    derivatives<kP + 1, kP + 1>(R, eps2, D);
#pragma unroll
    for (int q = 0; q < kNQ; ++q) {
      const int g = num_mi(kP - 1) + q;
      F[0] = fma(-Q[q], D[mi_id(kMI.a[g] + 1, kMI.b[g], kMI.c[g])], F[0]);
      F[1] = fma(-Q[q], D[mi_id(kMI.a[g], kMI.b[g] + 1, kMI.c[g])], F[1]);
      F[2] = fma(-Q[q], D[mi_id(kMI.a[g], kMI.b[g], kMI.c[g] + 1)], F[2]);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) F[k] = wave_sum(F[k]);
  if (lane == 0) {
    double* o = locg + (int64_t)X * kLocGen;
    const double MX = mx[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) o[kNL + k] = F[k] / MX;
  }
}

// locg[child] += the parent's expansion shifted to the child's centre,
// L'_alpha = sum_gamma L_(alpha+gamma) d^gamma / gamma!, d = Z_child - Z_parent;
// g_c adds (one thread per child)
__global__ void __launch_bounds__(kBS) k_l2l_order(int32_t c0, int32_t nl, const int32_t* __restrict__ par,
                                                   const double4* __restrict__ geo, double* __restrict__ locg) {
  const int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  const int32_t c = c0 + i;
  const int32_t P = par[c];
  const double4 gc = geo[c], gp = geo[P];
  const double d[3] = {gc.x - gp.x, gc.y - gp.y, gc.z - gp.z};
  double Dm[kNL];
  monomials(d, Dm);
  const double* L = locg + (int64_t)P * kLocGen;
  double* o = locg + (int64_t)c * kLocGen;
  double Lp[kNL], acc[kNL];
#pragma unroll
  for (int g = 0; g < kNL; ++g) {
    Lp[g] = L[g];
    acc[g] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < kNL2L; ++i) acc[kL2L.t[i].al] += Lp[kL2L.t[i].g] * (Dm[kL2L.t[i].be] * kL2L.t[i].coef);
#pragma unroll
  for (int g = 0; g < kNL; ++g) o[g] += acc[g];
#pragma unroll
  for (int k = 0; k < 3; ++k) o[kNL + k] += L[kNL + k];
}

// At every particle of the target leaves: G times minus the gradient of the
// leaf's expansion, plus g_c, added to the near field's outputs (caller
// order); the potential likewise (kL2PLanes lanes per leaf, over its particles).
// leaves == nullptr: the leaves among cells [c_lo, c_lo + count).
__global__ void __launch_bounds__(kBS) k_l2p_order(int32_t count, const int32_t* __restrict__ leaves, int32_t c_lo,
                                                   const int32_t* __restrict__ nch, const int32_t* __restrict__ beg,
                                                   const int32_t* __restrict__ cnt, const double4* __restrict__ pos,
                                                   const double4* __restrict__ geo, const double* __restrict__ locg,
                                                   const int32_t* __restrict__ perm, double G,
                                                   double* __restrict__ ax, double* __restrict__ ay,
                                                   double* __restrict__ az, double* __restrict__ pot) {
  // kL2PLanes lanes per leaf (leaves hold a few particles each)
  const int64_t li = ((int64_t)blockIdx.x * kBS + threadIdx.x) / kL2PLanes;
  const int sl = (int)(threadIdx.x % kL2PLanes);
  if (li >= count) return;
  const int32_t X = leaves ? leaves[li] : c_lo + (int32_t)li;
  if (!leaves && nch[X] != 0) return;
  const double4 z = geo[X];
  const double* L = locg + (int64_t)X * kLocGen;
  for (int32_t p = beg[X] + sl; p < beg[X] + cnt[X]; p += kL2PLanes) {
    const double4 q = pos[p];
    const double x[3] = {q.x - z.x, q.y - z.y, q.z - z.z};
    double Xm[kNL];
    monomials(x, Xm);
    // x^al / al!, the reciprocal factorials as constants
#pragma unroll
    for (int al = 0; al < kNL; ++al) Xm[al] *= kInvFact.c[al];
    double phi = 0.0;
#pragma unroll
    for (int al = 0; al < kNL; ++al) phi = fma(Xm[al], L[al], phi);
    double g[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
#pragma unroll
      for (int al = 0; al < kNL; ++al) {
        if (kMI.n[al] >= kP) continue;
        s = fma(Xm[al], L[mi_id(kMI.a[al] + (k == 0), kMI.b[al] + (k == 1), kMI.c[al] + (k == 2))], s);
      }
      g[k] = -s + L[kNL + k];
    }
    const int32_t o = perm[p];
    ax[o] += G * g[0];
    ay[o] += G * g[1];
    az[o] += G * g[2];
    if (pot) pot[o] += G * phi;
  }
}

}  // namespace

void order_upward(Ctx& c) {
  const int32_t nc = c.ncells;
  double* mono = (double*)ensure(c, c.mono, sizeof(double) * kNL * (size_t)nc);
  hipLaunchKernelGGL(k_mono_leaves, dim3(blocks_for(c.nleaves, kBS)), dim3(kBS), 0, c.stream,
                     (const double4*)c.pos4.p, as<int32_t>(c.leaves), c.nleaves, as<int32_t>(c.c_begin),
                     as<int32_t>(c.c_count), (const double4*)c.geo.p, mono);
  AMFMM_HIP(hipGetLastError());
  for (int l = c.depth - 1; l >= 0; --l) {
    const int32_t c0 = c.level_start[l], nl = c.level_start[l + 1] - c0;
    hipLaunchKernelGGL(k_mono_up, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, c0, nl,
                       as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild), (const double4*)c.geo.p, mono);
    AMFMM_HIP(hipGetLastError());
  }
}

void order_far(Ctx& c, int32_t c_lo, int32_t c_hi, double* loc) {
  const int32_t nc = c_hi - c_lo;
  if (nc <= 0) return;
  double* locg = (double*)ensure_keep(c, c.locg, sizeof(double) * kLocGen * (size_t)c.ncells,
                                      sizeof(double) * kLocGen * (size_t)c.ncells);
  hipLaunchKernelGGL(k_far_order, dim3(blocks_for(nc, kWaves)), dim3(kBS), 0, c.stream, c_lo, nc,
                     (const double4*)c.geo.p, (const double*)c.mono.p, (const int64_t*)c.far_start.p,
                     (const int32_t*)c.far_count.p, (const int32_t*)c.far_src.p, locg, loc,
                     c.opt.softening * c.opt.softening);
  AMFMM_HIP(hipGetLastError());
  if (c.opt.variant != AMFMM_UC) {
    hipLaunchKernelGGL(k_corr_order, dim3(blocks_for(nc, kWaves)), dim3(kBS), 0, c.stream, c_lo, nc,
                       (const double4*)c.geo.p, (const double*)c.mono.p, (const int64_t*)c.far_start.p,
                       (const int32_t*)c.far_count.p, (const int32_t*)c.far_src.p, locg,
                       c.opt.softening * c.opt.softening);
    AMFMM_HIP(hipGetLastError());
  }
}

void order_push_down(Ctx& c, int32_t c_lo, int32_t c_hi) {
  const int32_t nl = c_hi - c_lo;
  if (nl <= 0) return;
  hipLaunchKernelGGL(k_l2l_order, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, c_lo, nl,
                     as<int32_t>(c.c_parent), (const double4*)c.geo.p, as<double>(c.locg));
  AMFMM_HIP(hipGetLastError());
}

void order_l2p(Ctx& c, const int32_t* leaves, int32_t c_lo, int32_t count, double* ax, double* ay, double* az,
               double* pot) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_l2p_order, dim3(blocks_for((int64_t)count * kL2PLanes, kBS)), dim3(kBS), 0, c.stream, count,
                     leaves, c_lo,
                     as<int32_t>(c.c_nchild), as<int32_t>(c.c_begin), as<int32_t>(c.c_count),
                     (const double4*)c.pos4.p, (const double4*)c.geo.p, (const double*)c.locg.p, as<int32_t>(c.perm),
                     c.opt.G, ax, ay, az, pot);
  AMFMM_HIP(hipGetLastError());
}

}  // namespace amfmm
