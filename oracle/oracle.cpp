// CPU FP64 oracle of the angular-momentum-conserving Cartesian FMM
// (Marcello 2017).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke
// check and the CPU-baseline leg of the benchmark, never by the GPU solver.
//
// Plain, slow and written to be checked against the paper by eye:
//   * full 3-index / 4-index tensor loops, no symmetry packing;
//   * moments summed directly over each cell's particles (eq. 1, quad, the
//     octupole definition), not shifted from children;
//   * the far field of every accepted pair evaluated at each particle of
//     both cells with eqs. 2-4 as printed (no local-expansion push-down);
//   * the near field by direct mutual summation over particle pairs.
// Built with -O2 -ffp-contract=off so that every product and sum rounds on
// its own, in the order written here.
//
// Where the paper is silent the readings are (each is also listed in the
// design notes of the repository):
//   R := Z_A - Z_B for the pair (field cell A, source cell B): with the printed
//        D tensors this is the sign that makes eqs. 2-4 attractive and
//        consistent with the Taylor expansion of G(X - Y);
//   eq. 7 uses the appendix prefactor 1/(n!(P-n)!) = 1/6 at P = 3, with the
//        sign of eq. 7 (A gets +F_c/M_A, B gets -F_c/M_B);
//   dipole terms are dropped (they vanish about the centre of mass);
//   the correction is a force only; potentials exclude it;
//   tree: Morton keys on a 21-bit grid over the bounding cube, split iff
//        count > n_crit and level < max_level, children in octant order;
//   centres of mass are summed leaf-sequentially in key order and parents over
//        their children in octant order;
//   the walk follows a symmetric dual recursion (below).
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <utility>
#include <array>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int kMaxLevel = 21;  // key resolution: 21 bits per dimension

struct Cell {
  int32_t level;
  int64_t begin, count;
  int32_t parent, child0, nchild;
  uint64_t prefix;  // key >> 3*(21-level)
};

struct Moments {
  double M = 0.0;
  double S[3] = {0.0, 0.0, 0.0};  // sum of mu * X, used for Z
  double Z[3] = {0.0, 0.0, 0.0};
  double Rmax = 0.0;
  double M2[3][3] = {};     // sum mu x_i x_j about Z
  double M3[3][3][3] = {};  // sum mu x_i x_j x_k about Z
  std::vector<double> mono; // expansion order P != 3: sum mu x^alpha about Z, |alpha| <= P
};

}  // namespace

struct orc_tree {
  int64_t n = 0;
  int32_t n_crit = 25;
  int32_t max_level = kMaxLevel;
  double lo[3] = {0, 0, 0};
  double side = 1.0, scale = 1.0;
  std::vector<double> x, y, z, m;  // sorted copies
  std::vector<int64_t> perm;       // sorted index -> caller index
  std::vector<uint64_t> keys;      // sorted keys
  std::vector<Cell> cells;         // (level, begin) order
  std::vector<Moments> mom;
  bool have_moments = false;
  bool have_lists = false;
  double theta = 0.5;
  int mode = 0;  // 0 opening angle, 1 error estimate, 2 learned, 3 multipole error estimate
  double eps = 0.0, theta_max = 1.0;
  std::vector<double> fscale;  // per-cell field scale (modes 1 and 2)
  std::vector<float> model;    // mode 2: network and feature normalisation
  int64_t min_work = 0;        // mode 2: least N_A N_B for which the network decides
  std::vector<int> k2, k3;     // modes 2, 3: quantised traceless quadrupole and octupole norms
  std::vector<std::pair<int32_t, int32_t>> m2l, p2p;
  int64_t coincident = 0;
  double eps2 = 0.0;  // Plummer softening length squared (0: the plain 1/R)
  int order = 3;         // expansion order P (appendix)
  bool general = false;  // the appendix's general form (always at P != 3; at P = 3 on request)
};

namespace {

inline bool is_leaf(const Cell& c) { return c.nchild == 0; }

double kdelta(int a, int b) { return a == b ? 1.0 : 0.0; }

// ---------------------------------------------------------------- keys ---
// Root cube: lo_d = min over particles of X_d; side = largest extent (1 if the
// points coincide).  Each coordinate is quantised to 21 bits and the three
// integers are interleaved, x in the most significant bit of every triple.
uint64_t morton_key(const double X[3], const double lo[3], double scale) {
  const uint64_t qmax = (uint64_t(1) << kMaxLevel) - 1;
  uint64_t q[3];
  for (int d = 0; d < 3; ++d) {
    double v = (X[d] - lo[d]) * scale;
    double f = std::floor(v);
    uint64_t qi = f <= 0.0 ? 0 : (uint64_t)f;
    q[d] = qi > qmax ? qmax : qi;
  }
  uint64_t key = 0;
  for (int b = 0; b < kMaxLevel; ++b) {
    key |= ((q[0] >> b) & 1) << (3 * b + 2);
    key |= ((q[1] >> b) & 1) << (3 * b + 1);
    key |= ((q[2] >> b) & 1) << (3 * b + 0);
  }
  return key;
}

// ------------------------------------------------------- Green's function ---
// g(R) = -1/R and its derivatives, Sec. 2.  D..D_ijk as printed; D_ijkl is the
// fourth derivative (derived by differentiating D_ijk once more); D'_ijkl is
// the tensor of eq. 8.
struct Greens {
  double D0;
  double D1[3];
  double D2[3][3];
  double D3[3][3][3];
  double D4[3][3][3][3];
  double D4p[3][3][3][3];
};

void greens(const double R[3], Greens& g, bool want4) {
  double R2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
  double Rn = std::sqrt(R2);
  double inv = 1.0 / Rn;
  double inv3 = inv * inv * inv;
  double inv5 = inv3 * inv * inv;
  double inv7 = inv5 * inv * inv;
  double inv9 = inv7 * inv * inv;
  g.D0 = -inv;
  for (int i = 0; i < 3; ++i) g.D1[i] = R[i] * inv3;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) g.D2[i][j] = -(3.0 * R[i] * R[j] - kdelta(i, j) * R2) * inv5;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        g.D3[i][j][k] = (15.0 * R[i] * R[j] * R[k] -
                         3.0 * (kdelta(i, j) * R[k] + kdelta(j, k) * R[i] + kdelta(k, i) * R[j]) * R2) *
                        inv7;
  if (!want4) return;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double t4 = -105.0 * R[i] * R[j] * R[k] * R[l] * inv9;
          double t2 = 15.0 *
                      (kdelta(i, j) * R[k] * R[l] + kdelta(i, k) * R[j] * R[l] +
                       kdelta(i, l) * R[j] * R[k] + kdelta(j, k) * R[i] * R[l] +
                       kdelta(j, l) * R[i] * R[k] + kdelta(k, l) * R[i] * R[j]) *
                      inv7;
          double t0 = -3.0 *
                      (kdelta(i, j) * kdelta(k, l) + kdelta(i, k) * kdelta(j, l) +
                       kdelta(i, l) * kdelta(j, k)) *
                      inv5;
          g.D4[i][j][k][l] = t4 + t2 + t0;
          // eq. 8: only the delta_i. terms of the fourth derivative are kept
          double p2 = 15.0 *
                      (kdelta(i, j) * R[k] * R[l] + kdelta(i, k) * R[j] * R[l] +
                       kdelta(i, l) * R[j] * R[k]) *
                      inv7;
          g.D4p[i][j][k][l] = p2 + t0;
        }
}

// The same derivatives for the softened Green's function g = -1/sqrt(R^2 +
// eps^2) (Sec. 4: the correction holds for any g that depends on R only).
// For any such g, with f_k = (1/R d/dR)^k g (here f_k = (-1)^(k+1)
// (2k-1)!! s^-(2k+1)/2, s = R^2 + eps^2), the derivatives are sums over the
// ways to pair up indices: D_i = f1 R_i, D_ij = f1 d_ij + f2 R_i R_j,
// D_ijk = f2 (d_ij R_k + d_jk R_i + d_ki R_j) + f3 R_i R_j R_k, and
// D_ijkl = f2 (three dd) + f3 (six dRR) + f4 RRRR; at eps = 0 they are the
// printed tensors.  D'_ijkl keeps the d_i. terms, as in eq. 8.
void greens_softened(const double R[3], double eps2, Greens& g, bool want4) {
  double s = ((R[0] * R[0] + R[1] * R[1]) + R[2] * R[2]) + eps2;
  double rs = std::sqrt(s);
  double f0 = -1.0 / rs;
  double f1 = 1.0 / (s * rs);
  double f2 = -3.0 * f1 / s;
  double f3 = -5.0 * f2 / s;
  double f4 = -7.0 * f3 / s;
  g.D0 = f0;
  for (int i = 0; i < 3; ++i) g.D1[i] = f1 * R[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) g.D2[i][j] = f1 * kdelta(i, j) + f2 * R[i] * R[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        g.D3[i][j][k] = f2 * (kdelta(i, j) * R[k] + kdelta(j, k) * R[i] + kdelta(k, i) * R[j]) +
                        f3 * R[i] * R[j] * R[k];
  if (!want4) return;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double dd = kdelta(i, j) * kdelta(k, l) + kdelta(i, k) * kdelta(j, l) + kdelta(i, l) * kdelta(j, k);
          double di = kdelta(i, j) * R[k] * R[l] + kdelta(i, k) * R[j] * R[l] + kdelta(i, l) * R[j] * R[k];
          double dr = kdelta(j, k) * R[i] * R[l] + kdelta(j, l) * R[i] * R[k] + kdelta(k, l) * R[i] * R[j];
          g.D4[i][j][k][l] = f2 * dd + f3 * (di + dr) + f4 * R[i] * R[j] * R[k] * R[l];
          g.D4p[i][j][k][l] = f2 * dd + f3 * di;
        }
}

// --------------------------------------------------------------- moments ---
// M2_ij = sum mu x_i x_j and M3_ijk = sum mu x_i x_j x_k with x = X - Z, summed
// over the particles [b, b+cnt) of the sorted arrays (eq. quad and the
// octupole definition).  Rmax^2 is the largest squared distance to Z.
void moments_about(const orc_tree& t, int64_t b, int64_t cnt, Moments& mo) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      mo.M2[i][j] = 0.0;
      for (int k = 0; k < 3; ++k) mo.M3[i][j][k] = 0.0;
    }
  double r2max = 0.0;
  for (int64_t p = b; p < b + cnt; ++p) {
    double xv[3] = {t.x[p] - mo.Z[0], t.y[p] - mo.Z[1], t.z[p] - mo.Z[2]};
    double mu = t.m[p];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        mo.M2[i][j] += mu * xv[i] * xv[j];
        for (int k = 0; k < 3; ++k) mo.M3[i][j][k] += mu * xv[i] * xv[j] * xv[k];
      }
    double r2 = (xv[0] * xv[0] + xv[1] * xv[1]) + xv[2] * xv[2];
    if (r2 > r2max) r2max = r2;
  }
  mo.Rmax = std::sqrt(r2max);
}

// ------------------------------------------------ general expansion order ---
// The appendix's expansion to order P, written with multi-indices alpha =
// (a, b, c) (x^alpha = x^a y^b z^c, alpha! = a! b! c!): a full tensor index
// tuple with a ones, b twos and c threes stands for alpha, and a sum over all
// tuples of order n is a sum over |alpha| = n weighted by n!/alpha!.
constexpr int kMaxOrder = 6;  // P <= 6: derivatives up to order 7

struct MultiIndexTable {
  std::vector<std::array<int, 3>> e;  // exponents, graded by order
  std::vector<int> order;
  std::vector<double> fact;           // alpha!
  int id[kMaxOrder + 2][kMaxOrder + 2][kMaxOrder + 2];
  int count[kMaxOrder + 3];           // multi-indices of order < n
  MultiIndexTable() {
    for (int n = 0; n <= kMaxOrder + 1; ++n) {
      count[n] = (int)e.size();
      for (int a = n; a >= 0; --a)
        for (int b = n - a; b >= 0; --b) {
          int c = n - a - b;
          id[a][b][c] = (int)e.size();
          e.push_back({a, b, c});
          order.push_back(n);
          double f = 1.0;
          for (int k = 2; k <= a; ++k) f *= k;
          for (int k = 2; k <= b; ++k) f *= k;
          for (int k = 2; k <= c; ++k) f *= k;
          fact.push_back(f);
        }
    }
    count[kMaxOrder + 2] = (int)e.size();
  }
  int of(int a, int b, int c) const { return id[a][b][c]; }
};
const MultiIndexTable kMI;

double power(double v, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= v;
  return r;
}

// D_gamma = d^gamma g(R) for |gamma| <= nmax, g = -1/sqrt(R^2 + eps2) (the
// plain -1/R at eps2 = 0).  For any g of R alone, with f_k = (1/R d/dR)^k g
// (f_0 = -s^-1/2, f_{k+1} = -(2k+1) f_k / s, s = R^2 + eps2), the derivative is
// a sum over the ways to pair up equal indices: pairing b_i of the gamma_i
// indices of direction i (gamma_i! / (b_i! (gamma_i - 2 b_i)! 2^b_i) ways)
// leaves R_i^(gamma_i - 2 b_i) and the factor f_(|gamma| - |b|).  At order
// <= 4 this is the tensors of greens() and greens_softened().
void greens_general(const double R[3], double eps2, int nmax, std::vector<double>& D) {
  double s = ((R[0] * R[0] + R[1] * R[1]) + R[2] * R[2]) + eps2;
  double f[kMaxOrder + 2];
  f[0] = -1.0 / std::sqrt(s);
  for (int k = 0; k + 1 <= nmax; ++k) f[k + 1] = -(2.0 * k + 1.0) * f[k] / s;
  D.assign(kMI.count[nmax + 1], 0.0);
  for (int g = 0; g < kMI.count[nmax + 1]; ++g) {
    const auto& ge = kMI.e[g];
    double sum = 0.0;
    for (int b0 = 0; 2 * b0 <= ge[0]; ++b0)
      for (int b1 = 0; 2 * b1 <= ge[1]; ++b1)
        for (int b2 = 0; 2 * b2 <= ge[2]; ++b2) {
          int b[3] = {b0, b1, b2};
          double c = 1.0;
          for (int i = 0; i < 3; ++i) {
            double ways = 1.0;
            for (int k = 2; k <= ge[i]; ++k) ways *= k;
            for (int k = 2; k <= b[i]; ++k) ways /= k;
            for (int k = 2; k <= ge[i] - 2 * b[i]; ++k) ways /= k;
            ways /= power(2.0, b[i]);
            c *= ways * power(R[i], ge[i] - 2 * b[i]);
          }
          sum += f[kMI.order[g] - (b0 + b1 + b2)] * c;
        }
    D[g] = sum;
  }
}

// x^alpha for every |alpha| <= n (out holds kMI.count[n + 1] values)
constexpr int kMaxMono = (kMaxOrder + 1) * (kMaxOrder + 2) * (kMaxOrder + 3) / 6;
void monomials(const double x[3], int n, double* out) {
  for (int g = 0; g < kMI.count[n + 1]; ++g)
    out[g] = power(x[0], kMI.e[g][0]) * power(x[1], kMI.e[g][1]) * power(x[2], kMI.e[g][2]);
}

// M_alpha = sum mu x^alpha about Z, |alpha| <= P, of the particles [b, b+cnt)
void moments_general(const orc_tree& t, int64_t b, int64_t cnt, int P, Moments& mo) {
  mo.mono.assign(kMI.count[P + 1], 0.0);
  double xm[kMaxMono];
  for (int64_t p = b; p < b + cnt; ++p) {
    double xv[3] = {t.x[p] - mo.Z[0], t.y[p] - mo.Z[1], t.z[p] - mo.Z[2]};
    monomials(xv, P, xm);
    for (int g = 0; g < kMI.count[P + 1]; ++g) mo.mono[g] += t.m[p] * xm[g];
  }
}

// One accepted pair (a, b) at order P, R = Z_a - Z_b.  With G(R + x - y)
// expanded in both offsets, the potential at offset x from Z_a due to b is
// sum_alpha x^alpha/alpha! La_alpha, La_alpha = sum_beta (-1)^|beta|/beta!
// D_(alpha+beta) M_b,beta over |alpha| + |beta| <= P, and at offset y from
// Z_b due to a the same with Lb_alpha = (-1)^|alpha| sum_beta 1/beta!
// D_(alpha+beta) M_a,beta (D(-R) = (-1)^n D(R)).  Dipole terms (|beta| = 1,
// zero about the centre of mass) and the constant |alpha| = 0, |beta| = P
// are dropped, as at P = 3.  The acceleration is minus the gradient.  The
// correction (TC): F_c,k = -sum_n (-1)^n sum_{|alpha| = P-n, |beta| = n}
// M_a,alpha M_b,beta D_(alpha+beta+e_k) / (alpha! beta!), the appendix's
// corrective force (its expansion carries (-1)^n on the source offsets, so
// its D is taken at this R) in this sign convention: at P = 3 it is eq. 7,
// -(1/6)(M_a,jkl M_b - M_a M_b,jkl) D_ijkl.  +F_c/M_a on a's particles and
// -F_c/M_b on b's.
struct GeneralPair {
  std::vector<double> La, Lb;
  double Fc[3];
};

void general_pair(const Moments& A, const Moments& B, int variant, int P, double eps2, GeneralPair& gp) {
  double R[3] = {A.Z[0] - B.Z[0], A.Z[1] - B.Z[1], A.Z[2] - B.Z[2]};
  std::vector<double> D;
  greens_general(R, eps2, P + 1, D);
  int nl = kMI.count[P + 1];
  gp.La.assign(nl, 0.0);
  gp.Lb.assign(nl, 0.0);
  for (int al = 0; al < nl; ++al) {
    const auto& ae = kMI.e[al];
    for (int be = 0; be < nl; ++be) {
      int na = kMI.order[al], nb = kMI.order[be];
      if (na + nb > P || nb == 1 || (na == 0 && nb == P)) continue;
      const auto& bexp = kMI.e[be];
      double Dab = D[kMI.of(ae[0] + bexp[0], ae[1] + bexp[1], ae[2] + bexp[2])];
      double sb = (nb % 2) ? -1.0 : 1.0;
      gp.La[al] += sb / kMI.fact[be] * Dab * B.mono[be];
      gp.Lb[al] += 1.0 / kMI.fact[be] * Dab * A.mono[be];
    }
    if (kMI.order[al] % 2) gp.Lb[al] = -gp.Lb[al];
  }
  for (int k = 0; k < 3; ++k) gp.Fc[k] = 0.0;
  if (variant == ORC_UC) return;
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int n = 0; n <= P; ++n) {
      if (n == 1 || P - n == 1) continue;
      double sn = (n % 2) ? -1.0 : 1.0;
      for (int al = kMI.count[P - n]; al < kMI.count[P - n + 1]; ++al)
        for (int be = kMI.count[n]; be < kMI.count[n + 1]; ++be) {
          const auto& ae = kMI.e[al];
          const auto& bexp = kMI.e[be];
          int g[3] = {ae[0] + bexp[0], ae[1] + bexp[1], ae[2] + bexp[2]};
          g[k] += 1;
          s += sn * A.mono[al] * B.mono[be] * D[kMI.of(g[0], g[1], g[2])] / (kMI.fact[al] * kMI.fact[be]);
        }
    }
    gp.Fc[k] = -s;
  }
}

// acceleration (minus the gradient) and potential of a local expansion L of
// order P at offset x
void general_local_at(const std::vector<double>& L, int P, const double x[3], double g[3], double& phi) {
  double xm[kMaxMono];
  monomials(x, P, xm);
  phi = 0.0;
  for (int al = 0; al < kMI.count[P + 1]; ++al) phi += xm[al] / kMI.fact[al] * L[al];
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int al = 0; al < kMI.count[P]; ++al) {
      const auto& ae = kMI.e[al];
      int e[3] = {ae[0], ae[1], ae[2]};
      e[k] += 1;
      s += xm[al] / kMI.fact[al] * L[kMI.of(e[0], e[1], e[2])];
    }
    g[k] = -s;
  }
}

// ------------------------------------------------------------- far field ---
// One accepted pair, R = Z_A - Z_B.  Eq. 3 (field in A) and eq. 4 (field in B)
// with dipole terms dropped; eq. 2 for the potential in A and its mirror image
// for B (the expansion of G(Y - X) about -R, octupole constant dropped).
struct PairTerms {
  Greens g;
  double Fc[3];  // correction force of the variant (zero for UC)
};

void pair_terms(const Moments& A, const Moments& B, int variant, PairTerms& pt, double eps2 = 0.0) {
  double R[3] = {A.Z[0] - B.Z[0], A.Z[1] - B.Z[1], A.Z[2] - B.Z[2]};
  if (eps2 > 0.0)
    greens_softened(R, eps2, pt.g, variant != ORC_UC);
  else
    greens(R, pt.g, variant != ORC_UC);
  for (int i = 0; i < 3; ++i) pt.Fc[i] = 0.0;
  if (variant == ORC_UC) return;
  // eq. 7 / eq. 8: F_c,i = -(1/6) (M_A,jkl M_B - M_A M_B,jkl) D_ijkl
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double Q = A.M3[j][k][l] * B.M - A.M * B.M3[j][k][l];
          double D = variant == ORC_TC ? pt.g.D4[i][j][k][l] : pt.g.D4p[i][j][k][l];
          s += Q * D;
        }
    pt.Fc[i] = -(1.0 / 6.0) * s;
  }
}

// eq. 3: acceleration at x (relative to Z_A) caused by B
void eq3_accel(const Greens& g, const Moments& B, const double x[3], double out[3]) {
  for (int i = 0; i < 3; ++i) {
    double c0 = B.M * g.D1[i];
    double q = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) q += B.M2[j][k] * g.D3[i][j][k];
    c0 += 0.5 * q;
    double c1 = 0.0;
    for (int j = 0; j < 3; ++j) c1 += x[j] * (B.M * g.D2[i][j]);
    double c2 = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) c2 += x[j] * x[k] * B.M * g.D3[i][j][k];
    out[i] = -(c0 + c1 + 0.5 * c2);
  }
}

// eq. 4: acceleration at y (relative to Z_B) caused by A, same D(R)
void eq4_accel(const Greens& g, const Moments& A, const double y[3], double out[3]) {
  for (int i = 0; i < 3; ++i) {
    double c0 = -A.M * g.D1[i];
    double q = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) q += A.M2[j][k] * g.D3[i][j][k];
    c0 -= 0.5 * q;
    double c1 = 0.0;
    for (int j = 0; j < 3; ++j) c1 += y[j] * (A.M * g.D2[i][j]);
    double c2 = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) c2 += y[j] * y[k] * A.M * g.D3[i][j][k];
    out[i] = -(c0 + c1 - 0.5 * c2);
  }
}

// eq. 2: potential at x (relative to Z_A) caused by B
double eq2_pot_A(const Greens& g, const Moments& B, const double x[3]) {
  double q = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) q += B.M2[i][j] * g.D2[i][j];
  double p = B.M * g.D0 + 0.5 * q;
  for (int i = 0; i < 3; ++i) {
    double qi = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) qi += B.M2[j][k] * g.D3[i][j][k];
    p += x[i] * (B.M * g.D1[i] + 0.5 * qi);
  }
  double s2 = 0.0, s3 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      s2 += x[i] * x[j] * B.M * g.D2[i][j];
      for (int k = 0; k < 3; ++k) s3 += x[i] * x[j] * x[k] * B.M * g.D3[i][j][k];
    }
  return p + 0.5 * s2 + (1.0 / 6.0) * s3;
}

// potential at y (relative to Z_B) caused by A: the expansion of eq. 2 with the
// roles of the cells exchanged, written with the same D(R), so odd orders flip
double eq2_pot_B(const Greens& g, const Moments& A, const double y[3]) {
  double q = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) q += A.M2[i][j] * g.D2[i][j];
  double p = A.M * g.D0 + 0.5 * q;
  for (int i = 0; i < 3; ++i) {
    double qi = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) qi += A.M2[j][k] * g.D3[i][j][k];
    p -= y[i] * (A.M * g.D1[i] + 0.5 * qi);
  }
  double s2 = 0.0, s3 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      s2 += y[i] * y[j] * A.M * g.D2[i][j];
      for (int k = 0; k < 3; ++k) s3 += y[i] * y[j] * y[k] * A.M * g.D3[i][j][k];
    }
  return p + 0.5 * s2 - (1.0 / 6.0) * s3;
}

// The far-field terms of one accepted pair (a, b) at the tree's order: the
// printed equations at P = 3 (a the field cell of eq. 3, b that of eq. 4),
// the general form otherwise (or when asked for at P = 3).
struct PairField {
  int P;
  bool general;
  PairTerms pt;
  GeneralPair gp;
};

void pair_field(const orc_tree& t, int32_t a, int32_t b, int variant, PairField& pf) {
  pf.P = t.general ? t.order : 3;
  pf.general = t.general;
  if (!t.general)
    pair_terms(t.mom[a], t.mom[b], variant, pf.pt, t.eps2);
  else
    general_pair(t.mom[a], t.mom[b], variant, t.order, t.eps2, pf.gp);
}

// acceleration (the correction included) and potential at offset v from the
// centre of a (side 0) or of b (side 1)
void pair_field_at(const orc_tree& t, const PairField& pf, int32_t a, int32_t b, int side, const double v[3],
                   double g[3], double& phi) {
  const Moments& A = t.mom[a];
  const Moments& B = t.mom[b];
  double gg[3];
  if (!pf.general) {
    if (side == 0) {
      eq3_accel(pf.pt.g, B, v, gg);
      for (int d = 0; d < 3; ++d) g[d] = gg[d] + pf.pt.Fc[d] / A.M;
      phi = eq2_pot_A(pf.pt.g, B, v);
    } else {
      eq4_accel(pf.pt.g, A, v, gg);
      for (int d = 0; d < 3; ++d) g[d] = gg[d] - pf.pt.Fc[d] / B.M;
      phi = eq2_pot_B(pf.pt.g, A, v);
    }
  } else if (side == 0) {
    general_local_at(pf.gp.La, pf.P, v, gg, phi);
    for (int d = 0; d < 3; ++d) g[d] = gg[d] + pf.gp.Fc[d] / A.M;
  } else {
    general_local_at(pf.gp.Lb, pf.P, v, gg, phi);
    for (int d = 0; d < 3; ++d) g[d] = gg[d] - pf.gp.Fc[d] / B.M;
  }
}

// ------------------------------------------------- learned pair selection ---
// Not in the paper: a network predicts how far the force error the method
// makes on an accepted pair lies from the multipole error estimate (below;
// both take the role of the error-estimating pair selection cited in Sec.
// 2).  Every quantity below is defined so that a GPU implementation can
// reproduce the decision bit for bit: features use only IEEE-rounded
// operations on values both sides hold identically (centres, radii, masses,
// counts) and the traceless norm levels quantised to 1/128; the network runs
// in FP32 with fused multiply-adds in a fixed order on BF16-rounded weights.
//
// Model layout (floats): W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3,
// then the feature normalisation x = fma(f, a, b) (a[8], b[8]) and the
// training range of the raw features (lo[8], hi[8]).
constexpr int kFeat = 8, kHid = 64;
constexpr int kW1 = 0, kB1 = 512, kW2 = 576, kB2 = 4672, kW3 = 4736, kB3 = 4800;
constexpr int kNA = 4801, kNB = 4809, kLo = 4817, kHi = 4825, kModel = 4833, kParams = 4801;
constexpr int kLabelSample = 64;  // particles sampled per cell for a label
constexpr int64_t kCountCap = 1024;  // particle counts saturate here in the features

// round a float to the nearest BF16 value (ties to even), kept as float
float bf16(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  std::memcpy(&v, &u, 4);
  return v;
}

// piecewise-linear base-2 logarithm: x = 2^e (1 + f) with f in [0, 1) gives
// e + f (at most 0.086 below log2 x, never above)
double plog2(double x) {
  if (!(x > 0.0)) return -2048.0;
  if (std::isinf(x)) return 2048.0;
  int e;
  double m = std::frexp(x, &e);  // x = m 2^e, m in [0.5, 1)
  return (double)(e - 1) + (2.0 * m - 1.0);
}

// the eight features of an unordered pair (each symmetric in A and B); k2, k3
// are the traceless norm levels of the multipole estimate (0..128)
void pair_features(double d, const Moments& A, const Moments& B, int k2a, int k3a, int k2b, int k3b, int64_t na,
                   int64_t nb, float f[kFeat]) {
  double r = A.Rmax + B.Rmax;
  f[0] = (float)(r / d);                                           // (R_A + R_B) / d
  f[1] = (float)(r > 0.0 ? std::fabs(A.Rmax - B.Rmax) / r : 0.0);  // size asymmetry
  f[2] = (float)((double)(k2a + k2b) / 256.0);                     // mean quadrupole level
  f[3] = (float)((double)std::abs(k2a - k2b) / 128.0);             // its asymmetry
  f[4] = (float)((double)(k3a + k3b) / 256.0);                     // mean octupole level
  f[5] = (float)((double)std::abs(k3a - k3b) / 128.0);             // its asymmetry
  f[6] = (float)(std::fabs(A.M - B.M) / (A.M + B.M));             // mass asymmetry
  // particle counts, saturated at kCountCap: beyond it a cell behaves as a
  // continuum and the count carries no information about the error
  double ca = (double)std::min<int64_t>(na, kCountCap), cb = (double)std::min<int64_t>(nb, kCountCap);
  f[7] = (float)plog2(ca * cb);
}

double pair_distance(const Moments& A, const Moments& B) {
  double dx = A.Z[0] - B.Z[0];
  double dy = A.Z[1] - B.Z[1];
  double dz = A.Z[2] - B.Z[2];
  return std::sqrt((dx * dx + dy * dy) + dz * dz);
}

// network output (predicted log2 of the pair's error factor), FP32
float mlp_infer(const float* P, const float f[kFeat]) {
  float x[kFeat], h1[kHid], h2[kHid];
  for (int i = 0; i < kFeat; ++i) x[i] = bf16(std::fmaf(f[i], P[kNA + i], P[kNB + i]));
  for (int j = 0; j < kHid; ++j) {
    float s = P[kB1 + j];
    for (int i = 0; i < kFeat; ++i) s = std::fmaf(bf16(P[kW1 + kFeat * j + i]), x[i], s);
    h1[j] = bf16(s > 0.0f ? s : 0.0f);
  }
  for (int k = 0; k < kHid; ++k) {
    float s = P[kB2 + k];
    for (int j = 0; j < kHid; ++j) s = std::fmaf(bf16(P[kW2 + kHid * k + j]), h1[j], s);
    h2[k] = bf16(s > 0.0f ? s : 0.0f);
  }
  float y = P[kB3];
  for (int k = 0; k < kHid; ++k) y = std::fmaf(bf16(P[kW3 + k]), h2[k], y);
  return y;
}

// ------------------------------------------- multipole error estimate ---
// The force error of an accepted pair on cell A (field) from cell B (source)
// has three leading parts: B's traceless octupole (dropped by the expansion),
// B's traceless quadrupole times A's extent (the quadrupole enters only C and
// C_k), and the truncation of the Taylor series of B's field over A (third
// order in the potential); the next order adds R^4/d terms.  Per unit mass of
// B and with k3, k2 the traceless octupole and quadrupole norms in units of
// M R^3 and M R^2 (quantised to 1/128, rounded to nearest), the estimate is
//   e_A = ((w3 k3_B R_B^3 + w2 k2_B R_B^2 R_A + w1 R_A^3) d + w4 R_B^4 + w5 R_A^4) M_B / d^6
// with weights calibrated on measured pair errors of this method (the largest
// error over A's particles; least squares in log space over the accepted
// pairs of geometric walks of a 65536-particle Plummer sphere at opening
// angles 0.4, 0.6, 0.8), as fit_multipole.py beside this file computes them.
constexpr double kMw1 = 1.326, kMw2 = 4.095, kMw3 = 0.285, kMw4 = 0.1416, kMw5 = 1.618;
constexpr double kMq = 128.0;  // quantisation of the norm ratios

// traceless part of M_ij: M_ij - delta_ij tr/3; of M_ijk: M_ijk - (v_i
// delta_jk + v_j delta_ik + v_k delta_ij)/5 with v_i = M_ijj
double traceless_norm2(const Moments& mo) {
  double tr = mo.M2[0][0] + mo.M2[1][1] + mo.M2[2][2], s = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = mo.M2[i][j] - (i == j ? tr / 3.0 : 0.0);
      s += v * v;
    }
  return std::sqrt(s);
}

double traceless_norm3(const Moments& mo) {
  double v[3];
  for (int i = 0; i < 3; ++i) v[i] = mo.M3[i][0][0] + mo.M3[i][1][1] + mo.M3[i][2][2];
  double s = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        double w = mo.M3[i][j][k] - (v[i] * kdelta(j, k) + v[j] * kdelta(i, k) + v[k] * kdelta(i, j)) / 5.0;
        s += w * w;
      }
  return std::sqrt(s);
}

// norm / (M R^p) to the nearest 1/kMq, in [0, kMq]
int norm_level(double norm, double M, double R, int p) {
  double den = M * (p == 2 ? R * R : R * R * R);
  if (!(den > 0.0)) return 0;
  double k = std::floor(kMq * (norm / den) + 0.5);
  if (k < 0.0) return 0;
  if (k > kMq) return (int)kMq;
  return (int)k;
}

// the estimate's bracket for field cell T and source S at distance d:
// P d + Q with P = w3 k3_S R_S^3 + w2 k2_S R_S^2 R_T + w1 R_T^3, Q = w4 R_S^4 + w5 R_T^4
double multipole_bracket(double rt, double rs, int k2s, int k3s, double d) {
  double rt2 = rt * rt, rs2 = rs * rs;
  double P = ((kMw3 * (k3s / kMq)) * (rs2 * rs) + (kMw2 * (k2s / kMq)) * (rs2 * rt)) + kMw1 * (rt2 * rt);
  double Q = kMw4 * (rs2 * rs2) + kMw5 * (rt2 * rt2);
  return P * d + Q;
}

// ------------------------------------------------------------------ walk ---
// Symmetric dual recursion.  A pair is accepted when |Z_A - Z_B| >= (R_A +
// R_B)/theta (and the centres differ); two leaves that fail become a near-field
// pair; otherwise the larger cell (by R_max, ties to the lower index; the
// non-leaf when one is a leaf) is replaced by its children.  A cell with itself
// recurses into its children's self pairs and all child pairs.
bool accept(const orc_tree& t, int32_t a, int32_t b) {
  const Moments& A = t.mom[a];
  const Moments& B = t.mom[b];
  double dx = A.Z[0] - B.Z[0];
  double dy = A.Z[1] - B.Z[1];
  double dz = A.Z[2] - B.Z[2];
  double d = std::sqrt((dx * dx + dy * dy) + dz * dz);
  if (t.mode == 0) {
    double rhs = (A.Rmax + B.Rmax) / t.theta;
    return d > 0.0 && d >= rhs;
  }
  double r = A.Rmax + B.Rmax;
  if (t.mode == 3) {
    // multipole error estimate e_A M... in product form (one root, no
    // division): (P_A d + Q_A) M_B <= eps s_A d2^3 and the same for B
    double d2 = (dx * dx + dy * dy) + dz * dz;
    if (!(d2 > 0.0 && r * r <= (t.theta_max * t.theta_max) * d2)) return false;
    double d = std::sqrt(d2);
    double d6 = (d2 * d2) * d2;
    double ea = multipole_bracket(A.Rmax, B.Rmax, t.k2[b], t.k3[b], d) * B.M;
    double eb = multipole_bracket(B.Rmax, A.Rmax, t.k2[a], t.k3[a], d) * A.M;
    return ea <= (t.eps * t.fscale[a]) * d6 && eb <= (t.eps * t.fscale[b]) * d6;
  }
  if (t.mode == 1) {
    // error estimate (R_A + R_B)^3 M_other / d^5 against eps times each
    // cell's field scale, and (R_A + R_B) <= theta_max d, in product form
    // (squared, no division or root) with d2 = d^2
    double d2 = (dx * dx + dy * dy) + dz * dz;
    if (!(d2 > 0.0 && r * r <= (t.theta_max * t.theta_max) * d2)) return false;
    double r2 = r * r;
    double r6 = (r2 * r2) * r2;
    double d10 = ((d2 * d2) * (d2 * d2)) * d2;
    double wa = t.eps * t.fscale[a], wb = t.eps * t.fscale[b];
    return r6 * (B.M * B.M) <= (wa * wa) * d10 && r6 * (A.M * A.M) <= (wb * wb) * d10;
  }
  // mode 2, learned: the multipole estimate (as mode 3), with the network
  // deciding where it lies near the allowed error.  With rho the larger of
  // e / (eps s d^6) over the two cells: rho <= 1/4 accepts, rho > 2 opens
  // (eps scaled by powers of two, exactly); pairs with N_A N_B
  // below min_work or features outside the training range take rho <= 1;
  // the others are accepted when the predicted log2 ratio of the method's
  // error to the estimate is at most -plog2(rho).
  double d2 = (dx * dx + dy * dy) + dz * dz;
  if (!(d2 > 0.0 && r * r <= (t.theta_max * t.theta_max) * d2)) return false;
  double dl = std::sqrt(d2);
  double d6 = (d2 * d2) * d2;
  double ea = multipole_bracket(A.Rmax, B.Rmax, t.k2[b], t.k3[b], dl) * B.M;
  double eb = multipole_bracket(B.Rmax, A.Rmax, t.k2[a], t.k3[a], dl) * A.M;
  double sa = t.fscale[a], sb = t.fscale[b];
  double lo = 0.25 * t.eps, hi = 2.0 * t.eps;
  if (ea <= (lo * sa) * d6 && eb <= (lo * sb) * d6) return true;
  if (!(ea <= (hi * sa) * d6 && eb <= (hi * sb) * d6)) return false;
  bool plain = ea <= (t.eps * sa) * d6 && eb <= (t.eps * sb) * d6;
  if (t.cells[a].count * t.cells[b].count < t.min_work) return plain;
  float f[kFeat];
  pair_features(dl, A, B, t.k2[a], t.k3[a], t.k2[b], t.k3[b], t.cells[a].count, t.cells[b].count, f);
  const float* P = t.model.data();
  for (int i = 0; i < kFeat; ++i)
    if (!(f[i] >= P[kLo + i] && f[i] <= P[kHi + i])) return plain;
  double ra = ea / ((t.eps * sa) * d6), rb = eb / ((t.eps * sb) * d6);
  double rho = std::max(ra, rb);
  return mlp_infer(P, f) <= (float)(-plog2(rho));
}

void walk_pair(orc_tree& t, int32_t a, int32_t b) {
  if (accept(t, a, b)) {
    t.m2l.emplace_back(std::min(a, b), std::max(a, b));
    return;
  }
  const Cell& A = t.cells[a];
  const Cell& B = t.cells[b];
  if (is_leaf(A) && is_leaf(B)) {
    t.p2p.emplace_back(std::min(a, b), std::max(a, b));
    return;
  }
  double ra = t.mom[a].Rmax, rb = t.mom[b].Rmax;
  bool split_a;
  if (is_leaf(A))
    split_a = false;
  else if (is_leaf(B))
    split_a = true;
  else
    split_a = ra > rb || (ra == rb && a < b);
  if (split_a) {
    for (int32_t c = A.child0; c < A.child0 + A.nchild; ++c) walk_pair(t, c, b);
  } else {
    for (int32_t c = B.child0; c < B.child0 + B.nchild; ++c) walk_pair(t, a, c);
  }
}

void walk_self(orc_tree& t, int32_t c) {
  const Cell& C = t.cells[c];
  if (is_leaf(C)) {
    t.p2p.emplace_back(c, c);
    return;
  }
  for (int32_t a = C.child0; a < C.child0 + C.nchild; ++a) walk_self(t, a);
  for (int32_t a = C.child0; a < C.child0 + C.nchild; ++a)
    for (int32_t b = a + 1; b < C.child0 + C.nchild; ++b) walk_pair(t, a, b);
}

bool finite_inputs(int64_t n, const double* x, const double* y, const double* z, const double* m,
                   int32_t* status) {
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(z[i]) ||
        !std::isfinite(m[i])) {
      *status = ORC_E_NONFINITE;
      return false;
    }
    if (!(m[i] > 0.0)) {
      *status = ORC_E_INVALID;
      return false;
    }
  }
  return true;
}

}  // namespace

extern "C" {

orc_tree* orc_build_tree(int64_t n, const double* x, const double* y, const double* z,
                         const double* m, int32_t n_crit, int32_t max_level, int32_t* status) {
  int32_t st_dummy;
  if (!status) status = &st_dummy;
  *status = ORC_OK;
  if (n < 1 || n_crit < 1 || max_level < 0 || max_level > kMaxLevel) {
    *status = ORC_E_INVALID;
    return nullptr;
  }
  if (!finite_inputs(n, x, y, z, m, status)) return nullptr;
  orc_tree* t = new orc_tree();
  t->n = n;
  t->n_crit = n_crit;
  t->max_level = max_level;
  // root cube
  double hi[3];
  t->lo[0] = hi[0] = x[0];
  t->lo[1] = hi[1] = y[0];
  t->lo[2] = hi[2] = z[0];
  for (int64_t i = 1; i < n; ++i) {
    t->lo[0] = std::min(t->lo[0], x[i]);
    hi[0] = std::max(hi[0], x[i]);
    t->lo[1] = std::min(t->lo[1], y[i]);
    hi[1] = std::max(hi[1], y[i]);
    t->lo[2] = std::min(t->lo[2], z[i]);
    hi[2] = std::max(hi[2], z[i]);
  }
  double side = 0.0;
  for (int d = 0; d < 3; ++d) side = std::max(side, hi[d] - t->lo[d]);
  if (side == 0.0) side = 1.0;
  t->side = side;
  t->scale = double(uint64_t(1) << kMaxLevel) / side;
  // keys, then a stable sort: equal keys keep caller order
  std::vector<uint64_t> key(n);
  for (int64_t i = 0; i < n; ++i) {
    double X[3] = {x[i], y[i], z[i]};
    key[i] = morton_key(X, t->lo, t->scale);
  }
  t->perm.resize(n);
  std::iota(t->perm.begin(), t->perm.end(), int64_t(0));
  std::stable_sort(t->perm.begin(), t->perm.end(),
                   [&](int64_t a, int64_t b) { return key[a] < key[b]; });
  t->keys.resize(n);
  t->x.resize(n);
  t->y.resize(n);
  t->z.resize(n);
  t->m.resize(n);
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = t->perm[s];
    t->keys[s] = key[i];
    t->x[s] = x[i];
    t->y[s] = y[i];
    t->z[s] = z[i];
    t->m[s] = m[i];
  }
  // octree, one level at a time: a cell with more than n_crit particles below
  // the finest level is split into its non-empty octants, in octant order
  Cell root{0, 0, n, -1, -1, 0, 0};
  t->cells.push_back(root);
  size_t level_begin = 0;
  for (int lev = 0;; ++lev) {
    size_t level_end = t->cells.size();
    if (level_begin == level_end) break;
    for (size_t c = level_begin; c < level_end; ++c) {
      Cell cur = t->cells[c];
      if (!(cur.count > n_crit && lev < max_level)) continue;
      int shift = 3 * (kMaxLevel - (lev + 1));
      int32_t first_child = (int32_t)t->cells.size();
      int32_t nch = 0;
      for (uint64_t oct = 0; oct < 8; ++oct) {
        int64_t b = -1, cnt = 0;
        for (int64_t p = cur.begin; p < cur.begin + cur.count; ++p) {
          if (((t->keys[p] >> shift) & 7) == oct) {
            if (b < 0) b = p;
            ++cnt;
          }
        }
        if (cnt == 0) continue;
        Cell ch{lev + 1, b, cnt, (int32_t)c, -1, 0, (cur.prefix << 3) | oct};
        t->cells.push_back(ch);
        ++nch;
      }
      t->cells[c].child0 = first_child;
      t->cells[c].nchild = nch;
    }
    level_begin = level_end;
  }
  return t;
}

void orc_free(orc_tree* t) { delete t; }

int64_t orc_num_cells(const orc_tree* t) { return (int64_t)t->cells.size(); }

int32_t orc_depth(const orc_tree* t) {
  int32_t d = 0;
  for (const Cell& c : t->cells) d = std::max(d, c.level);
  return d;
}

void orc_get_cube(const orc_tree* t, double* lo3, double* side, double* scale) {
  for (int d = 0; d < 3; ++d) lo3[d] = t->lo[d];
  *side = t->side;
  *scale = t->scale;
}

void orc_get_keys(const orc_tree* t, uint64_t* keys, int64_t* perm) {
  for (int64_t s = 0; s < t->n; ++s) {
    if (keys) keys[s] = t->keys[s];
    if (perm) perm[s] = t->perm[s];
  }
}

void orc_get_cells(const orc_tree* t, int32_t* level, int64_t* begin, int64_t* count,
                   int32_t* parent, int32_t* child0, int32_t* nchild) {
  for (size_t c = 0; c < t->cells.size(); ++c) {
    const Cell& C = t->cells[c];
    if (level) level[c] = C.level;
    if (begin) begin[c] = C.begin;
    if (count) count[c] = C.count;
    if (parent) parent[c] = C.parent;
    if (child0) child0[c] = C.nchild ? C.child0 : -1;
    if (nchild) nchild[c] = C.nchild;
  }
}

int32_t orc_compute_moments(orc_tree* t) {
  size_t nc = t->cells.size();
  t->mom.assign(nc, Moments());
  // mass and first moment: leaves sequentially over their particles, parents
  // over their children in octant order (deepest cells first)
  for (size_t ci = nc; ci-- > 0;) {
    const Cell& C = t->cells[ci];
    Moments& mo = t->mom[ci];
    if (is_leaf(C)) {
      for (int64_t p = C.begin; p < C.begin + C.count; ++p) {
        mo.M += t->m[p];
        mo.S[0] += t->m[p] * t->x[p];
        mo.S[1] += t->m[p] * t->y[p];
        mo.S[2] += t->m[p] * t->z[p];
      }
    } else {
      for (int32_t c = C.child0; c < C.child0 + C.nchild; ++c) {
        mo.M += t->mom[c].M;
        for (int d = 0; d < 3; ++d) mo.S[d] += t->mom[c].S[d];
      }
    }
    for (int d = 0; d < 3; ++d) mo.Z[d] = mo.S[d] / mo.M;
  }
  // higher moments and R_max directly from the particles of each cell
  for (size_t ci = 0; ci < nc; ++ci) {
    moments_about(*t, t->cells[ci].begin, t->cells[ci].count, t->mom[ci]);
    if (t->general) moments_general(*t, t->cells[ci].begin, t->cells[ci].count, t->order, t->mom[ci]);
  }
  t->have_moments = true;
  t->have_lists = false;
  return ORC_OK;
}

void orc_get_moments(const orc_tree* t, double* out) {
  for (size_t c = 0; c < t->mom.size(); ++c) {
    const Moments& mo = t->mom[c];
    double* o = out + 21 * c;
    o[0] = mo.M;
    o[1] = mo.Z[0];
    o[2] = mo.Z[1];
    o[3] = mo.Z[2];
    o[4] = mo.Rmax;
    int q = 5;
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) o[q++] = mo.M2[i][j];
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j)
        for (int k = j; k < 3; ++k) o[q++] = mo.M3[i][j][k];
  }
}

}  // extern "C"

namespace {
// Field scale of every cell from per-particle field magnitudes: the smallest
// |g| over its particles, but at least 0.1 times their mean (sums over leaves
// in key order, parents over children in octant order)
void set_field_scales(orc_tree* t, const double* gmag) {
  size_t nc = t->cells.size();
  std::vector<double> gsum(nc, 0.0), gmin(nc, INFINITY);
  for (size_t ci = nc; ci-- > 0;) {
    const Cell& C = t->cells[ci];
    if (is_leaf(C)) {
      for (int64_t p = C.begin; p < C.begin + C.count; ++p) {
        double g = std::fabs(gmag[t->perm[p]]);
        gsum[ci] += g;
        gmin[ci] = std::min(gmin[ci], g);
      }
    } else {
      for (int32_t c = C.child0; c < C.child0 + C.nchild; ++c) {
        gsum[ci] += gsum[c];
        gmin[ci] = std::min(gmin[ci], gmin[c]);
      }
    }
  }
  t->fscale.assign(nc, 0.0);
  for (size_t ci = 0; ci < nc; ++ci)
    t->fscale[ci] = std::max(gmin[ci], 0.1 * (gsum[ci] / (double)t->cells[ci].count));
}

// traceless quadrupole and octupole norm levels of every cell (modes 2 and 3)
void set_norm_levels(orc_tree* t) {
  size_t nc = t->cells.size();
  t->k2.resize(nc);
  t->k3.resize(nc);
  for (size_t c = 0; c < nc; ++c) {
    const Moments& mo = t->mom[c];
    t->k2[c] = norm_level(traceless_norm2(mo), mo.M, mo.Rmax, 2);
    t->k3[c] = norm_level(traceless_norm3(mo), mo.M, mo.Rmax, 3);
  }
}

void run_walk(orc_tree* t) {
  t->m2l.clear();
  t->p2p.clear();
  walk_self(*t, 0);
  std::sort(t->m2l.begin(), t->m2l.end());
  std::sort(t->p2p.begin(), t->p2p.end());
  t->have_lists = true;
}
}  // namespace

extern "C" {

int32_t orc_walk_field(orc_tree* t, double eps, double theta_max, const double* gmag) {
  if (!(eps > 0.0) || !(theta_max > 0.0 && theta_max <= 1.0) || !gmag) return ORC_E_INVALID;
  if (!t->have_moments) return ORC_E_STATE;
  set_field_scales(t, gmag);
  t->mode = 1;
  t->eps = eps;
  t->theta_max = theta_max;
  run_walk(t);
  return ORC_OK;
}

int32_t orc_walk_multipole(orc_tree* t, double eps, double theta_max, const double* gmag) {
  if (!(eps > 0.0) || !(theta_max > 0.0 && theta_max <= 1.0) || !gmag) return ORC_E_INVALID;
  if (!t->have_moments) return ORC_E_STATE;
  set_field_scales(t, gmag);
  set_norm_levels(t);
  t->mode = 3;
  t->eps = eps;
  t->theta_max = theta_max;
  run_walk(t);
  return ORC_OK;
}

void orc_multipole_levels(const orc_tree* t, int32_t* k2, int32_t* k3) {
  for (size_t c = 0; c < t->cells.size(); ++c) {
    const Moments& mo = t->mom[c];
    k2[c] = norm_level(traceless_norm2(mo), mo.M, mo.Rmax, 2);
    k3[c] = norm_level(traceless_norm3(mo), mo.M, mo.Rmax, 3);
  }
}

int32_t orc_walk_learned(orc_tree* t, double eps, double theta_max, double theta, const double* gmag,
                         const float* model, int64_t min_work) {
  if (!(theta > 0.0 && theta <= 1.0)) return ORC_E_INVALID;
  if (!model) return orc_walk(t, theta);  // no network: the opening angle
  if (!(eps > 0.0) || !(theta_max > 0.0 && theta_max <= 1.0) || !gmag) return ORC_E_INVALID;
  if (!t->have_moments) return ORC_E_STATE;
  set_field_scales(t, gmag);
  t->model.assign(model, model + kModel);
  set_norm_levels(t);
  t->mode = 2;
  t->min_work = min_work;
  t->eps = eps;
  t->theta_max = theta_max;
  t->theta = theta;
  run_walk(t);
  return ORC_OK;
}

void orc_pair_features(const orc_tree* t, int64_t np, const int32_t* pairs, float* feats) {
  size_t nc = t->cells.size();
  std::vector<int> k2(nc), k3(nc);
  for (size_t c = 0; c < nc; ++c) {
    k2[c] = norm_level(traceless_norm2(t->mom[c]), t->mom[c].M, t->mom[c].Rmax, 2);
    k3[c] = norm_level(traceless_norm3(t->mom[c]), t->mom[c].M, t->mom[c].Rmax, 3);
  }
  for (int64_t k = 0; k < np; ++k) {
    int32_t a = pairs[2 * k], b = pairs[2 * k + 1];
    const Moments& A = t->mom[a];
    const Moments& B = t->mom[b];
    pair_features(pair_distance(A, B), A, B, k2[a], k3[a], k2[b], k3[b], t->cells[a].count, t->cells[b].count,
                  feats + kFeat * k);
  }
}

// The method's largest error on field cell T from the pair (T, S) alone: the
// acceleration of eq. 3 about Z_T plus the correction of the variant at up to
// kLabelSample particles of T (evenly spread over T's range) against the
// direct sum over S's particles.
static double pair_side_error(const orc_tree* t, int32_t ct, int32_t cs, int32_t variant) {
  const Cell& T = t->cells[ct];
  const Cell& S = t->cells[cs];
  const Moments& MT = t->mom[ct];
  const Moments& MS = t->mom[cs];
  PairTerms pt;
  pair_terms(MT, MS, variant, pt);  // R = Z_T - Z_S: T is the field cell of eq. 3
  int64_t ns = std::min<int64_t>(T.count, kLabelSample);
  double E = 0.0;
  for (int64_t s = 0; s < ns; ++s) {
    int64_t p = T.begin + (s * T.count) / ns;
    double xv[3] = {t->x[p] - MT.Z[0], t->y[p] - MT.Z[1], t->z[p] - MT.Z[2]};
    double g[3];
    eq3_accel(pt.g, MS, xv, g);
    for (int dd = 0; dd < 3; ++dd) g[dd] += pt.Fc[dd] / MT.M;
    double gd[3] = {0.0, 0.0, 0.0};
    for (int64_t j = S.begin; j < S.begin + S.count; ++j) {
      double dx = t->x[j] - t->x[p];
      double dy = t->y[j] - t->y[p];
      double dz = t->z[j] - t->z[p];
      double r2 = (dx * dx + dy * dy) + dz * dz;
      double r3 = r2 * std::sqrt(r2);
      gd[0] += t->m[j] * dx / r3;
      gd[1] += t->m[j] * dy / r3;
      gd[2] += t->m[j] * dz / r3;
    }
    double ex = g[0] - gd[0], ey = g[1] - gd[1], ez = g[2] - gd[2];
    E = std::max(E, std::sqrt((ex * ex + ey * ey) + ez * ez));
  }
  return E;
}

static int32_t check_pairs(const orc_tree* t, int32_t variant, int64_t np, const int32_t* pairs) {
  if (!t->have_moments) return ORC_E_STATE;
  if (variant < ORC_UC || variant > ORC_TCO) return ORC_E_INVALID;
  int64_t nc = (int64_t)t->cells.size();
  for (int64_t k = 0; k < np; ++k) {
    int32_t a = pairs[2 * k], b = pairs[2 * k + 1];
    if (a < 0 || b < 0 || a >= nc || b >= nc || a == b) return ORC_E_INVALID;
    if (!(pair_distance(t->mom[a], t->mom[b]) > 0.0)) return ORC_E_INVALID;
  }
  return ORC_OK;
}

void orc_multipole_weights(double* w) {
  w[0] = kMw1;
  w[1] = kMw2;
  w[2] = kMw3;
  w[3] = kMw4;
  w[4] = kMw5;
}

int32_t orc_pair_errors(const orc_tree* t, int32_t variant, int64_t np, const int32_t* pairs, double* err) {
  int32_t st = check_pairs(t, variant, np, pairs);
  if (st != ORC_OK) return st;
  for (int64_t k = 0; k < np; ++k) {
    err[2 * k] = pair_side_error(t, pairs[2 * k], pairs[2 * k + 1], variant);
    err[2 * k + 1] = pair_side_error(t, pairs[2 * k + 1], pairs[2 * k], variant);
  }
  return ORC_OK;
}

// Label of a pair: for each cell T (the other S) the largest error of the
// pair on T (pair_side_error) divided by the multipole estimate of the error
// on T.  The label is log2 of the larger ratio of the two cells; a cell whose
// estimate is zero (a point mass: exact) is left out, -inf when both are.
int32_t orc_pair_labels(const orc_tree* t, int32_t variant, int64_t np, const int32_t* pairs,
                        double* labels) {
  int32_t st = check_pairs(t, variant, np, pairs);
  if (st != ORC_OK) return st;
  for (int64_t k = 0; k < np; ++k) {
    int32_t a = pairs[2 * k], b = pairs[2 * k + 1];
    double d = pair_distance(t->mom[a], t->mom[b]);
    double worst = -INFINITY;
    for (int side = 0; side < 2; ++side) {
      int32_t ct = side ? b : a, cs = side ? a : b;
      const Moments& MT = t->mom[ct];
      const Moments& MS = t->mom[cs];
      double E = pair_side_error(t, ct, cs, variant);
      int k2s = norm_level(traceless_norm2(MS), MS.M, MS.Rmax, 2);
      int k3s = norm_level(traceless_norm3(MS), MS.M, MS.Rmax, 3);
      double d2 = d * d;
      double est = multipole_bracket(MT.Rmax, MS.Rmax, k2s, k3s, d) * MS.M / ((d2 * d2) * d2);
      if (est > 0.0) worst = std::max(worst, E / est);
    }
    labels[k] = worst > 0.0 ? std::log2(worst) : -INFINITY;
  }
  return ORC_OK;
}

float orc_bf16_round(float v) { return bf16(v); }
double orc_plog2(double x) { return plog2(x); }

void orc_mlp_predict(const float* model, int64_t n, const float* feats, float* y) {
  for (int64_t r = 0; r < n; ++r) y[r] = mlp_infer(model, feats + kFeat * r);
}

// Mean pinball loss at quantile tau of the network over n rows and its
// gradient with respect to the parameters (FP64 arithmetic).  With round != 0
// the forward pass rounds weights, inputs and hidden activations to BF16 as
// inference does and the gradient passes straight through the roundings;
// with round == 0 nothing is rounded (the exact function, for finite
// differences).  The subgradient at a zero residual is -tau.
double orc_mlp_grad(const float* model, int64_t n, const float* feats, const float* labels, double tau,
                    int32_t round, double* grad) {
  auto rd = [&](double v) { return round ? (double)bf16((float)v) : v; };
  std::vector<double> W1(kHid * kFeat), W2(kHid * kHid), w3(kHid);
  for (int i = 0; i < kHid * kFeat; ++i) W1[i] = rd(model[kW1 + i]);
  for (int i = 0; i < kHid * kHid; ++i) W2[i] = rd(model[kW2 + i]);
  for (int i = 0; i < kHid; ++i) w3[i] = rd(model[kW3 + i]);
  for (int i = 0; i < kParams; ++i) grad[i] = 0.0;
  double loss = 0.0;
  for (int64_t r = 0; r < n; ++r) {
    double x[kFeat], z1[kHid], h1[kHid], z2[kHid], h2[kHid];
    for (int i = 0; i < kFeat; ++i) {
      double v = round ? (double)std::fmaf(feats[kFeat * r + i], model[kNA + i], model[kNB + i])
                       : (double)feats[kFeat * r + i] * model[kNA + i] + model[kNB + i];
      x[i] = rd(v);
    }
    for (int j = 0; j < kHid; ++j) {
      double s = model[kB1 + j];
      for (int i = 0; i < kFeat; ++i) s += W1[kFeat * j + i] * x[i];
      z1[j] = s;
      h1[j] = rd(s > 0.0 ? s : 0.0);
    }
    for (int k = 0; k < kHid; ++k) {
      double s = model[kB2 + k];
      for (int j = 0; j < kHid; ++j) s += W2[kHid * k + j] * h1[j];
      z2[k] = s;
      h2[k] = rd(s > 0.0 ? s : 0.0);
    }
    double y = model[kB3];
    for (int k = 0; k < kHid; ++k) y += w3[k] * h2[k];
    double res = (double)labels[r] - y;
    loss += res < 0.0 ? (tau - 1.0) * res : tau * res;
    double dy = (res < 0.0 ? 1.0 - tau : -tau) / (double)n;
    grad[kB3] += dy;
    double dz2[kHid];
    for (int k = 0; k < kHid; ++k) {
      grad[kW3 + k] += dy * h2[k];
      dz2[k] = z2[k] > 0.0 ? dy * w3[k] : 0.0;
      grad[kB2 + k] += dz2[k];
      for (int j = 0; j < kHid; ++j) grad[kW2 + kHid * k + j] += dz2[k] * h1[j];
    }
    for (int j = 0; j < kHid; ++j) {
      double dh = 0.0;
      for (int k = 0; k < kHid; ++k) dh += dz2[k] * W2[kHid * k + j];
      double dz1 = z1[j] > 0.0 ? dh : 0.0;
      grad[kB1 + j] += dz1;
      for (int i = 0; i < kFeat; ++i) grad[kW1 + kFeat * j + i] += dz1 * x[i];
    }
  }
  return loss / (double)n;
}

// One Adam step (Kingma & Ba 2015) on the first kParams entries, step t >= 1
void orc_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t t, double lr, double beta1,
                  double beta2, double eps) {
  double c1 = 1.0 - std::pow(beta1, (double)t), c2 = 1.0 - std::pow(beta2, (double)t);
  for (int i = 0; i < kParams; ++i) {
    double g = grad[i];
    double mi = beta1 * m[i] + (1.0 - beta1) * g;
    double vi = beta2 * v[i] + (1.0 - beta2) * g * g;
    m[i] = (float)mi;
    v[i] = (float)vi;
    params[i] = (float)(params[i] - lr * (mi / c1) / (std::sqrt(vi / c2) + eps));
  }
}

int32_t orc_walk(orc_tree* t, double theta) {
  if (!(theta > 0.0 && theta <= 1.0)) return ORC_E_INVALID;
  if (!t->have_moments) return ORC_E_STATE;
  t->mode = 0;
  t->theta = theta;
  run_walk(t);
  return ORC_OK;
}

int64_t orc_num_m2l(const orc_tree* t) { return (int64_t)t->m2l.size(); }
int64_t orc_num_p2p(const orc_tree* t) { return (int64_t)t->p2p.size(); }

void orc_get_lists(const orc_tree* t, int32_t* m2l_ab, int32_t* p2p_ab) {
  for (size_t i = 0; i < t->m2l.size(); ++i) {
    m2l_ab[2 * i] = t->m2l[i].first;
    m2l_ab[2 * i + 1] = t->m2l[i].second;
  }
  for (size_t i = 0; i < t->p2p.size(); ++i) {
    p2p_ab[2 * i] = t->p2p[i].first;
    p2p_ab[2 * i + 1] = t->p2p[i].second;
  }
}

int32_t orc_evaluate(orc_tree* t, int32_t variant, double G, double* ax, double* ay, double* az,
                     double* pot) {
  if (!t->have_lists) return ORC_E_STATE;
  if (variant < ORC_UC || variant > ORC_TCO) return ORC_E_INVALID;
  if (variant == ORC_TCO && t->general) return ORC_E_INVALID;  // eq. 8's tensor is printed for P = 3 only
  int64_t n = t->n;
  std::vector<double> gx(n, 0.0), gy(n, 0.0), gz(n, 0.0), ph(n, 0.0);
  // far field: every accepted pair, at every particle of both cells
  for (const auto& pr : t->m2l) {
    const Cell& CA = t->cells[pr.first];
    const Cell& CB = t->cells[pr.second];
    const Moments& A = t->mom[pr.first];
    const Moments& B = t->mom[pr.second];
    PairField pf;
    pair_field(*t, pr.first, pr.second, variant, pf);
    for (int64_t p = CA.begin; p < CA.begin + CA.count; ++p) {
      double xv[3] = {t->x[p] - A.Z[0], t->y[p] - A.Z[1], t->z[p] - A.Z[2]};
      double g[3], phi;
      pair_field_at(*t, pf, pr.first, pr.second, 0, xv, g, phi);
      gx[p] += g[0];
      gy[p] += g[1];
      gz[p] += g[2];
      ph[p] += phi;
    }
    for (int64_t p = CB.begin; p < CB.begin + CB.count; ++p) {
      double yv[3] = {t->x[p] - B.Z[0], t->y[p] - B.Z[1], t->z[p] - B.Z[2]};
      double g[3], phi;
      pair_field_at(*t, pf, pr.first, pr.second, 1, yv, g, phi);
      gx[p] += g[0];
      gy[p] += g[1];
      gz[p] += g[2];
      ph[p] += phi;
    }
  }
  // near field: every particle pair of every non-accepted leaf pair, once
  t->coincident = 0;
  for (const auto& pr : t->p2p) {
    const Cell& CA = t->cells[pr.first];
    const Cell& CB = t->cells[pr.second];
    bool self = pr.first == pr.second;
    for (int64_t i = CA.begin; i < CA.begin + CA.count; ++i) {
      int64_t jb = self ? i + 1 : CB.begin;
      for (int64_t j = jb; j < CB.begin + CB.count; ++j) {
        double dx = t->x[j] - t->x[i];
        double dy = t->y[j] - t->y[i];
        double dz = t->z[j] - t->z[i];
        double r2 = (dx * dx + dy * dy) + dz * dz;
        if (r2 == 0.0) {
          ++t->coincident;
          continue;
        }
        double s2 = r2 + t->eps2;  // softened distance squared
        double r = std::sqrt(s2);
        double r3 = s2 * r;
        // acceleration on i towards j and on j towards i
        gx[i] += t->m[j] * dx / r3;
        gy[i] += t->m[j] * dy / r3;
        gz[i] += t->m[j] * dz / r3;
        gx[j] -= t->m[i] * dx / r3;
        gy[j] -= t->m[i] * dy / r3;
        gz[j] -= t->m[i] * dz / r3;
        ph[i] -= t->m[j] / r;
        ph[j] -= t->m[i] / r;
      }
    }
  }
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = t->perm[s];
    ax[i] = G * gx[s];
    ay[i] = G * gy[s];
    az[i] = G * gz[s];
    if (pot) pot[i] = G * ph[s];
  }
  return ORC_OK;
}

int32_t orc_evaluate_sample(orc_tree* t, int32_t variant, double G, int64_t ns, const int64_t* idx,
                            double* ax, double* ay, double* az, double* pot) {
  if (!t->have_lists) return ORC_E_STATE;
  if (variant < ORC_UC || variant > ORC_TCO) return ORC_E_INVALID;
  if (variant == ORC_TCO && t->general) return ORC_E_INVALID;  // eq. 8's tensor is printed for P = 3 only
  int64_t n = t->n;
  // caller index -> sorted position, cell -> partners of each list
  std::vector<int64_t> pos(n);
  for (int64_t s = 0; s < n; ++s) pos[t->perm[s]] = s;
  size_t nc = t->cells.size();
  std::vector<std::vector<int32_t>> far(nc), near(nc);
  for (const auto& pr : t->m2l) {
    far[pr.first].push_back(pr.second);
    far[pr.second].push_back(pr.first);
  }
  for (const auto& pr : t->p2p) {
    near[pr.first].push_back(pr.second);
    if (pr.first != pr.second) near[pr.second].push_back(pr.first);
  }
  for (int64_t q = 0; q < ns; ++q) {
    if (idx[q] < 0 || idx[q] >= n) return ORC_E_INVALID;
    int64_t p = pos[idx[q]];
    double g[3] = {0.0, 0.0, 0.0}, ph = 0.0;
    // the leaf holding p, then every ancestor up to the root
    int32_t c = 0;
    std::vector<int32_t> chain{0};
    while (t->cells[c].nchild) {
      const Cell& C = t->cells[c];
      int32_t next = -1;
      for (int32_t k = C.child0; k < C.child0 + C.nchild; ++k)
        if (p >= t->cells[k].begin && p < t->cells[k].begin + t->cells[k].count) next = k;
      c = next;
      chain.push_back(c);
    }
    for (int32_t cell : chain) {
      for (int32_t other : far[cell]) {
        // the pair is stored once as (lower, higher); the lower index is the
        // field cell of eq. 3 and the higher that of eq. 4
        int32_t a = std::min(cell, other), b = std::max(cell, other);
        PairField pf;
        pair_field(*t, a, b, variant, pf);
        const Moments& own = t->mom[cell];
        double xv[3] = {t->x[p] - own.Z[0], t->y[p] - own.Z[1], t->z[p] - own.Z[2]};
        double gg[3], phi;
        pair_field_at(*t, pf, a, b, cell == a ? 0 : 1, xv, gg, phi);
        for (int d = 0; d < 3; ++d) g[d] += gg[d];
        ph += phi;
      }
    }
    int32_t leaf = chain.back();
    for (int32_t other : near[leaf]) {
      const Cell& O = t->cells[other];
      for (int64_t j = O.begin; j < O.begin + O.count; ++j) {
        double dx = t->x[j] - t->x[p];
        double dy = t->y[j] - t->y[p];
        double dz = t->z[j] - t->z[p];
        double r2 = (dx * dx + dy * dy) + dz * dz;
        if (r2 == 0.0) continue;
        double s2 = r2 + t->eps2;
        double r = std::sqrt(s2);
        double r3 = s2 * r;
        g[0] += t->m[j] * dx / r3;
        g[1] += t->m[j] * dy / r3;
        g[2] += t->m[j] * dz / r3;
        ph -= t->m[j] / r;
      }
    }
    ax[q] = G * g[0];
    ay[q] = G * g[1];
    az[q] = G * g[2];
    if (pot) pot[q] = G * ph;
  }
  return ORC_OK;
}

int32_t orc_evaluate_targets(orc_tree* t, int32_t variant, double G, double* ax, double* ay,
                             double* az, double* pot) {
  if (!t->have_lists) return ORC_E_STATE;
  if (variant < ORC_UC || variant > ORC_TCO) return ORC_E_INVALID;
  if (variant == ORC_TCO && t->general) return ORC_E_INVALID;  // eq. 8's tensor is printed for P = 3 only
  int64_t n = t->n;
  int64_t nc = (int64_t)t->cells.size();
  std::vector<double> gx(n, 0.0), gy(n, 0.0), gz(n, 0.0), ph(n, 0.0);
  // the partners of every cell, in list order
  std::vector<std::vector<int32_t>> far(nc), near(nc);
  for (const auto& pr : t->m2l) {
    far[pr.first].push_back(pr.second);
    far[pr.second].push_back(pr.first);
  }
  for (const auto& pr : t->p2p) {
    near[pr.first].push_back(pr.second);
    if (pr.first != pr.second) near[pr.second].push_back(pr.first);
  }
  // far field, one level at a time: the lower index of a pair is the field
  // cell of eq. 3, the higher that of eq. 4 (as in orc_evaluate)
  int32_t depth = orc_depth(t);
  for (int32_t lev = 0; lev <= depth; ++lev) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ci = 0; ci < nc; ++ci) {
      const Cell& C = t->cells[ci];
      if (C.level != lev) continue;
      const Moments& own = t->mom[ci];
      for (int32_t other : far[ci]) {
        int32_t a = std::min((int32_t)ci, other), b = std::max((int32_t)ci, other);
        PairField pf;
        pair_field(*t, a, b, variant, pf);
        for (int64_t p = C.begin; p < C.begin + C.count; ++p) {
          double xv[3] = {t->x[p] - own.Z[0], t->y[p] - own.Z[1], t->z[p] - own.Z[2]};
          double g[3], phi;
          pair_field_at(*t, pf, a, b, ci == a ? 0 : 1, xv, g, phi);
          gx[p] += g[0];
          gy[p] += g[1];
          gz[p] += g[2];
          ph[p] += phi;
        }
      }
    }
  }
  // near field: every leaf sums its partners' particles onto its own
  int64_t skipped = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : skipped)
  for (int64_t ci = 0; ci < nc; ++ci) {
    const Cell& C = t->cells[ci];
    if (!is_leaf(C)) continue;
    for (int32_t other : near[ci]) {
      const Cell& O = t->cells[other];
      for (int64_t i = C.begin; i < C.begin + C.count; ++i) {
        for (int64_t j = O.begin; j < O.begin + O.count; ++j) {
          double dx = t->x[j] - t->x[i];
          double dy = t->y[j] - t->y[i];
          double dz = t->z[j] - t->z[i];
          double r2 = (dx * dx + dy * dy) + dz * dz;
          if (r2 == 0.0) {
            if (j != i) ++skipped;
            continue;
          }
          double s2 = r2 + t->eps2;
          double r = std::sqrt(s2);
          double r3 = s2 * r;
          gx[i] += t->m[j] * dx / r3;
          gy[i] += t->m[j] * dy / r3;
          gz[i] += t->m[j] * dz / r3;
          ph[i] -= t->m[j] / r;
        }
      }
    }
  }
  t->coincident = skipped / 2;  // each coincident pair was seen from both sides
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = t->perm[s];
    ax[i] = G * gx[s];
    ay[i] = G * gy[s];
    az[i] = G * gz[s];
    if (pot) pot[i] = G * ph[s];
  }
  return ORC_OK;
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

int64_t orc_num_coincident(const orc_tree* t) { return t->coincident; }

int32_t orc_solve(int64_t n, const double* x, const double* y, const double* z, const double* m,
                  double theta, int32_t n_crit, int32_t variant, double G, double* ax, double* ay,
                  double* az, double* pot) {
  if (!(theta > 0.0 && theta <= 1.0)) return ORC_E_INVALID;
  int32_t st = ORC_OK;
  orc_tree* t = orc_build_tree(n, x, y, z, m, n_crit, kMaxLevel, &st);
  if (!t) return st;
  orc_compute_moments(t);
  st = orc_walk(t, theta);
  if (st == ORC_OK) st = orc_evaluate(t, variant, G, ax, ay, az, pot);
  orc_free(t);
  return st;
}

int32_t orc_direct(int64_t n, const double* x, const double* y, const double* z, const double* m,
                   int64_t ntarget, const int64_t* targets, double G, double* ax, double* ay,
                   double* az, double* pot, double* gabs) {
  return orc_direct_softened(n, x, y, z, m, ntarget, targets, G, 0.0, ax, ay, az, pot, gabs);
}

int32_t orc_direct_softened(int64_t n, const double* x, const double* y, const double* z, const double* m,
                            int64_t ntarget, const int64_t* targets, double G, double eps, double* ax,
                            double* ay, double* az, double* pot, double* gabs) {
  if (n < 1 || ntarget < 0 || !(eps >= 0.0)) return ORC_E_INVALID;
  double eps2 = eps * eps;
  for (int64_t q = 0; q < ntarget; ++q) {
    int64_t i = targets ? targets[q] : q;
    if (i < 0 || i >= n) return ORC_E_INVALID;
    double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0, sa = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double dx = x[j] - x[i];
      double dy = y[j] - y[i];
      double dz = z[j] - z[i];
      double r2 = (dx * dx + dy * dy) + dz * dz;
      if (r2 == 0.0) continue;
      double s2 = r2 + eps2;
      double r = std::sqrt(s2);
      double r3 = s2 * r;
      sx += m[j] * dx / r3;
      sy += m[j] * dy / r3;
      sz += m[j] * dz / r3;
      sp -= m[j] / r;
      sa += m[j] / s2;
    }
    ax[q] = G * sx;
    ay[q] = G * sy;
    az[q] = G * sz;
    if (pot) pot[q] = G * sp;
    if (gabs) gabs[q] = G * sa;
  }
  return ORC_OK;
}

int32_t orc_set_order_form(orc_tree* t, int32_t P, int32_t general) {
  if (P < 2 || P > kMaxOrder || (P != 3 && !general)) return ORC_E_INVALID;
  t->order = P;
  t->general = general != 0;
  if (t->have_moments && t->general)
    for (size_t ci = 0; ci < t->cells.size(); ++ci)
      moments_general(*t, t->cells[ci].begin, t->cells[ci].count, P, t->mom[ci]);
  return ORC_OK;
}

int32_t orc_set_order(orc_tree* t, int32_t P) { return orc_set_order_form(t, P, P != 3); }

int32_t orc_num_multi_indices(int32_t n) { return n < 0 || n > kMaxOrder + 1 ? 0 : kMI.count[n + 1]; }

void orc_multi_indices(int32_t n, int32_t* exps) {
  for (int g = 0; g < kMI.count[n + 1]; ++g)
    for (int i = 0; i < 3; ++i) exps[3 * g + i] = kMI.e[g][i];
}

void orc_greens_general(const double* R3, double eps, int32_t n, double* D) {
  std::vector<double> v;
  greens_general(R3, eps * eps, n, v);
  std::copy(v.begin(), v.end(), D);
}

int32_t orc_set_softening(orc_tree* t, double eps) {
  if (!(eps >= 0.0) || !std::isfinite(eps)) return ORC_E_INVALID;
  t->eps2 = eps * eps;
  return ORC_OK;
}

void orc_greens_softened(const double* R3, double eps, double* D0, double* D1, double* D2, double* D3,
                         double* D4, double* D4p) {
  Greens g;
  greens_softened(R3, eps * eps, g, true);
  *D0 = g.D0;
  std::memcpy(D1, g.D1, sizeof(g.D1));
  std::memcpy(D2, g.D2, sizeof(g.D2));
  std::memcpy(D3, g.D3, sizeof(g.D3));
  std::memcpy(D4, g.D4, sizeof(g.D4));
  std::memcpy(D4p, g.D4p, sizeof(g.D4p));
}

void orc_greens(const double* R3, double* D0, double* D1, double* D2, double* D3, double* D4,
                double* D4p) {
  Greens g;
  greens(R3, g, true);
  *D0 = g.D0;
  std::memcpy(D1, g.D1, sizeof(g.D1));
  std::memcpy(D2, g.D2, sizeof(g.D2));
  std::memcpy(D3, g.D3, sizeof(g.D3));
  std::memcpy(D4, g.D4, sizeof(g.D4));
  std::memcpy(D4p, g.D4p, sizeof(g.D4p));
}

void orc_cluster_moments(int64_t n, const double* x, const double* y, const double* z,
                         const double* m, double* out21) {
  int32_t st;
  orc_tree* t = orc_build_tree(n, x, y, z, m, (int32_t)n, 0, &st);  // one leaf
  if (!t) return;
  // keep caller order inside the single leaf so the sums run in caller order
  for (int64_t i = 0; i < n; ++i) {
    t->x[i] = x[i];
    t->y[i] = y[i];
    t->z[i] = z[i];
    t->m[i] = m[i];
    t->perm[i] = i;
  }
  orc_compute_moments(t);
  orc_get_moments(t, out21);
  orc_free(t);
}

void orc_pair_far_order(int32_t order, int32_t general, int64_t nA, const double* xa, const double* ya, const double* za,
                        const double* ma, int64_t nB, const double* xb, const double* yb, const double* zb,
                        const double* mb, int32_t variant, double* gA, double* phiA, double* gB, double* phiB) {
  // the two clusters as cells 0 and 1 of one tree, particles in caller order
  orc_tree t;
  t.n = nA + nB;
  t.order = order;
  t.general = general != 0 || order != 3;
  t.x.assign(xa, xa + nA);
  t.y.assign(ya, ya + nA);
  t.z.assign(za, za + nA);
  t.m.assign(ma, ma + nA);
  t.x.insert(t.x.end(), xb, xb + nB);
  t.y.insert(t.y.end(), yb, yb + nB);
  t.z.insert(t.z.end(), zb, zb + nB);
  t.m.insert(t.m.end(), mb, mb + nB);
  t.cells.push_back(Cell{0, 0, nA, -1, -1, 0, 0});
  t.cells.push_back(Cell{0, nA, nB, -1, -1, 0, 0});
  for (int c = 0; c < 2; ++c) {
    const Cell& C = t.cells[c];
    Moments mo;
    for (int64_t p = C.begin; p < C.begin + C.count; ++p) {
      mo.M += t.m[p];
      mo.S[0] += t.m[p] * t.x[p];
      mo.S[1] += t.m[p] * t.y[p];
      mo.S[2] += t.m[p] * t.z[p];
    }
    for (int d = 0; d < 3; ++d) mo.Z[d] = mo.S[d] / mo.M;
    moments_about(t, C.begin, C.count, mo);
    if (t.general) moments_general(t, C.begin, C.count, order, mo);
    t.mom.push_back(mo);
  }
  const Moments& A = t.mom[0];
  const Moments& B = t.mom[1];
  PairField pf;
  pair_field(t, 0, 1, variant, pf);
  for (int64_t p = 0; p < nA; ++p) {
    double xv[3] = {xa[p] - A.Z[0], ya[p] - A.Z[1], za[p] - A.Z[2]};
    double g[3], phi;
    pair_field_at(t, pf, 0, 1, 0, xv, g, phi);
    for (int d = 0; d < 3; ++d) gA[3 * p + d] = g[d];
    if (phiA) phiA[p] = phi;
  }
  for (int64_t p = 0; p < nB; ++p) {
    double yv[3] = {xb[p] - B.Z[0], yb[p] - B.Z[1], zb[p] - B.Z[2]};
    double g[3], phi;
    pair_field_at(t, pf, 0, 1, 1, yv, g, phi);
    for (int d = 0; d < 3; ++d) gB[3 * p + d] = g[d];
    if (phiB) phiB[p] = phi;
  }
}

void orc_pair_far(int64_t nA, const double* xa, const double* ya, const double* za,
                  const double* ma, int64_t nB, const double* xb, const double* yb,
                  const double* zb, const double* mb, int32_t variant, double* gA, double* phiA,
                  double* gB, double* phiB) {
  orc_pair_far_order(3, 0, nA, xa, ya, za, ma, nB, xb, yb, zb, mb, variant, gA, phiA, gB, phiB);
}

}  // extern "C"
