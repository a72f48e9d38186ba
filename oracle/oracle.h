/*
 * CPU FP64 oracle for the angular-momentum-conserving Cartesian FMM
 * (Marcello 2017, "A Very Fast And Angular Momentum Conserving Tree Code").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU library is judged against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the GPU solver never
 * calls, links or includes anything from here, and nothing here is shared
 * with it.
 *
 * Every routine follows the paper's definitions directly (full index loops,
 * no symmetry packing, no blocking):
 *   - octree with at most n_crit particles per leaf          (Sec. 2)
 *   - centre of mass Z and R_max of every cell               (Sec. 2, opening criterion)
 *   - moments M, M_ij, M_ijk about Z                          (Sec. 2, eqs. 1, quad, octupole def.)
 *   - Green's function derivatives D .. D_ijk (printed), D_ijkl (fourth
 *     derivative, Sec. 2 eq. 7 text; closed form derived), D'_ijkl (eq. 8)
 *   - far field of an accepted pair, eqs. 2-4, evaluated at every particle
 *   - torque correction F_c, eq. 7 with the prefactor of the appendix (1/6)
 *   - direct near field between particles of non-accepted leaf pairs
 *
 * All arrays are host memory owned by the caller.  Functions return 0 on
 * success and a negative code on invalid input (see ORC_E_*).
 */
#ifndef AMFMM_ORACLE_H
#define AMFMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_NONFINITE (-2)
#define ORC_E_STATE (-5)

/* variants of Sec. 3: UC = uncorrected, TC = eq. 7, TCO = eq. 8 */
#define ORC_UC 0
#define ORC_TC 1
#define ORC_TCO 2

typedef struct orc_tree orc_tree;

/* Steps: bounding cube + Morton keys, stable sort, octree (Sec. 2).
 * n >= 1, all inputs finite, m > 0.  max_level <= 21.  Returns NULL and sets
 * *status on invalid input. */
orc_tree* orc_build_tree(int64_t n, const double* x, const double* y, const double* z,
                         const double* m, int32_t n_crit, int32_t max_level, int32_t* status);
void orc_free(orc_tree* t);

int64_t orc_num_cells(const orc_tree* t);
int32_t orc_depth(const orc_tree* t); /* deepest level present */
/* bounding cube: lo[3], side, scale */
void orc_get_cube(const orc_tree* t, double* lo3, double* side, double* scale);
/* sorted keys and permutation: perm[s] = caller index of the s-th sorted particle */
void orc_get_keys(const orc_tree* t, uint64_t* keys, int64_t* perm);
/* cells in (level, first particle) order */
void orc_get_cells(const orc_tree* t, int32_t* level, int64_t* begin, int64_t* count,
                   int32_t* parent, int32_t* child0, int32_t* nchild);

/* Upward pass: M, Z, R_max, M_ij, M_ijk of every cell. */
int32_t orc_compute_moments(orc_tree* t);
/* per cell 21 doubles: M, Zx,Zy,Zz, Rmax, M_xx,M_xy,M_xz,M_yy,M_yz,M_zz,
 * M_xxx,M_xxy,M_xxz,M_xyy,M_xyz,M_xzz,M_yyy,M_yyz,M_yzz,M_zzz */
void orc_get_moments(const orc_tree* t, double* out21);

/* Dual tree walk under the opening criterion (Sec. 2).  theta in (0,1]. */
int32_t orc_walk(orc_tree* t, double theta);
/* The same walk with the error-estimate criterion: a pair is accepted when
 * d > 0, R_A + R_B <= theta_max d and, with q = (R_A + R_B)/d and
 * e = q^3 / d^2 (the force-error scale of a quadrupole-order pair per unit
 * source mass), e M_B <= eps s_A and e M_A <= eps s_B, where s is a cell's
 * field scale: the smallest |gmag| over its particles, but at least 0.1 times
 * their mean (sums taken leaf-sequentially in key order and over children in
 * octant order).  gmag: per-particle field magnitudes, caller order. */
int32_t orc_walk_field(orc_tree* t, double eps, double theta_max, const double* gmag);
/* Walk with the multipole error estimate (see oracle.cpp): per-pair error
 * from the source's traceless octupole and quadrupole norms and both cells'
 * extents, against eps times each cell's field scale (as orc_walk_field). */
int32_t orc_walk_multipole(orc_tree* t, double eps, double theta_max, const double* gmag);
/* Quantised traceless quadrupole and octupole norm levels of every cell. */
void orc_multipole_levels(const orc_tree* t, int32_t* k2, int32_t* k3);
int64_t orc_num_m2l(const orc_tree* t);
int64_t orc_num_p2p(const orc_tree* t);
/* unordered pairs {a,b}: m2l with a<b, p2p with a<=b, each list sorted */
void orc_get_lists(const orc_tree* t, int32_t* m2l_ab, int32_t* p2p_ab);

/* Evaluation: far field (eqs. 2-4) + correction of the variant + near field.
 * Outputs in caller order, scaled by G.  pot may be NULL. */
int32_t orc_evaluate(orc_tree* t, int32_t variant, double G, double* ax, double* ay, double* az,
                     double* pot);
/* The same evaluation at a sample of particles only (caller indices idx[0..ns)),
 * for checks at sizes where evaluating every particle is too slow.  Needs the
 * walk.  Outputs are per sample entry. */
int32_t orc_evaluate_sample(orc_tree* t, int32_t variant, double G, int64_t ns, const int64_t* idx,
                            double* ax, double* ay, double* az, double* pot);
/* The same evaluation organised by target, for timing on many cores: the far
 * pairs of every cell are applied to its own particles one tree level at a
 * time (cells of a level hold disjoint particles), the near field of every
 * leaf is summed over its own particles only.  Each particle's sums run in an
 * order fixed by the lists, so the result does not depend on the number of
 * threads (OpenMP when built with it; serial otherwise).  Equal to
 * orc_evaluate up to summation order. */
int32_t orc_evaluate_targets(orc_tree* t, int32_t variant, double G, double* ax, double* ay,
                             double* az, double* pot);
/* threads orc_evaluate_targets runs on (1 in a build without OpenMP) */
int32_t orc_num_threads(void);
/* Plummer softening of the Green's function, g = -1/sqrt(R^2 + eps^2) (Sec. 4:
 * the correction carries over to any g of R alone), for the far field (the
 * derivatives of the softened g), the near field and every later evaluation
 * of the tree; eps = 0 restores -1/R.  Pairs at r = 0 are still skipped. */
int32_t orc_set_softening(orc_tree* t, double eps);
/* number of particle pairs skipped because they coincide (r == 0, i != j) */
int64_t orc_num_coincident(const orc_tree* t);

/* Whole solve in one call (build, moments, walk, evaluate). */
int32_t orc_solve(int64_t n, const double* x, const double* y, const double* z, const double* m,
                  double theta, int32_t n_crit, int32_t variant, double G, double* ax, double* ay,
                  double* az, double* pot);

/* Direct summation (the exact result the method approximates).  For each
 * target index t (all particles when targets == NULL, ntarget = n) returns the
 * acceleration, the potential and gabs = sum_j m_j / r^2 (the magnitude scale
 * of the sum).  Coincident pairs are skipped. */
int32_t orc_direct(int64_t n, const double* x, const double* y, const double* z, const double* m,
                   int64_t ntarget, const int64_t* targets, double G, double* ax, double* ay,
                   double* az, double* pot, double* gabs);
/* The same with the softened Green's function (eps >= 0; gabs = sum_j m_j /
 * (r^2 + eps^2)). */
int32_t orc_direct_softened(int64_t n, const double* x, const double* y, const double* z, const double* m,
                            int64_t ntarget, const int64_t* targets, double G, double eps, double* ax,
                            double* ay, double* az, double* pot, double* gabs);

/* Building blocks exposed for the pins. */
/* full tensors: D0[1], D1[3], D2[9], D3[27], D4[81], D4p[81] at R (Sec. 2) */
void orc_greens(const double* R3, double* D0, double* D1, double* D2, double* D3, double* D4,
                double* D4p);
/* the same tensors of the softened g = -1/sqrt(R^2 + eps^2) */
void orc_greens_softened(const double* R3, double eps, double* D0, double* D1, double* D2, double* D3,
                         double* D4, double* D4p);
/* Moments of one cluster (as one cell): out21 as in orc_get_moments. */
void orc_cluster_moments(int64_t n, const double* x, const double* y, const double* z,
                         const double* m, double* out21);
/* One accepted pair (cluster A = field of eq. 3, cluster B = field of eq. 4),
 * evaluated at every particle of both, with the correction of the variant.
 * Outputs are accelerations (3 per particle, interleaved xyz) and potentials. */
void orc_pair_far(int64_t nA, const double* xa, const double* ya, const double* za,
                  const double* ma, int64_t nB, const double* xb, const double* yb,
                  const double* zb, const double* mb, int32_t variant, double* gA, double* phiA,
                  double* gB, double* phiB);
/* The same at expansion order P (the appendix's general form when general
 * != 0 or P != 3; P = 3 otherwise is orc_pair_far; TCO only in the printed
 * form). */
void orc_pair_far_order(int32_t order, int32_t general, int64_t nA, const double* xa, const double* ya, const double* za,
                        const double* ma, int64_t nB, const double* xb, const double* yb, const double* zb,
                        const double* mb, int32_t variant, double* gA, double* phiA, double* gB, double* phiB);
/* Expansion order P of the tree's evaluation (2 <= P <= 6; default 3, the
 * printed equations; other orders use the appendix's general expansion and
 * correction, UC and TC only).  Recomputes the moments it needs. */
int32_t orc_set_order(orc_tree* t, int32_t P);
/* The same with the form chosen: general != 0 evaluates the appendix's
 * general form also at P = 3 (a check of it against the printed equations). */
int32_t orc_set_order_form(orc_tree* t, int32_t P, int32_t general);
/* Multi-indices (a, b, c) of order <= n in the graded order the general form
 * uses (count, then 3 ints each), and D_alpha(R) of the softened Green's
 * function (eps = 0: -1/R) for |alpha| <= n in that order. */
int32_t orc_num_multi_indices(int32_t n);
void orc_multi_indices(int32_t n, int32_t* exps);
void orc_greens_general(const double* R3, double eps, int32_t n, double* D);

/* ---- learned pair selection (not in the paper; see the notes in oracle.cpp) ----
 * Model: ORC_MLP_MODEL floats (network, then feature normalisation a[8], b[8]
 * and the training range lo[8], hi[8]); the trainable parameters are its first
 * ORC_MLP_PARAMS entries. */
#define ORC_MLP_PARAMS 4801
#define ORC_MLP_MODEL 4833
/* Walk on the multipole estimate (as orc_walk_multipole) whose accept
 * decision asks the network where the estimate lies near the bound (rho in
 * (1/4, 2], rho the larger of e / (eps s d^6) over the two cells) for pairs
 * with N_A N_B >= min_work and features inside the training range; below the
 * band pairs are accepted, above it opened, other pairs in it take rho <= 1.
 * model == NULL gives the opening-angle walk with theta. */
int32_t orc_walk_learned(orc_tree* t, double eps, double theta_max, double theta, const double* gmag,
                         const float* model, int64_t min_work);
/* Features (8 floats per pair) and labels (log2 error factor) of cell pairs
 * (a, b), 2 int32 per pair; labels need moments and a != b, d > 0.
 * orc_pair_errors: the method's largest error from the pair alone on a
 * (err[2k]) and on b (err[2k+1]), the measurements behind the labels and the
 * fit of the multipole estimate's weights. */
void orc_pair_features(const orc_tree* t, int64_t np, const int32_t* pairs, float* feats);
int32_t orc_pair_labels(const orc_tree* t, int32_t variant, int64_t np, const int32_t* pairs,
                        double* labels);
int32_t orc_pair_errors(const orc_tree* t, int32_t variant, int64_t np, const int32_t* pairs, double* err);
/* The multipole estimate's weights w1..w5 (5 doubles). */
void orc_multipole_weights(double* w);
/* BF16 rounding (nearest, ties to even) and the piecewise-linear log2 that
 * the features and the decision use. */
float orc_bf16_round(float v);
double orc_plog2(double x);
/* FP32 inference exactly as the walk runs it. */
void orc_mlp_predict(const float* model, int64_t n, const float* feats, float* y);
/* Mean pinball loss at quantile tau and its gradient (ORC_MLP_PARAMS doubles). */
double orc_mlp_grad(const float* model, int64_t n, const float* feats, const float* labels, double tau,
                    int32_t round, double* grad);
/* One Adam step (t >= 1) on the ORC_MLP_PARAMS parameters. */
void orc_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t t, double lr, double beta1,
                  double beta2, double eps);

#ifdef __cplusplus
}
#endif
#endif
