/*
 * amfmm: angular-momentum-conserving Cartesian fast multipole gravity solver
 * for AMD Instinct MI355X (gfx950), after Marcello 2017, "A Very Fast And
 * Angular Momentum Conserving Tree Code" (a modification of Dehnen's symmetric
 * Cartesian FMM).
 *
 * C ABI of libamfmm_hip.so.  Every array argument named as a device pointer is
 * memory on the current HIP device, owned by the caller; the library never
 * frees it and never keeps it beyond the call.  All work is enqueued on the
 * stream given to amfmm_create; calls return after enqueueing, except where a
 * size must be read back (validation, tree levels, walk levels), which
 * synchronises that stream.  A context is not thread-safe: use one per stream.
 * Functions return AMFMM_OK (0) or a negative amfmm_status; nothing throws
 * across this boundary, and amfmm_last_error() describes the last failure.
 */
#ifndef AMFMM_H
#define AMFMM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMFMM_OK = 0,
  AMFMM_E_INVALID = -1,   /* bad size, theta outside (0,1], m <= 0, bad option */
  AMFMM_E_NONFINITE = -2, /* a NaN or infinite position or mass */
  AMFMM_E_OOM = -3,       /* device allocation failed or exceeds the context cap */
  AMFMM_E_HIP = -4,       /* a HIP runtime call failed */
  AMFMM_E_STATE = -5      /* call order violated (e.g. moments before a tree) */
} amfmm_status;

/* Variants of Sec. 3: UC = the uncorrected method, TC = torque correction of
 * eq. 7, TCO = the alternative correction of eq. 8. */
typedef enum { AMFMM_UC = 0, AMFMM_TC = 1, AMFMM_TCO = 2 } amfmm_variant;

/* Arithmetic of the near field and of the far-field coefficients.
 * FP64: everything in double precision.
 * MIXED: near-field pair terms and far-field coefficient terms in FP32, on
 * offsets taken relative to cell centres (each offset and the centre-to-centre
 * vector formed in FP64, then rounded).  Per-particle near-field sums are
 * compensated FP64 sums: blocks of at most 32 FP32 terms are added to an FP64
 * accumulator with TwoSum, the rounding errors collected in a compensation
 * term added back at the end.  Far-field coefficients are summed per cell in
 * FP32 blocks of at most 8 terms added to FP64.  Centres of mass, the moment
 * reduction, the correction of eq. 7/8, the push-down and the evaluation at
 * the particles stay in FP64. */
typedef enum { AMFMM_FP64 = 0, AMFMM_MIXED = 1 } amfmm_precision;

/* Accept/open decision of the walk.
 * GEOMETRIC: the opening criterion of Sec. 2, |Z_A - Z_B| >= (R_A + R_B)/theta.
 * ESTIMATE: an error-estimate criterion (the role of the error-based pair
 *   selection that Sec. 2 cites): with q = (R_A + R_B)/d and field scales s
 *   (per cell: the smallest field estimate over its particles, at least 0.1
 *   times their mean), a pair is accepted when q <= theta_max and
 *   q^3 M_B / d^2 <= error_tol s_A and q^3 M_A / d^2 <= error_tol s_B.
 * LEARNED: MULTIPOLE (below), with a network (amfmm_set_model) deciding the
 *   pairs whose estimate lies near the bound: with rho the larger of
 *   e_A / (error_tol s_A) and e_B / (error_tol s_B), rho <= 1/4 accepts and
 *   rho > 2 opens; in between, for pairs with N_A N_B >= learned_min_work and
 *   features inside the model's training range, the network predicts log2 of
 *   the ratio of the method's error to the estimate and the pair is accepted
 *   when that prediction is at most -plog2(rho) (the error then predicted
 *   stays within error_tol s); other pairs take the MULTIPOLE decision rho <= 1.
 * MULTIPOLE: an error-estimate criterion from the parts a third-order
 *   expansion drops: with k2, k3 the Frobenius norms of the source's traceless
 *   quadrupole and octupole in units of M R_max^2 and M R_max^3 (held to the
 *   nearest 1/128), the error on A from B is estimated as
 *   e_A = ((w3 k3_B R_B^3 + w2 k2_B R_B^2 R_A + w1 R_A^3) d + w4 R_B^4 + w5 R_A^4) M_B / d^6
 *   (w1..w5 = 1.326, 4.095, 0.285, 0.1416, 1.618: least squares in log space
 *   on the largest error this method makes from each accepted pair of
 *   geometric walks of a 65536-particle Plummer sphere at theta 0.4, 0.6 and
 *   0.8); a pair is accepted when (R_A + R_B) <= theta_max d,
 *   e_A <= error_tol s_A and e_B <= error_tol s_B.
 * Every rule is a function of the unordered pair, so pairwise momentum
 * conservation holds.  Without a field estimate (amfmm_set_field_estimate),
 * and for LEARNED without a model, the geometric rule is used. */
typedef enum { AMFMM_GEOMETRIC = 0, AMFMM_ESTIMATE = 1, AMFMM_LEARNED = 2, AMFMM_MULTIPOLE = 3 } amfmm_criterion;

typedef struct {
  int32_t n_crit;     /* most particles in a leaf; the paper runs 25 (Sec. 2) */
  int32_t variant;    /* amfmm_variant */
  int32_t precision;  /* amfmm_precision */
  int32_t criterion;  /* amfmm_criterion */
  double G;           /* gravitational constant applied to all outputs */
  double error_tol;   /* ESTIMATE / LEARNED / MULTIPOLE: accepted pair error relative to the field scale */
  double theta_max;   /* ESTIMATE / LEARNED / MULTIPOLE: pairs with (R_A+R_B)/d > theta_max always open */
  int64_t max_bytes;  /* cap on device scratch owned by the context (0 = no cap) */
  int64_t list_bytes; /* device bytes the interaction lists of one batch may take
                         (0 = automatic: two fifths of the free device memory
                         plus the lists and staging room the context already
                         holds); when the whole tree's lists would not fit, or
                         a device allocation fails during the whole walk,
                         amfmm_solve_gravity walks and evaluates the tree in
                         batches of subtrees, with the same pairs */
  int64_t learned_min_work; /* LEARNED: the network decides pairs with N_A N_B >=
                               this (default 262144); smaller pairs, where a network
                               evaluation (about 9 kFLOP) costs more than the work
                               it can save, take the multipole estimate's decision */
  double softening;   /* Plummer softening length eps >= 0 of the Green's function
                         g = -1/sqrt(R^2 + eps^2) (Sec. 4: the correction holds for
                         any g of the distance alone): the far-field derivatives, the
                         correction, the near field and amfmm_direct use it; 0 (the
                         default) is the plain -1/R.  Pairs at r = 0 are skipped
                         either way.  The walk's criteria and the learned features and
                         labels do not depend on it. */
  int32_t order;      /* expansion order P of the far field (appendix: the Green's
                         function expanded to order P in both cells' offsets, with the
                         corrective force of order P that cancels each pair's torque):
                         3 (default) is eqs. 2-4 and 7/8 as printed; 4 adds the octupole
                         to the field and the hexadecapole (and the quadrupole-quadrupole
                         term) to the correction, UC or TC (eq. 8's tensor is printed for
                         P = 3 only); its far field, push-down and evaluation at the
                         particles are FP64 at either precision (MIXED then makes the near
                         field's pair terms FP32); other values are AMFMM_E_INVALID.  The
                         walk's criteria are unchanged; amfmm_solve_gravity_noalloc takes
                         order 3 only. */
} amfmm_options;

typedef struct amfmm_ctx amfmm_ctx;

/* Fills *opt with n_crit = 25, TC, FP64, geometric, G = 1, error_tol = 1e-4,
 * theta_max = 1, max_bytes = 0, list_bytes = 0, learned_min_work = 262144,
 * softening = 0, order = 3. */
int amfmm_default_options(amfmm_options* opt);

/* Creates a context bound to hip_stream (a hipStream_t; NULL = null stream)
 * on the current device.  The context owns all scratch. */
int amfmm_create(const amfmm_options* opt, void* hip_stream, amfmm_ctx** out);
int amfmm_destroy(amfmm_ctx* ctx);
/* Per-particle field estimates for the ESTIMATE, LEARNED and MULTIPOLE criteria, e.g. the
 * accelerations of the previous time step or of a cheaper solve: device
 * pointers to n doubles in caller order, either the three components (gx, gy,
 * gz) or magnitudes in gx with gy = gz = NULL.  The arrays are read during the
 * next walks and must stay valid until they return.  gx = NULL clears them. */
int amfmm_set_field_estimate(amfmm_ctx* ctx, const double* gx, const double* gy, const double* gz);
/* Rebinds the context to another stream of the same device. */
int amfmm_set_stream(amfmm_ctx* ctx, void* hip_stream);

/* Sec. 2, the octree: bounding cube, 63-bit Morton keys (21 bits per
 * coordinate), stable radix sort by key, and cells that split while they hold
 * more than n_crit particles (below level 21).  x,y,z,m: device pointers to n
 * doubles each (SoA, any order); 1 <= n < 2^31, all finite, m > 0.  Inputs are
 * copied into sorted order; the caller's arrays are only read. */
int amfmm_build_tree(amfmm_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                     const double* m);

/* Sec. 2, upward pass: mass M (eq. 1), centre of mass Z, quadrupole M_ij (eq.
 * quad) and octupole M_ijk about Z, and R_max (largest particle distance to Z)
 * of every cell.  Needs amfmm_build_tree, else AMFMM_E_STATE. */
int amfmm_compute_moments(amfmm_ctx* ctx);

/* Sec. 2, interaction selection: a symmetric dual walk accepting cell pairs
 * with |Z_A - Z_B| >= (R_A,max + R_B,max)/theta (far field), leaf pairs that
 * fail go to direct summation.  theta in (0,1].  Needs moments. */
int amfmm_walk(amfmm_ctx* ctx, double theta);

/* Far field (eqs. 2-4 with the correction of the variant, eq. 7 or 8) pushed
 * down to the particles, plus the direct near field.  Writes accelerations
 * (device pointers ax, ay, az; n doubles each, caller order) and potentials
 * (pot, may be NULL), scaled by G.  The potential excludes the self term and
 * the correction (a force only).  Needs the walk. */
int amfmm_evaluate(amfmm_ctx* ctx, double* ax, double* ay, double* az, double* pot);

/* The whole solve: build_tree + compute_moments + walk + evaluate. */
int amfmm_solve_gravity(amfmm_ctx* ctx, int64_t n, const double* x, const double* y,
                        const double* z, const double* m, double theta, double* ax, double* ay,
                        double* az, double* pot);

/* Time integration with the solver's forces (Sec. 1 and Sec. 4: the torque
 * correction conserves angular momentum when every particle takes the same
 * time step): `steps` kick-drift-kick leapfrog steps of dt,
 *   v += (dt/2) a;  x += dt v;  a = solve(x);  v += (dt/2) a,
 * in place on the device arrays x, y, z, vx, vy, vz (n doubles each, caller
 * order) with the masses m, the opening angle theta and the context's
 * options (variant, precision, criterion, field estimate).  On entry ax, ay,
 * az must hold the accelerations at x, y, z (as amfmm_solve_gravity returns
 * them); on return they hold those at the new positions.  The positions are
 * validated at every solve (a non-finite position stops the integration with
 * AMFMM_E_NONFINITE after the steps already taken).  steps >= 0, dt finite. */
int amfmm_leapfrog(amfmm_ctx* ctx, int64_t n, double* x, double* y, double* z, double* vx, double* vy,
                   double* vz, const double* m, double theta, double dt, int32_t steps, double* ax,
                   double* ay, double* az);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as amfmm_solve_gravity (same arguments, outputs to rounding: a cell's
 * pairs may be summed in another order), with every scratch buffer carved from
 * one static device array of 256 MiB that the library holds on each device it
 * runs on until the process ends.  It calls no hipMalloc, hipFree or other
 * allocating routine and records no timing events.  n may be at most 2^18
 * (else AMFMM_E_INVALID); a solve whose scratch (particles, cells, interaction
 * lists, walk staging) would outgrow the array returns AMFMM_E_OOM: near that
 * size, small opening angles or tight error tolerances can (the geometric
 * theta = 0.5 solve of 2^18 particles fits).  The context's own
 * buffers are set aside for the call: afterwards it holds no tree, lists or
 * phase times (introspection returns AMFMM_E_STATE) and the next
 * amfmm_solve_gravity proceeds as before.  Every call on a device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device (other contexts or streams) race and must be serialised by the caller;
 * calls on one stream are ordered by it.  The context must be used on the
 * device it was created on. */
int amfmm_solve_gravity_noalloc(amfmm_ctx* ctx, int64_t n, const double* x, const double* y,
                                const double* z, const double* m, double theta, double* ax,
                                double* ay, double* az, double* pot);

/* Direct summation at ntarget particles (device int64 indices; NULL = all n
 * particles in order): the exact sum that the method approximates (Sec. 3,
 * g_PP).  Coincident particles are skipped.  Outputs are device arrays of
 * ntarget doubles (pot and gabs may be NULL; gabs = G * sum_j m_j / r^2); a
 * target index outside [0, n) is read as no particle and gets NaN outputs. */
int amfmm_direct(amfmm_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                 const double* m, int64_t ntarget, const int64_t* targets, double* ax, double* ay,
                 double* az, double* pot, double* gabs);

/* Sec. 3 net balances of an acceleration field, sqrt(sum_d (sum_n m A_nd)^2 /
 * sum_d (sum_n m |A_nd|)^2) for A = g (out[0]) and A = X x g (out[1]), summed
 * on the device with compensated sums.  out: host pointer to 2 doubles;
 * synchronises the stream. */
int amfmm_balance(amfmm_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                  const double* m, const double* ax, const double* ay, const double* az,
                  double* out);

/* ---- learned pair selection (not in the paper; see amfmm_criterion) ----
 * A model is AMFMM_MLP_MODEL floats: a network 8 -> 64 -> 64 -> 1 with ReLU,
 * W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3 (the AMFMM_MLP_PARAMS
 * trainable parameters), then the feature normalisation x = fma(f, a, b),
 * a[8], b[8], and the training range of the raw features, lo[8], hi[8].
 * Inference rounds weights, inputs and hidden activations to BF16 and sums
 * in FP32 (fused multiply-adds in index order).  Its output is the predicted
 * log2 of the ratio, for the worse of the pair's two cells, of the largest
 * error |g_pair - g_direct| over the cell's particles to the multipole
 * estimate of that cell's error.  Features of a pair (A, B), d the centre
 * distance, all symmetric: (R_A+R_B)/d, |R_A-R_B|/(R_A+R_B), (k2_A+k2_B)/256,
 * |k2_A-k2_B|/128, (k3_A+k3_B)/256, |k3_A-k3_B|/128 (the traceless norm levels
 * of MULTIPOLE), |M_A-M_B|/(M_A+M_B), plog2(N_A N_B) (counts saturated at
 * 1024), where plog2(2^e (1+f)) = e + f. */
#define AMFMM_MLP_PARAMS 4801
#define AMFMM_MLP_MODEL 4833

/* Installs a model (host pointer, AMFMM_MLP_MODEL finite floats, copied) for
 * the LEARNED criterion; NULL removes it. */
int amfmm_set_model(amfmm_ctx* ctx, const float* model);
/* Features (8 floats per pair) and labels (log2 error factor, doubles) of np
 * cell pairs of the context's tree (after amfmm_compute_moments); pairs:
 * device int32, 2 per pair.  The two cells must be distinct with distinct
 * centres, as in a walk's far field; that is not checked.  A label samples up
 * to 64 particles of each cell (particle k of ns is first + k N / ns),
 * evaluates the pair alone with the variant given against direct summation
 * over the other cell, and is log2 of the larger of the two cells' ratios
 * (largest sampled error over the multipole estimate); a cell whose estimate
 * is zero (a point mass: exact) is left out, -inf when both are.  Outputs are
 * device arrays; a pair naming no cell of the tree gets NaN features or a NaN
 * label. */
int amfmm_pair_features(amfmm_ctx* ctx, int64_t np, const int32_t* pairs, float* feats);
int amfmm_pair_labels(amfmm_ctx* ctx, int32_t variant, int64_t np, const int32_t* pairs, double* labels);
/* FP32 inference exactly as the walk runs it: model (device, AMFMM_MLP_MODEL
 * floats, weights rounded on the fly), feats (device, 8 per row), y (device). */
int amfmm_mlp_predict(amfmm_ctx* ctx, int64_t n, const float* model, const float* feats, float* y);
/* Mean pinball loss at quantile tau over n rows and its gradient with respect
 * to the AMFMM_MLP_PARAMS parameters (device float array grad), computed on
 * the GPU: forward with BF16 matrix-core products and FP32 accumulation,
 * backward with FP32 matrix-core products, gradients straight through the
 * BF16 roundings, subgradient -tau at a zero residual.  loss: host double. */
int amfmm_mlp_grad(amfmm_ctx* ctx, int64_t n, const float* model, const float* feats, const float* labels,
                   double tau, float* grad, double* loss);
/* steps Adam steps (Kingma & Ba) of the pinball loss on batches of `batch`
 * rows: step s uses rows (step0 + s) * batch + r modulo n, r < batch, and
 * Adam step number step0 + s + 1 (beta1 0.9, beta2 0.999, eps 1e-8).  model,
 * adam_m, adam_v: device, updated in place (the moment arrays start at zero
 * for step0 = 0).  last_loss (host, may be NULL): loss of the last batch. */
int amfmm_mlp_train(amfmm_ctx* ctx, int64_t n, const float* feats, const float* labels, float* model,
                    float* adam_m, float* adam_v, int64_t step0, int32_t steps, int32_t batch, double lr,
                    double tau, double* last_loss);

/* Environment (read by the library, for tests and diagnosis only):
 *   AMFMM_WALK_WINDOWS=f  scales the walk's staging windows by f in [0, 1]
 *                         (small values force the spill and re-walk paths);
 *   AMFMM_DEBUG_WALK      prints per-level walk statistics to stderr (adds a
 *                         synchronisation per level). */

/* ---- introspection (host buffers owned by the caller; synchronising) ---- */
/* counts[0..11] = cells, depth, far-field pairs, near-field pairs (unordered,
 * as amfmm_get_lists returns them), leaves, particles, near-field particle
 * interactions (directed, i != j), far-field evaluations (directed cell
 * pairs), far-field kernel launches and near-field kernel launches of the
 * last evaluation, candidate pairs of the last walk (directed pairs it took a
 * decision on, self pairs included) and launches of the walk's pass kernel.
 * The near-field pair count is taken on the device from the kept lists (one
 * short kernel); it is 0 after a batched solve, which keeps no lists. */
int amfmm_get_counts(amfmm_ctx* ctx, int64_t* counts12);
/* sorted keys (n), permutation perm[s] = caller index of sorted particle s (n),
 * and per cell (in (level, first particle) order): level, begin, count,
 * parent, first child (-1 for leaves), child count.  Any pointer may be NULL. */
int amfmm_get_tree(amfmm_ctx* ctx, uint64_t* keys, int64_t* perm, int32_t* level, int64_t* begin,
                   int64_t* count, int32_t* parent, int32_t* child0, int32_t* nchild);
/* 21 doubles per cell: M, Zx, Zy, Zz, R_max, M_xx, M_xy, M_xz, M_yy, M_yz,
 * M_zz, M_xxx, M_xxy, M_xxz, M_xyy, M_xyz, M_xzz, M_yyy, M_yyz, M_yzz, M_zzz */
int amfmm_get_moments(amfmm_ctx* ctx, double* out21);
/* unordered pairs (2 int32 each), sorted: far field {a<b}, near field {a<=b};
 * far_ab holds counts[2] pairs and near_ab counts[3] of amfmm_get_counts
 * (either may be NULL).  Expands the lists on the host: meant for checks at
 * small sizes.  AMFMM_E_STATE without lists, or (writing nothing) when the
 * lists do not hold the counted pairs. */
int amfmm_get_lists(amfmm_ctx* ctx, int32_t* far_ab, int32_t* near_ab);
/* milliseconds of the phases of the last solve: [0] validate+bbox, [1] keys+sort,
 * [2] tree levels, [3] moments, [4] walk, [5] far field, [6] push-down,
 * [7] near field + evaluation at particles, [8] total, [9] the walk's pass
 * over the pairs (its staging kernel alone; part of [4]).  Returns the count
 * written (at most cap, at most 10). */
int amfmm_get_phase_times(amfmm_ctx* ctx, double* ms, int32_t cap);

const char* amfmm_status_string(int status);
const char* amfmm_last_error(amfmm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
