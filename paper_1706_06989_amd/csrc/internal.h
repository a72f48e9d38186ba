// Internal declarations of libamfmm_hip.so (host orchestration + kernels).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "amfmm.h"

namespace amfmm {

constexpr int kMaxLevel = 21;  // Morton key resolution per coordinate
constexpr int kGeo = 4;        // per cell: Zx, Zy, Zz, R_max
constexpr int kMom = 18;       // per cell: M, M_ij (6), M_ijk (10), pad
constexpr int kLoc = 24;       // per cell: C (1), C_k (3), C_kl (6), C_klm (10), g_c (3), pad
constexpr int kLocGen = 40;    // expansion order 4: 35 local coefficients, g_c (3), pad

// index of a symmetric pair / triple inside the packed arrays
//   pairs   xx xy xz yy yz zz
//   triples xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// the walk of a batch would exceed the list budget: retry with a smaller batch
struct BudgetExceeded : Error {
  BudgetExceeded() : Error(AMFMM_E_OOM, "interaction lists exceed the list budget") {}
};

#define AMFMM_HIP(call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::amfmm::Error(AMFMM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Grow-only device buffer owned by a context.
struct Arena;
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Ctx {
  amfmm_options opt;
  hipStream_t stream = nullptr;
  int device = 0;
  std::string last_error;
  size_t bytes = 0;  // device bytes currently held
  std::vector<DevBuf*> bufs;

  // particles, sorted by key
  int64_t n = 0;
  DevBuf pos4;    // double4 (x, y, z, m)
  DevBuf keys;    // uint64
  DevBuf perm;    // int32, sorted -> caller
  DevBuf keys2;   // sort ping-pong
  DevBuf perm2;
  DevBuf bbox;    // 8 doubles: lo[3], hi[3], flags
  DevBuf scratch; // scan / sort temporaries
  DevBuf scratch2;
  DevBuf hist;
  // cells in (level, begin) order
  int32_t ncells = 0, depth = 0, nleaves = 0;
  std::vector<int32_t> level_start;  // host copy, size depth+2
  DevBuf c_begin, c_count, c_parent, c_child0, c_nchild;  // int32
  DevBuf leaves;   // int32 ids of leaf cells
  DevBuf geo;      // double4 per cell
  DevBuf mom;      // kMom doubles per cell
  DevBuf msum;     // double4 per cell: sum m*X (x,y,z), unused
  DevBuf loc;      // kLoc doubles per cell
  DevBuf mono;     // expansion order 4: 35 moments per cell (sum mu x^alpha, |alpha| <= 4)
  DevBuf locg;     // expansion order 4: kLocGen doubles per cell
  // directed interaction lists grouped by target cell
  int64_t n_far = 0, n_near = 0;
  DevBuf far_start, far_count, far_src;     // int32 (start as int64)
  DevBuf near_start, near_count, near_src;
  // walk frontier
  DevBuf fx, fy, fx2, fy2, fcnt, grp, walkrec, fsave, gsave, counters, gqueue;
  DevBuf stage;  // walk: per-chunk staging windows of one level's terminal pairs
  DevBuf farrec; // far field, mixed UC/TC: 128-byte source record per cell
  // walk: terminal pairs per frontier entry of every level (far, near, split-X
  // bases; -1 = unknown) from the last walk under the rule walk_ratio_key
  std::vector<double> walk_ratio;
  double walk_ratio_key[4] = {-1.0, -1.0, -1.0, -1.0};
  int64_t grp_width = 0, frontier = 0;
  double walk_abs_tol = 0.0;
  int walk_mode = 0;              // 0 geometric, 1 error estimate, 2 learned
  DevBuf model;                   // learned criterion: network with BF16-rounded weights
  DevBuf mlp_tmp, mlp_part, mlp_grad;  // inference and training scratch
  // caller's per-particle field estimate (device): magnitudes in `field`, or
  // components in field, field_y, field_z
  const double* field = nullptr;
  const double* field_y = nullptr;
  const double* field_z = nullptr;
  DevBuf gmin;
  // unordered near-field leaf pairs of the kept lists (built on request)
  std::vector<std::pair<int32_t, int32_t>> near_pairs_host;
  bool near_pairs_valid = false;
  int grp_cur = 0;
  int64_t* pinned = nullptr;  // small pinned host buffer for read-backs
  int64_t far_evals = 0;      // directed far-field evaluations of the last solve
  int64_t far_launches = 0, near_launches = 0;  // kernel launches of the last evaluation
  int64_t pass_launches = 0;    // launches of the walk's pass kernel in the last walk
  int64_t walk_candidates = 0;  // pairs the last walk decided on (batches over budget excluded)
  bool batched = false;       // last solve ran batch by batch (lists not kept)
  size_t walk_budget = 0;     // bytes of lists + frontier a walk may take (0 = unlimited)
  // batch size that worked for the last solve of the same size and criterion
  int64_t batch_hint = 0, hint_n = 0;
  int64_t batch_fail = 0;  // smallest batch (particles) that exceeded the budget, same problem
  double hint_theta = 0.0, hint_tol = 0.0;
  int hint_mode = -1;
  double theta = 0.5;
  bool have_tree = false, have_moments = false, have_lists = false;
  // timing: events recorded at phase changes; the time between two marks
  // belongs to the phase of the first
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_phase;
  size_t ev_used = 0;
  // allocation-free solve: while arena is set, every device buffer is carved
  // from [arena, arena + arena_cap) (a static device array) instead of being
  // allocated (first fit over the free blocks, released blocks merged with
  // their neighbours), and no timing events are recorded
  char* arena = nullptr;
  size_t arena_cap = 0;
  std::map<size_t, size_t> arena_free;  // offset -> bytes of each free block
};

// device bytes a solve may still take in one buffer: the free device memory,
// or the largest free block of the arena in an allocation-free solve
size_t free_device_bytes(Ctx& c);

// allocate (grow-only) a device buffer of at least `bytes`; contents are lost on growth
void* ensure(Ctx& c, DevBuf& b, size_t bytes);
// grow keeping the first `keep` bytes
void* ensure_keep(Ctx& c, DevBuf& b, size_t bytes, size_t keep);
template <typename T>
T* as(DevBuf& b) {
  return static_cast<T*>(b.p);
}
void sync(Ctx& c);

// ---- scan.hip ----
// exclusive prefix sum of n int32 values into out[0..n], out[n] = total
void scan_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n);
// the same for int64 values
void scan_i64(Ctx& c, const int64_t* in, int64_t* out, int64_t n);

// ---- sort.hip ----
// stable LSD radix sort of (key, value) pairs by the low `bits` bits of key;
// results end in keys/vals (the alt buffers are scratch)
void radix_sort(Ctx& c, uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt,
                int64_t n, int bits);

// ---- tree.hip ----
// validate + bounding box; returns 0 or an amfmm_status (reads back flags)
int bbox_validate(Ctx& c, const double* x, const double* y, const double* z, const double* m,
                  int64_t n);
void build_keys_sort(Ctx& c, const double* x, const double* y, const double* z, const double* m,
                     int64_t n);
void build_levels(Ctx& c);

// ---- moments.hip ----
void upward_pass(Ctx& c);

// ---- walk.hip ----
void dual_walk(Ctx& c, double theta);  // whole walk, lists kept for every cell
void walk_prepare(Ctx& c, double theta);
void walk_start(Ctx& c);  // frontier = {(root, root)} at level 0
// walks levels [lev_first, lev_last] over the cells [lo[l], hi[l]) of each level,
// starting from the frontier held in c.fy / c.grp; appends lists at the bases;
// returns the size of the frontier left for level lev_last + 1
int64_t walk_levels(Ctx& c, int lev_first, int lev_last, const std::vector<int32_t>& lo,
                    const std::vector<int32_t>& hi, int64_t& far_base, int64_t& near_base);
void group_arrays(Ctx& c, int64_t** gbeg, int32_t** gcnt);  // current level's groups

// ---- eval.hip ----
// mixed precision, UC and TC: one 128-byte source record per cell for the far
// field (after the moments)
void far_prepare(Ctx& c);
void far_field(Ctx& c, int32_t c_lo, int32_t c_hi);
// expansion order 4 (order.hip): moments, far field, push-down, evaluation at the particles
void order_upward(Ctx& c);
void order_far(Ctx& c, int32_t c_lo, int32_t c_hi, double* loc);
void order_push_down(Ctx& c, int32_t c_lo, int32_t c_hi);
void order_l2p(Ctx& c, const int32_t* leaves, int32_t c_lo, int32_t count, double* ax, double* ay, double* az,
               double* pot);
void push_down(Ctx& c, int32_t c_lo, int32_t c_hi);  // cells of one level
// leaves != nullptr: the first `count` leaves of that list; else the leaves
// among cells [c_lo, c_lo + count)
void near_field(Ctx& c, const int32_t* leaves, int32_t c_lo, int32_t count, double* ax, double* ay, double* az,
                double* pot);
// fills n (<= 64) device words with zero (a kernel, so it can sit in a graph)
void zero_u64(Ctx& c, unsigned long long* p, int n);

// ---- mlp.hip ----
// features (8 floats) and labels (log2 error factor) of cell pairs (device)
void compute_pair_features(Ctx& c, int64_t np, const int32_t* pairs, float* feats);
void compute_pair_labels(Ctx& c, int variant, int64_t np, const int32_t* pairs, double* labels);
// model with its weights rounded to BF16 (device to device)
void round_model(Ctx& c, const float* in, float* out);
void mlp_predict(Ctx& c, int64_t n, const float* model, const float* feats, float* y);
// gradient into grad (device); returns the loss (synchronises)
double mlp_grad(Ctx& c, int64_t n, const float* model, const float* feats, const float* labels, double tau,
                float* grad);
// Adam steps; returns the loss of the last batch (synchronises)
double mlp_train(Ctx& c, int64_t n, const float* feats, const float* labels, float* model, float* am, float* av,
                 int64_t step0, int32_t steps, int32_t batch, double lr, double tau);

// ---- integrate.hip ----
// v += h a and x += dt v over n particles (device SoA arrays)
void kick(Ctx& c, int64_t n, double h, const double* ax, const double* ay, const double* az, double* vx, double* vy,
          double* vz);
void drift(Ctx& c, int64_t n, double dt, const double* vx, const double* vy, const double* vz, double* x, double* y,
           double* z);

// ---- direct.hip ----
void direct_sum(Ctx& c, int64_t n, const double* x, const double* y, const double* z,
                const double* m, int64_t ntarget, const int64_t* targets, double* ax, double* ay,
                double* az, double* pot, double* gabs);
void balance(Ctx& c, int64_t n, const double* x, const double* y, const double* z,
             const double* m, const double* ax, const double* ay, const double* az, double* out);

// phases of a solve (amfmm_get_phase_times order)
// kPhWalkPass: the walk's one pass over the pairs (its staging kernel), a part
// of the walk that is also reported on its own
enum Phase { kPhValidate = 0, kPhSort, kPhTree, kPhMoments, kPhWalk, kPhFar, kPhPush, kPhNear, kPhWalkPass, kPhEnd };
void mark(Ctx& c, int phase);  // records an event; phase kPhEnd closes the timeline

inline unsigned blocks_for(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}

}  // namespace amfmm
