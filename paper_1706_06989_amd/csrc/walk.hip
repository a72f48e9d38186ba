// Interaction selection (Sec. 2): symmetric dual walk under the opening
// criterion |Z_A - Z_B| >= (R_A + R_B)/theta, or an error-estimate criterion
// (the error-based selection Sec. 2 cites), organised by target cell.
//
// The walk of cell pairs is reproduced pair for pair, but every visited pair
// is held twice, once by each of its cells (directed entries (X, Y)), and the
// frontier is processed one tree level of X at a time, grouped by X.  A wave
// takes a chunk of X's entries and expands them breadth first (a work queue
// in LDS or global memory; a lane descends a subtree alone when the queue is
// full) while the symmetric split rule opens Y; each terminal pair ends as
//   * a far-field entry X <- Y when accepted,
//   * a near-field entry X <- Y when both are leaves (or no cell below Y can
//     be accepted with the leaf X: Y's whole subtree),
//   * a "split X" base that hands (X_c, Y) to every child X_c of X.
// A self entry (X, X) of a split cell hands (X_c, X_c') to every child for all
// children X_c' (self included); of a leaf it becomes the near-field entry X<-X.
// The decision on a pair depends only on the unordered pair (the criterion is
// symmetric and the split rule picks the larger R_max, ties to the lower
// index, and the non-leaf when one is a leaf), so both cells of a pair make
// the same decision.  One pass per level writes every chunk's terminal pairs
// to staging room, scans of the per-chunk counts place them, and a copy
// gives lists grouped by target with no sort (chunks that outgrew their room
// are walked a second time straight into place); the result is
// deterministic.
//
// Compiled with -ffp-contract=off: the criterion must round exactly as the
// plain definition does.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "device_math.h"
#include "internal.h"
#include "learned.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;

enum : int { kAccept = 0, kNear = 1, kSplitX = 2, kSplitY = 3, kAsk = 4 };

// per cell, everything a walk step reads, in one 64-byte record
struct alignas(16) WalkRec {
  double gx, gy, gz, gw;  // centre of mass, R_max
  double m, gmin;         // mass, field scale of the cell (see k_gscale)
  // first child, parent, particles, meta: nch (bits 0-3) | has_next (4) |
  // traceless quadrupole level (12-19) | traceless octupole level (20-27)
  int32_t ch0, par, count, meta;
};

struct WalkCell {
  double gx, gy, gz, gw, m, gmin;
  int32_t ch0, nch, par, next, count, k2, k3;
};

struct TreeView {
  const WalkRec* rec;
  double theta;
  double abs_tol;    // bound on the rounding of any centre of mass (absolute)
  int mode;          // 0: opening angle theta; 1: error estimate; 2: learned; 3: multipole estimate
  double eps;        // modes 1-3: accepted error per pair, relative to each cell's field
  double theta_max;  // modes 1-3: (R_A + R_B)/d above this never accepted
  double theta_max2; // theta_max^2
  const float* model;  // mode 2: network (BF16-rounded weights)
  int64_t min_work;    // mode 2: least N_A N_B for which the network is asked
  const double* mmin;  // modes 1-3: smallest leaf mass below each cell
  const float* lmodel; // mode 2, in the kernels: the network's LDS copy (lds_model_index layout)
};

__device__ inline WalkCell load_cell(const WalkRec* __restrict__ r, int32_t c) {
  const double2* p = reinterpret_cast<const double2*>(r + c);
  const int4* q = reinterpret_cast<const int4*>(reinterpret_cast<const char*>(r + c) + 48);
  WalkCell w;
  const double2 p0 = p[0], p1 = p[1], p2 = p[2];
  w.gx = p0.x;
  w.gy = p0.y;
  w.gz = p1.x;
  w.gw = p1.y;
  w.m = p2.x;
  w.gmin = p2.y;
  const int4 v = q[0];
  w.ch0 = v.x;
  w.par = v.y;
  w.count = v.z;
  w.nch = v.w & 0xf;
  w.next = ((v.w >> 4) & 1) ? c + 1 : -1;
  w.k2 = (v.w >> 12) & 0xff;
  w.k3 = (v.w >> 20) & 0xff;
  return w;
}

// Which decisions a kernel carries besides modes 0 and 1: the network's
// (mode 2) or the multipole estimate's (mode 3); kernels of the other modes
// stay free of their code and registers.
enum : int { kExtBase = 0, kExtLearned = 2, kExtMultipole = 3 };

// The rules for a pair that is not accepted: near field, or which cell opens.
template <int EXT>
__device__ inline int open_rule(const TreeView& t, int32_t X, const WalkCell& a, int32_t Y, const WalkCell& b,
                                double d) {
  const int mode = EXT == kExtBase ? t.mode : EXT;
  const bool lx = a.nch == 0, ly = b.nch == 0;
  if (lx && ly) return kNear;
  if (lx) {
    // Every centre of mass inside Y lies within R_Y of Z_Y, so when even
    // d + R_Y falls short of R_X/theta no cell below Y can be accepted with the
    // leaf X and the walk would pair X with every leaf under Y: record Y once
    // as a near-field source (its whole particle range).  The margin makes the
    // test safe against rounding of d and of the centres.
    const double cut = mode == 0 ? t.theta : t.theta_max;
    if ((d + b.gw) * (1.0 + 1e-12) + t.abs_tol < a.gw / cut) return kNear;
    if (mode != 0) {
      // Error-estimate modes: a cell Y' below Y has d' <= d + R_Y, mass at
      // least the smallest leaf mass m below Y, and R_X + R_Y' >= R_X, so its
      // estimate e' M_Y' = (R_X + R_Y')^3 M_Y' / d'^5 is at least
      // R_X^3 m / (d + R_Y)^5, and in modes 2 and 3 the multipole estimate's
      // w1 R_X^3 M_Y' / d'^5 term alone is at least as large (w1 >= 1).  When
      // that exceeds what any rule accepts (eps s_X, times the network's upper
      // gate in mode 2) no pair below Y is accepted with X either: Y is a
      // near-field source as a whole.
      const double D = (d + b.gw + t.abs_tol) * (1.0 + 1e-9);
      const double D2 = D * D;
      const double lim = (mode == 2 ? kGateHi : 1.0) * t.eps * a.gmin;
      if ((a.gw * a.gw * a.gw) * t.mmin[Y] > lim * (D2 * D2 * D)) return kNear;
    }
    return kSplitY;
  }
  if (ly) return kSplitX;
  if (a.gw > b.gw) return kSplitX;
  if (a.gw < b.gw) return kSplitY;
  return X < Y ? kSplitX : kSplitY;
}

// The walk's decision on pair (X, Y).  Mode 2 with f given: a pair the
// network has to decide returns kAsk with its features in f and the
// threshold in *thr (the caller runs the network for the wave and finishes
// with open_rule); without f the lane runs the network itself.  *dist: the
// centre distance, for open_rule.
template <int EXT>
__device__ inline int decide(const TreeView& t, int32_t X, const WalkCell& a, int32_t Y, const WalkCell& b,
                             float* f = nullptr, float* thr = nullptr, double* dist = nullptr) {
  // the learned and multipole kernels serve only their own mode: a constant
  const int mode = EXT == kExtBase ? t.mode : EXT;
  const double dx = a.gx - b.gx, dy = a.gy - b.gy, dz = a.gz - b.gz;
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double r = a.gw + b.gw;
  // one root per pair, shared by the acceptance tests and the leaf rule below
  // (lanes of a wave take both paths)
  const double d = sqrt(d2);
  if (dist) *dist = d;
  if (mode == 0) {
    const double rhs = r / t.theta;
    if (d > 0.0 && d >= rhs) return kAccept;
  } else if (EXT == kExtBase || mode == 1) {
    // The force error of a quadrupole-order pair scales as M_other r^3 / d^5
    // with r = R_A + R_B; accept when that estimate stays below eps times the
    // field scale of each cell (both cells: a symmetric decision) and r <=
    // theta_max d.  Product form, squared: no division or root.
    if (d2 > 0.0 && r * r <= t.theta_max2 * d2) {
      const double r2 = r * r;
      const double r6 = (r2 * r2) * r2;
      const double d10 = ((d2 * d2) * (d2 * d2)) * d2;
      const double wa = t.eps * a.gmin, wb = t.eps * b.gmin;
      if (r6 * (b.m * b.m) <= (wa * wa) * d10 && r6 * (a.m * a.m) <= (wb * wb) * d10) return kAccept;
    }
  } else if (EXT == kExtMultipole) {
    // mode 3: (P_A d + Q_A) M_B <= eps s_A d^6 and the same for B, in product
    // form (one root, no division)
    if (d2 > 0.0 && r * r <= t.theta_max2 * d2) {
      const double d6 = (d2 * d2) * d2;
      const double ea = multipole_bracket(a.gw, b.gw, b.k2, b.k3, d) * b.m;
      const double eb = multipole_bracket(b.gw, a.gw, a.k2, a.k3, d) * a.m;
      if (ea <= (t.eps * a.gmin) * d6 && eb <= (t.eps * b.gmin) * d6) return kAccept;
    }
  } else {
    // mode 2: the multipole estimate, the network deciding where it is close
    // to the bound (same theta_max guard as mode 3)
    if (d2 > 0.0 && r * r <= t.theta_max2 * d2) {
      const PairSide A{a.gw, a.m, a.k2, a.k3, a.count, a.gmin}, B{b.gw, b.m, b.k2, b.k3, b.count, b.gmin};
      float g[kFeat], th = 0.0f;
      float* fo = f ? f : g;
      const int v = learned_gate(t.lmodel, t.eps, t.min_work, d, d2, A, B, fo, &th);
      if (v == kLrnAccept) return kAccept;
      if (v == kLrnAsk) {
        if (f) {
          *thr = th;
          return kAsk;
        }
        if (mlp_infer(t.model, g) <= th) return kAccept;
      }
    }
  }
  return open_rule<EXT>(t, X, a, Y, b, d);
}

// Visits the pairs of entry (X, Y) in depth-first order (children of Y in
// octant order) and calls f(kind, Y') for each decision: the terminal ones
// and the opened ones (kSplitY, Y itself first).
template <int EXT, typename F>
__device__ inline void traverse(const TreeView& t, int32_t X, int32_t Y, F&& f) {
  const WalkCell a = load_cell(t.rec, X);
  if (X == Y) {
    if (a.nch == 0) {
      f(kNear, X);
    } else {
      for (int32_t j = 0; j < a.nch; ++j) f(kSplitX, a.ch0 + j);
    }
    return;
  }
  int32_t cur = Y;
  WalkCell b = load_cell(t.rec, cur);
  for (;;) {
    int d = decide<EXT>(t, X, a, cur, b);
    if (d == kSplitY) {
      f(kSplitY, cur);
      cur = b.ch0;
      b = load_cell(t.rec, cur);
      continue;
    }
    f(d, cur);
    for (;;) {
      if (cur == Y) return;
      if (b.next >= 0) {
        cur = b.next;
        b = load_cell(t.rec, cur);
        break;
      }
      cur = b.par;
      b = load_cell(t.rec, cur);
    }
  }
}

__global__ void __launch_bounds__(kBS) k_pack_cells(int32_t nc, const double4* __restrict__ geo,
                                                    const double* __restrict__ mom, const int32_t* __restrict__ ch0,
                                                    const int32_t* __restrict__ nch, const int32_t* __restrict__ par,
                                                    const int32_t* __restrict__ cnt, const double* __restrict__ gmin,
                                                    WalkRec* __restrict__ rec) {
  int32_t c = blockIdx.x * kBS + threadIdx.x;
  if (c >= nc) return;
  WalkRec w;
  const double4 g = geo[c];
  w.gx = g.x;
  w.gy = g.y;
  w.gz = g.z;
  w.gw = g.w;
  const double* mo = mom + (int64_t)c * kMom;
  w.m = mo[0];
  w.gmin = gmin ? gmin[c] : 0.0;
  w.ch0 = nch[c] ? ch0[c] : -1;
  const int32_t p = par[c];
  w.par = p;
  w.count = cnt[c];
  const int has_next = (p >= 0 && c + 1 < ch0[p] + nch[p]) ? 1 : 0;
  const int k2 = norm_level(traceless_norm2(mo + 1), mo[0], g.w, 2);
  const int k3 = norm_level(traceless_norm3(mo + 7), mo[0], g.w, 3);
  w.meta = nch[c] | (has_next << 4) | (k2 << 12) | (k3 << 20);
  rec[c] = w;
}

// Field scale of every cell: the smallest field estimate over its particles,
// but at least kFieldFloor times their mean (a cell holding a point where the
// field vanishes would otherwise never be accepted).  Sums run leaf-sequentially
// in key order and for parents over their children in octant order (a fixed
// order, so the value is reproducible bit for bit); min is order-free.
constexpr double kFieldFloor = 0.1;

// gy == nullptr: gx holds field magnitudes; else (gx, gy, gz) are components
__global__ void __launch_bounds__(kBS) k_gsum_leaves(const int32_t* __restrict__ leaves, int32_t nleaves,
                                                     const int32_t* __restrict__ beg, const int32_t* __restrict__ cnt,
                                                     const int32_t* __restrict__ perm, const double* __restrict__ gx,
                                                     const double* __restrict__ gy, const double* __restrict__ gz,
                                                     double* __restrict__ gsum, double* __restrict__ gmn) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nleaves) return;
  const int32_t c = leaves[i];
  double v = 0.0, w = INFINITY;
  for (int32_t p = beg[c]; p < beg[c] + cnt[c]; ++p) {
    const int32_t o = perm[p];
    const double g = gy ? sqrt((gx[o] * gx[o] + gy[o] * gy[o]) + gz[o] * gz[o]) : fabs(gx[o]);
    v += g;
    w = fmin(w, g);
  }
  gsum[c] = v;
  gmn[c] = w;
}

__global__ void __launch_bounds__(kBS) k_gsum_up(int32_t c0, int32_t nl, const int32_t* __restrict__ ch0,
                                                 const int32_t* __restrict__ nch, double* __restrict__ gsum,
                                                 double* __restrict__ gmn) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  const int32_t c = c0 + i;
  if (nch[c] == 0) return;
  double v = 0.0, w = INFINITY;
  for (int32_t q = ch0[c]; q < ch0[c] + nch[c]; ++q) {
    v += gsum[q];
    w = fmin(w, gmn[q]);
  }
  gsum[c] = v;
  gmn[c] = w;
}

__global__ void __launch_bounds__(kBS) k_gscale(int32_t nc, const int32_t* __restrict__ cnt,
                                                const double* __restrict__ gsum, const double* __restrict__ gmn,
                                                double* __restrict__ gscale) {
  int32_t c = blockIdx.x * kBS + threadIdx.x;
  if (c < nc) gscale[c] = fmax(gmn[c], kFieldFloor * (gsum[c] / (double)cnt[c]));
}

// smallest leaf mass below every cell (leaves: their mass; parents: the
// smallest over their children), for the subtree near-field test
__global__ void __launch_bounds__(kBS) k_mmin_leaves(const int32_t* __restrict__ leaves, int32_t nleaves,
                                                     const double* __restrict__ mom, double* __restrict__ mmin) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nleaves) return;
  const int32_t c = leaves[i];
  mmin[c] = mom[(int64_t)c * kMom];
}

__global__ void __launch_bounds__(kBS) k_mmin_up(int32_t c0, int32_t nl, const int32_t* __restrict__ ch0,
                                                 const int32_t* __restrict__ nch, double* __restrict__ mmin) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  const int32_t c = c0 + i;
  if (nch[c] == 0) return;
  double w = INFINITY;
  for (int32_t q = ch0[c]; q < ch0[c] + nch[c]; ++q) w = fmin(w, mmin[q]);
  mmin[c] = w;
}

__device__ inline int32_t wave_excl_scan(int32_t v, int32_t* total) {
  const int32_t inc = wave_incl_scan(v);
  *total = __builtin_amdgcn_readlane(inc, 63);
  return inc - v;
}

// set bits of a wave mask in the lanes below this one
__device__ inline int32_t lanes_below(uint64_t mask) {
  return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

constexpr int kQ = 1024;  // per-wave LDS work queue (power of two)

// orders this wave's queue writes (LDS or global) before its lanes read them
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Staging of a level's terminal pairs.  Every chunk owns a window of each
// staging array (far, near, split-X bases) sized by the pairs its entries are
// expected to produce; a chunk that outgrows a window continues in spill
// regions taken from that list's shared pool (one atomic each), of doubling
// sizes: region j holds u 2^j entries, u the power of two at least twice the
// window and at least kSpillMin, so kRegions regions hold 255 u.  A chunk that
// outgrows them, or finds the pool exhausted, stops writing (its counts still
// run on) and is walked again by the emitting kernel.
constexpr int64_t kSpillMin = 1024;
constexpr int kRegions = 8;

// log2 of the first spill region's size for a window of `cap` entries
__host__ __device__ inline int spill_shift(int64_t cap) {
  int sh = 10;  // kSpillMin
  while ((int64_t(1) << sh) < 2 * cap) ++sh;
  return sh;
}

// spill region of position g past the window, and the offset inside it
__device__ inline int spill_region(int64_t g, int sh, int64_t* off) {
  const uint64_t q = (uint64_t)(g >> sh) + 1;
  const int j = 63 - __builtin_clzll(q);
  *off = g - (((int64_t(1) << j) - 1) << sh);
  return j;
}

struct StageLayout {
  int32_t* win[3];             // window arrays
  int32_t* spill[3];           // spill pools
  int64_t* ksec;               // per chunk and list: kRegions spill region offsets
  unsigned long long* used;    // spill entries handed out, per list
  int64_t spill_cap[3];        // entries in each spill pool
  int64_t cap16[3];            // window capacity per entry, in 1/16
  int64_t slack[3];            // window slack per chunk
};

// window of list w of the chunk whose entries start at frontier position e
// (chunk index k): [lo(e, k), lo(e + n, k + 1)); the windows tile the array
__device__ inline int64_t stage_lo(const StageLayout& s, int w, int64_t e, int64_t k) {
  return ((s.cap16[w] * e) >> 4) + k * s.slack[w];
}

// Where a wave's terminal pairs go.  EMIT: straight to their final places
// (far/near lists at fo/no, split-X bases replicated for every child of X in
// fy_n).  STAGE: to its windows and spill regions (positions fo, no, B count
// from 0, split-X bases once each).
struct EmitDst {
  int64_t fo, no, nb, S;
  int32_t* far_src;
  int32_t* near_src;
  int32_t* fy_n;
  int64_t B0;  // rank of this chunk's first split-X base inside the cell
  // STAGE
  const StageLayout* sl;
  int32_t* win[3];
  int64_t wcap[3];
  int64_t chunk;
  int64_t* lreg;  // this wave's spill region offsets in LDS (3 x kRegions)
  int wsh;        // spill_shift of window w in bits 8w..8w+7
};

enum : int { kStage = 0, kEmit = 1 };

// All pairs held by target cell X at this level, processed by one wave
// breadth-first: each step gives every lane one pair (taken first from the
// wave's queue, else from X's frontier entries); a pair whose rule opens Y
// pushes Y's children to the queue; when the queue is full the lane descends
// Y's subtree itself.  The order is a fixed function of the inputs, so the
// staging run and an emitting run visit the same pairs in the same order.
// Returns the chunk's totals in tm, tp, tq, the pairs it decided on (its
// candidate pairs, taken from the frontier or the queue, self pairs included)
// in td, and (STAGE) whether it ran out of room.
template <int PASS, int EXT, typename Q>
__device__ inline bool wave_walk(const TreeView& t, int32_t X, const WalkCell& cx, const int32_t* __restrict__ fy,
                                 int64_t b, int32_t n, Q qbuf, int32_t qcap, int64_t& tm, int64_t& tp, int64_t& tq,
                                 int64_t& td, EmitDst dst, unsigned long long* dbg) {
  const int32_t qmask = qcap - 1;
  const int lane = threadIdx.x & 63;
  // mode 2: this lane's part of the network, for the wave's cooperative
  // inference
  MlpLane ml{};
  if (EXT == kExtLearned) ml = mlp_lane(t.lmodel);
  int32_t head = 0, tail = 0, fpos = 0;
  int64_t fo = dst.fo, no = dst.no, B = dst.B0;
  unsigned long long dsteps = 0, ddeep = 0, dpairs = 0, dask = 0, daskw = 0;
  int32_t nreg[3] = {0, 0, 0};  // STAGE: spill regions held (wave-uniform)
  bool ovf = false;              // STAGE: out of room; writes stop
  auto stage_put = [&](int w, int64_t f, int32_t v) {
    if (!ovf) {
      if (f < dst.wcap[w]) {
        dst.win[w][f] = v;
      } else {
        int64_t off;
        const int j = spill_region(f - dst.wcap[w], (dst.wsh >> (8 * w)) & 0xff, &off);
        dst.sl->spill[w][dst.lreg[w * kRegions + j] + off] = v;
      }
    }
  };
  auto put_far = [&](int64_t f, int32_t v) {
    if (PASS == kEmit) dst.far_src[f] = v;
    else stage_put(0, f, v);
  };
  auto put_near = [&](int64_t g, int32_t v) {
    if (PASS == kEmit) dst.near_src[g] = v;
    else stage_put(1, g, v);
  };
  auto put_split = [&](int64_t r, int32_t v) {
    if (PASS == kEmit) {
      for (int32_t c = 0; c < cx.nch; ++c) dst.fy_n[dst.nb + c * dst.S + r] = v;
    } else {
      stage_put(2, r, v);
    }
  };
  // STAGE: room for positions below `end` of list w
  auto reserve = [&](int w, int64_t end) {
    const int64_t cap = dst.wcap[w];
    const int sh = (dst.wsh >> (8 * w)) & 0xff;
    while (!ovf && end > cap + ((((int64_t)1 << nreg[w]) - 1) << sh)) {
      if (nreg[w] == kRegions) {
        ovf = true;
        break;
      }
      const int64_t size = int64_t(1) << (sh + nreg[w]);
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(&dst.sl->used[w], (unsigned long long)size);
      base = __shfl(base, 0, 64);
      if (base + (unsigned long long)size > (unsigned long long)dst.sl->spill_cap[w]) {
        ovf = true;
        break;
      }
      if (lane == 0) {
        dst.lreg[w * kRegions + nreg[w]] = (int64_t)base;
        dst.sl->ksec[(3 * dst.chunk + w) * kRegions + nreg[w]] = (int64_t)base;
      }
      ++nreg[w];
    }
  };
  while (head < tail || fpos < n) {
    int32_t Y = -1;
    if (head < tail) {
      const int k = min(64, tail - head);
      if (lane < k) Y = qbuf[(head + lane) & qmask];
      head += k;
    } else {
      const int k = min(64, n - fpos);
      if (lane < k) Y = fy[b + fpos + lane];
      fpos += k;
    }
    wave_sync();  // queue slots just read may be reused by this step's pushes
    td += __popcll(__ballot(Y >= 0));
    int32_t m = 0, p = 0, q = 0, push = 0, ych0 = 0;
    const bool self = Y >= 0 && Y == X;
    WalkCell cy{};
    int d = -1;
    float f[kFeat], thr = 0.0f;
    double dist = 0.0;
    if (Y >= 0 && !self) {
      cy = load_cell(t.rec, Y);
      d = EXT == kExtLearned ? decide<EXT>(t, X, cx, Y, cy, f, &thr, &dist) : decide<EXT>(t, X, cx, Y, cy);
    }
    if (EXT == kExtLearned) {
      // Pairs for the network are decided by the whole wave (every lane
      // active again here), one after the other, each lane holding a hidden
      // unit.
      const bool ask = d == kAsk;
      float mine = 0.0f;
      const uint64_t asked = __ballot(ask);
      if (dbg) {
        dask += __popcll(asked);
        daskw += asked != 0;
      }
      for (uint64_t am = asked; am; am &= am - 1) {
        const int L = __ffsll((unsigned long long)am) - 1;
        float g[kFeat];
#pragma unroll
        for (int i = 0; i < kFeat; ++i) g[i] = lane_value(f[i], L);
        const float y = mlp_infer_wave(t.lmodel, ml, g);
        if (lane == L) mine = y;
      }
      if (ask) d = mine <= thr ? kAccept : open_rule<EXT>(t, X, cx, Y, cy, dist);
    }
    if (self) {
      if (cx.nch == 0) p = 1;
      else q = cx.nch;
    } else if (Y >= 0) {
      m = d == kAccept;
      p = d == kNear;
      q = d == kSplitX;
      if (d == kSplitY) {
        push = cy.nch;
        ych0 = cy.ch0;
      }
    }
    int32_t ptot;
    const int32_t poff = wave_excl_scan(push, &ptot);
    const int32_t freeq = qcap - (tail - head);
    const bool fits = poff + push <= freeq;
    const uint64_t over = __ballot(push > 0 && !fits);
    const int32_t pushed = over ? __shfl(poff, __ffsll((unsigned long long)over) - 1, 64) : ptot;
    if (push > 0 && fits)
      for (int32_t j = 0; j < push; ++j) qbuf[(tail + poff + j) & qmask] = ych0 + j;
    tail += pushed;
    wave_sync();
    const bool deep = push > 0 && !fits;  // queue full: descend in this lane
    if (dbg) {
      const uint64_t dm = __ballot(deep), ym = __ballot(Y >= 0);
      dsteps += 1;
      ddeep += __popcll(dm);
      dpairs += __popcll(ym);
    }
    int32_t nd = 0;  // decisions inside a descent
    if (deep)
      traverse<EXT>(t, X, Y, [&](int d, int32_t) {
        m += d == kAccept;
        p += d == kNear;
        q += d == kSplitX;
        ++nd;
      });
    if (__ballot(deep)) {
      // candidate pairs decided inside descents (the entry's own, decided
      // again first, is counted already)
      int32_t ndt;
      (void)wave_excl_scan(deep ? nd - 1 : 0, &ndt);
      td += ndt;
    }
    int32_t Tm, Tp, Tq, om, op, oq;
    if (__ballot(deep || self) == 0) {
      // no descent and no self pair: every lane holds at most one terminal
      // pair, so the offsets are counts of lanes below
      const uint64_t bm = __ballot(m != 0), bp = __ballot(p != 0), bq = __ballot(q != 0);
      om = lanes_below(bm);
      op = lanes_below(bp);
      oq = lanes_below(bq);
      Tm = __popcll(bm);
      Tp = __popcll(bp);
      Tq = __popcll(bq);
    } else {
      om = wave_excl_scan(m, &Tm);
      op = wave_excl_scan(p, &Tp);
      oq = wave_excl_scan(q, &Tq);
    }
    if (PASS == kStage) {
      reserve(0, fo + Tm);
      reserve(1, no + Tp);
      reserve(2, B + Tq);
      wave_sync();  // new region offsets in LDS before they are read
    }
    if (deep) {
      int64_t f = fo + om, g = no + op, bb = B + oq;
      traverse<EXT>(t, X, Y, [&](int d, int32_t Z) {
        if (d == kAccept) put_far(f++, Z);
        else if (d == kNear) put_near(g++, Z);
        else if (d == kSplitX) put_split(bb++, Z);
      });
    } else if (self) {
      if (p) put_near(no + op, X);
      for (int32_t j = 0; j < q; ++j) put_split(B + oq + j, cx.ch0 + j);
    } else if (m) {
      put_far(fo + om, Y);
    } else if (p) {
      put_near(no + op, Y);
    } else if (q) {
      put_split(B + oq, Y);
    }
    fo += Tm;
    no += Tp;
    B += Tq;
  }
  tm = fo - dst.fo;
  tp = no - dst.no;
  tq = B - dst.B0;

  if (dbg && (threadIdx.x & 63) == 0) {
    atomicAdd(&dbg[0], dsteps);
    atomicAdd(&dbg[1], ddeep);
    atomicAdd(&dbg[2], dpairs);
    atomicAdd(&dbg[3], dask);
    atomicAdd(&dbg[4], daskw);
  }
  return ovf;
}
constexpr int kChunkMax = 4096;               // frontier entries per wave: at most this many,
constexpr int64_t kWavesPerLevel = 1 << 17;   // aiming at about this many waves per level
constexpr int64_t kGlobalQueueBytes = int64_t(1) << 31;  // global work queues of a level: at most this many bytes,
constexpr int32_t kGlobalQueueMax = 1 << 18;  // at most this many entries per wave, used when at least 4 kQ

// chunk -> cell map of the level: kcell[k] = i for cbase[i] <= k < cbase[i+1]
__global__ void __launch_bounds__(kBS) k_chunk_map(int32_t nl, const int64_t* __restrict__ cbase,
                                                   int32_t* __restrict__ kcell) {
  const int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  for (int64_t k = cbase[i]; k < cbase[i + 1]; ++k) kcell[k] = i;
}

__global__ void __launch_bounds__(kBS) k_chunk_counts(int32_t nl, const int32_t* __restrict__ gcnt, int32_t chunk,
                                                      int64_t* __restrict__ nck) {
  const int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i < nl) nck[i] = (gcnt[i] + chunk - 1) / chunk;
}

// The learned kernels' copy of the network in LDS (W2 transposed, see
// lds_model_index), loaded by the whole workgroup before any wave leaves.
__device__ inline const float* stage_model(const float* __restrict__ g, float* lds) {
  for (int i = threadIdx.x; i < AMFMM_MLP_MODEL; i += kBS) lds[lds_model_index(i)] = g[i];
  __syncthreads();
  return lds;
}

// One wave per chunk of a cell's frontier entries: walk it once, writing its
// terminal pairs to its staging room, and record its counts (and whether it
// ran out of room).
template <int EXT>
__global__ void __launch_bounds__(kBS) k_walk_stage(TreeView t, int32_t c0, int64_t kn, int32_t chunk,
                                                    const int32_t* __restrict__ kcell, const int64_t* __restrict__ cbase,
                                                    const int64_t* __restrict__ gbeg, const int32_t* __restrict__ gcnt,
                                                    const int32_t* __restrict__ fy, const StageLayout* __restrict__ sl,
                                                    int64_t* __restrict__ km, int64_t* __restrict__ kp,
                                                    int64_t* __restrict__ kq, int32_t* __restrict__ kov,
                                                    int64_t* __restrict__ kd, unsigned long long* __restrict__ nov,
                                                    int32_t* __restrict__ gq, int32_t qcap, unsigned long long* dbg) {
  __shared__ int32_t queue[kBS / 64][kQ];
  __shared__ int64_t regions[kBS / 64][3 * kRegions];
  __shared__ float model[EXT == kExtLearned ? AMFMM_MLP_MODEL : 1];
  if (EXT == kExtLearned) t.lmodel = stage_model(t.model, model);
  const int lane = threadIdx.x & 63;
  // wave-uniform (readfirstlane): the cell's record and bookkeeping are
  // loaded once per wave into scalar registers
  const int64_t k = uniform((int32_t)(xcd_block(blockIdx.x, gridDim.x) * (kBS / 64) + (threadIdx.x >> 6)));
  if (k >= kn) return;
  const int32_t i = kcell[k];
  const int32_t X = c0 + i;
  const WalkCell cx = load_cell(t.rec, X);
  const int64_t e0 = (k - cbase[i]) * chunk;
  const int32_t n = (int32_t)min<int64_t>(chunk, gcnt[i] - e0);
  const int64_t e = gbeg[i] + e0;
  EmitDst dst{0, 0, 0, 0, nullptr, nullptr, nullptr, 0, sl, {}, {}, k, regions[threadIdx.x >> 6]};
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const int64_t lo = stage_lo(*sl, w, e, k);
    dst.win[w] = sl->win[w] + lo;
    dst.wcap[w] = stage_lo(*sl, w, e + n, k + 1) - lo;
    dst.wsh |= spill_shift(dst.wcap[w]) << (8 * w);
  }
  int64_t tm = 0, tp = 0, tq = 0, td = 0;
  bool over;
  if (gq)
    over = wave_walk<kStage, EXT>(t, X, cx, fy, e, n, gq + k * qcap, qcap, tm, tp, tq, td, dst, dbg);
  else
    over = wave_walk<kStage, EXT>(t, X, cx, fy, e, n, queue[threadIdx.x >> 6], kQ, tm, tp, tq, td, dst, dbg);
  if (lane == 0) {
    kd[k] = td;
    km[k] = tm;
    kp[k] = tp;
    kq[k] = tq;
    kov[k] = over ? 1 : 0;
    if (over) atomicAdd(nov, 1ull);
  }
}

// per cell: list extents, the size of its children's entries, and their groups
__global__ void __launch_bounds__(kBS) k_walk_cells(TreeView t, int32_t c0, int32_t nl, int32_t c0n,
                                                    const int64_t* __restrict__ cbase, const int64_t* __restrict__ mex,
                                                    const int64_t* __restrict__ pex, const int64_t* __restrict__ qex,
                                                    int64_t far_base, int64_t near_base, int64_t* __restrict__ far_start,
                                                    int32_t* __restrict__ far_count, int64_t* __restrict__ near_start,
                                                    int32_t* __restrict__ near_count, int64_t* __restrict__ ns) {
  const int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  const int32_t X = c0 + i;
  const int64_t k0 = cbase[i], k1 = cbase[i + 1];
  far_start[X] = far_base + mex[k0];
  far_count[X] = (int32_t)(mex[k1] - mex[k0]);
  near_start[X] = near_base + pex[k0];
  near_count[X] = (int32_t)(pex[k1] - pex[k0]);
  ns[i] = (int64_t)load_cell(t.rec, X).nch * (qex[k1] - qex[k0]);
}

__global__ void __launch_bounds__(kBS) k_walk_groups(TreeView t, int32_t c0, int32_t nl, int32_t c0n,
                                                     const int64_t* __restrict__ cbase, const int64_t* __restrict__ qex,
                                                     const int64_t* __restrict__ nbase, int64_t* __restrict__ gbeg_n,
                                                     int32_t* __restrict__ gcnt_n) {
  const int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  const WalkCell cx = load_cell(t.rec, c0 + i);
  const int64_t S = qex[cbase[i + 1]] - qex[cbase[i]], nb = nbase[i];
  for (int32_t r = 0; r < cx.nch; ++r) {
    gbeg_n[cx.ch0 + r - c0n] = nb + r * S;
    gcnt_n[cx.ch0 + r - c0n] = (int32_t)S;
  }
}

// One wave per staged chunk that did not run out of room: copy its windows
// (and spill regions) to the final lists (split-X bases once for every child
// of the cell).
__global__ void __launch_bounds__(kBS) k_walk_compact(TreeView t, int32_t c0, int64_t kn, int32_t chunk,
                                                      const int32_t* __restrict__ kcell,
                                                      const int64_t* __restrict__ cbase,
                                                      const int64_t* __restrict__ gbeg,
                                                      const int32_t* __restrict__ gcnt,
                                                      const StageLayout* __restrict__ slp,
                                                      const int64_t* __restrict__ mex, const int64_t* __restrict__ pex,
                                                      const int64_t* __restrict__ qex, const int64_t* __restrict__ nbase,
                                                      const int32_t* __restrict__ kov, int64_t far_base,
                                                      int64_t near_base, int32_t* __restrict__ far_src,
                                                      int32_t* __restrict__ near_src, int32_t* __restrict__ fy_n) {
  const int lane = threadIdx.x & 63;
  const int64_t k = uniform((int32_t)(blockIdx.x * (kBS / 64) + (threadIdx.x >> 6)));
  if (k >= kn || kov[k]) return;
  const StageLayout& sl = *slp;
  const int32_t i = kcell[k];
  const int64_t e0 = (k - cbase[i]) * chunk;
  const int64_t e = gbeg[i] + e0;
  const int64_t n = min<int64_t>(chunk, gcnt[i] - e0);
  // source position j >= cap of list w (window capacity cap, spill shift sh):
  // the spill regions
  auto spilled = [&](int w, int64_t j, int64_t cap, int sh) {
    int64_t off;
    const int r = spill_region(j - cap, sh, &off);
    return sl.spill[w][sl.ksec[(3 * k + w) * kRegions + r] + off];
  };
  // list w to d: the window part with eight loads in flight per lane, then
  // the spill part
  auto copy = [&](int w, int32_t* __restrict__ d, int64_t cnt) {
    const int64_t lo = stage_lo(sl, w, e, k);
    const int64_t cap = stage_lo(sl, w, e + n, k + 1) - lo;
    const int64_t nw = cnt < cap ? cnt : cap;
    const int32_t* __restrict__ s = sl.win[w] + lo;
    int64_t j = lane;
    for (; j + 7 * 64 < nw; j += 8 * 64) {
      int32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = s[j + u * 64];
#pragma unroll
      for (int u = 0; u < 8; ++u) d[j + u * 64] = v[u];
    }
    for (; j < nw; j += 64) d[j] = s[j];
    if (cnt > cap) {
      const int sh = spill_shift(cap);
      for (j = nw + lane; j < cnt; j += 64) d[j] = spilled(w, j, cap, sh);
    }
  };
  const int64_t nm = mex[k + 1] - mex[k], np = pex[k + 1] - pex[k], nq = qex[k + 1] - qex[k];
  copy(0, far_src + far_base + mex[k], nm);
  copy(1, near_src + near_base + pex[k], np);
  if (nq) {
    const int32_t nch = load_cell(t.rec, c0 + i).nch;
    const int64_t S = qex[cbase[i + 1]] - qex[cbase[i]];
    int32_t* dq = fy_n + nbase[i] + (qex[k] - qex[cbase[i]]);
    const int64_t lo = stage_lo(sl, 2, e, k);
    const int64_t cap = stage_lo(sl, 2, e + n, k + 1) - lo;
    const int sh = spill_shift(cap);
    for (int64_t j = lane; j < nq; j += 64) {
      const int32_t v = j < cap ? sl.win[2][lo + j] : spilled(2, j, cap, sh);
      for (int32_t r = 0; r < nch; ++r) dq[r * S + j] = v;
    }
  }
}

// One wave per chunk whose staging overflowed: walk it again, writing its far
// and near entries and its children's entries straight to their places.
template <int EXT>
__global__ void __launch_bounds__(kBS) k_walk_emit(TreeView t, int32_t c0, int64_t kn, int32_t chunk,
                                                   const int32_t* __restrict__ kcell, const int64_t* __restrict__ cbase,
                                                   const int64_t* __restrict__ gbeg, const int32_t* __restrict__ gcnt,
                                                   const int32_t* __restrict__ fy, const int64_t* __restrict__ mex,
                                                   const int64_t* __restrict__ pex, const int64_t* __restrict__ qex,
                                                   const int64_t* __restrict__ nbase, const int32_t* __restrict__ kov,
                                                   int64_t far_base, int64_t near_base, int32_t* __restrict__ far_src,
                                                   int32_t* __restrict__ near_src, int32_t* __restrict__ fy_n,
                                                   int32_t* __restrict__ gq, int32_t qcap) {
  __shared__ int32_t queue[kBS / 64][kQ];
  __shared__ float model[EXT == kExtLearned ? AMFMM_MLP_MODEL : 1];
  if (EXT == kExtLearned) t.lmodel = stage_model(t.model, model);
  const int64_t k = uniform((int32_t)(xcd_block(blockIdx.x, gridDim.x) * (kBS / 64) + (threadIdx.x >> 6)));
  if (k >= kn || !kov[k]) return;
  const int32_t i = kcell[k];
  const int32_t X = c0 + i;
  const WalkCell cx = load_cell(t.rec, X);
  const int64_t e0 = (k - cbase[i]) * chunk;
  const int32_t n = (int32_t)min<int64_t>(chunk, gcnt[i] - e0);
  const int64_t S = qex[cbase[i + 1]] - qex[cbase[i]];
  int64_t tm = 0, tp = 0, tq = 0, td = 0;
  EmitDst dst{far_base + mex[k], near_base + pex[k], nbase[i], S, far_src, near_src, fy_n,
              qex[k] - qex[cbase[i]], nullptr, {}, {}, k, nullptr};
  if (gq)
    wave_walk<kEmit, EXT>(t, X, cx, fy, gbeg[i] + e0, n, gq + k * qcap, qcap, tm, tp, tq, td, dst, nullptr);
  else
    wave_walk<kEmit, EXT>(t, X, cx, fy, gbeg[i] + e0, n, queue[threadIdx.x >> 6], kQ, tm, tp, tq, td, dst, nullptr);
}

__global__ void k_walk_init(int64_t* gbeg, int32_t* gcnt, int32_t* fy) {
  gbeg[0] = 0;
  gcnt[0] = 1;
  fy[0] = 0;
}

__global__ void k_gather_totals(const int64_t* mex, const int64_t* pex, const int64_t* qex, const int64_t* nbase,
                                const int64_t* kdex, int64_t kmax, int32_t nl, int64_t* out) {
  out[0] = mex[kmax];
  out[1] = pex[kmax];
  out[2] = nbase[nl];
  out[3] = qex[kmax];
  out[5] = kdex[kmax];
}

}  // namespace

void walk_prepare(Ctx& c, double theta) {
  const int32_t nc = c.ncells;
  WalkRec* rec = (WalkRec*)ensure(c, c.walkrec, sizeof(WalkRec) * (size_t)nc);
  const double* gmin = nullptr;
  c.walk_mode = 0;
  if (c.field && c.opt.criterion == AMFMM_ESTIMATE) c.walk_mode = 1;
  if (c.field && c.opt.criterion == AMFMM_LEARNED && c.model.p) c.walk_mode = 2;
  if (c.field && c.opt.criterion == AMFMM_MULTIPOLE) c.walk_mode = 3;
  if (c.walk_mode != 0) {
    double* gs = (double*)ensure(c, c.gmin, 4 * sizeof(double) * nc);
    double* gm = gs + nc;
    double* g = gm + nc;
    double* mm = g + nc;
    hipLaunchKernelGGL(k_mmin_leaves, dim3(blocks_for(c.nleaves, kBS)), dim3(kBS), 0, c.stream,
                       as<int32_t>(c.leaves), c.nleaves, (const double*)c.mom.p, mm);
    for (int l = c.depth - 1; l >= 0; --l) {
      const int32_t c0 = c.level_start[l], nl = c.level_start[l + 1] - c0;
      hipLaunchKernelGGL(k_mmin_up, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, c0, nl,
                         as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild), mm);
    }
    hipLaunchKernelGGL(k_gsum_leaves, dim3(blocks_for(c.nleaves, kBS)), dim3(kBS), 0, c.stream,
                       as<int32_t>(c.leaves), c.nleaves, as<int32_t>(c.c_begin), as<int32_t>(c.c_count),
                       as<int32_t>(c.perm), c.field, c.field_y, c.field_z, gs, gm);
    for (int l = c.depth - 1; l >= 0; --l) {
      const int32_t c0 = c.level_start[l], nl = c.level_start[l + 1] - c0;
      hipLaunchKernelGGL(k_gsum_up, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, c0, nl,
                         as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild), gs, gm);
    }
    hipLaunchKernelGGL(k_gscale, dim3(blocks_for(nc, kBS)), dim3(kBS), 0, c.stream, nc, as<int32_t>(c.c_count),
                       (const double*)gs, (const double*)gm, g);
    gmin = g;
  }
  hipLaunchKernelGGL(k_pack_cells, dim3(blocks_for(nc, kBS)), dim3(kBS), 0, c.stream, nc, (const double4*)c.geo.p,
                     (const double*)c.mom.p, as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild),
                     as<int32_t>(c.c_parent), as<int32_t>(c.c_count), gmin, rec);
  AMFMM_HIP(hipGetLastError());
  ensure(c, c.far_start, sizeof(int64_t) * nc);
  ensure(c, c.far_count, sizeof(int32_t) * nc);
  ensure(c, c.near_start, sizeof(int64_t) * nc);
  ensure(c, c.near_count, sizeof(int32_t) * nc);
  int32_t maxw = 1;
  for (size_t l = 0; l + 1 < c.level_start.size(); ++l)
    maxw = std::max(maxw, c.level_start[l + 1] - c.level_start[l]);
  c.grp_width = maxw + 1;
  ensure(c, c.grp, 2 * (sizeof(int64_t) + sizeof(int32_t)) * (size_t)c.grp_width);
  ensure(c, c.fy, sizeof(int32_t) * 16);
  c.theta = theta;
  double box[6];
  AMFMM_HIP(hipMemcpyAsync(box, c.bbox.p, sizeof(box), hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
  double scale = 0.0;
  for (double v : box) scale = std::max(scale, std::fabs(v));
  c.walk_abs_tol = 1e-9 * scale;
}

// the two group arrays (current, next) of the level ping-pong inside c.grp
static void group_ptrs(Ctx& c, int which, int64_t** gbeg, int32_t** gcnt) {
  int64_t* g64 = (int64_t*)c.grp.p;
  int32_t* g32 = (int32_t*)(g64 + 2 * c.grp_width);
  *gbeg = g64 + which * c.grp_width;
  *gcnt = g32 + which * c.grp_width;
}

void group_arrays(Ctx& c, int64_t** gbeg, int32_t** gcnt) { group_ptrs(c, c.grp_cur, gbeg, gcnt); }

void walk_start(Ctx& c) {
  int64_t* gbeg;
  int32_t* gcnt;
  group_ptrs(c, 0, &gbeg, &gcnt);
  c.grp_cur = 0;
  hipLaunchKernelGGL(k_walk_init, dim3(1), dim3(1), 0, c.stream, gbeg, gcnt, as<int32_t>(c.fy));
  AMFMM_HIP(hipGetLastError());
  c.frontier = 1;
  c.walk_candidates = 0;
  c.pass_launches = 0;
}

// Staging room of a level.  Expected terminal pairs per entry: those the
// level produced the last time it was walked under the same rule (windows
// 1.5x that), else the level above's in this walk (2.5x), else a default;
// plus a slack per chunk.  Spill pools: as large as the windows, plus a
// minimal spill region for one chunk in 16.  The whole is held
// within `limit` bytes (scaled down; below a quarter of the wanted size no
// staging: every chunk with output is emitted by the second pass).  Returns
// the bytes: the spill region offsets (3 kRegions int64 per chunk), then
// windows and spill pools.
static size_t stage_layout(Ctx& c, int lev, int64_t F, int64_t kn, const double* prev, size_t limit,
                           StageLayout& sl) {
  double r[3] = {4.0, 1.0, 2.0}, alpha = 1.0;
  const size_t at = 3 * (size_t)lev;
  if (at + 2 < c.walk_ratio.size() && c.walk_ratio[at] >= 0.0) {
    for (int w = 0; w < 3; ++w) r[w] = c.walk_ratio[at + w];
    alpha = 1.5;
  } else if (prev) {
    for (int w = 0; w < 3; ++w) r[w] = prev[w];
    alpha = 2.5;
  }
  constexpr double kSpill = 1.0;
  const int64_t slack[3] = {32, 8, 8};
  const double offsets = 3.0 * kRegions * sizeof(int64_t) * (double)kn;
  double ints = 0.0;
  for (int w = 0; w < 3; ++w)
    ints += (1.0 + kSpill) * (alpha * r[w] * (double)F + (double)(kn * slack[w])) + (double)(kn / 16 * kSpillMin);
  double scale = 1.0;
  if (ints * sizeof(int32_t) + offsets > (double)limit)
    scale = std::max(0.0, ((double)limit - offsets) / (ints * sizeof(int32_t)));
  if (scale < 0.25) scale = 0.0;
  // AMFMM_WALK_WINDOWS (tests): a factor on the windows alone, to drive chunks
  // into the spill regions (small factors) or the second pass (0)
  double wf = 1.0;
  if (const char* e = getenv("AMFMM_WALK_WINDOWS")) wf = std::max(0.0, std::min(1.0, atof(e)));
  size_t n = 0;
  for (int w = 0; w < 3; ++w) {
    sl.cap16[w] = (int64_t)std::ceil(16.0 * alpha * r[w] * scale * wf);
    sl.slack[w] = (int64_t)((double)slack[w] * scale * wf);
    const int64_t win = ((sl.cap16[w] * F) >> 4) + kn * sl.slack[w] + 1;
    sl.spill_cap[w] = (int64_t)(kSpill * (double)win + scale * (double)(kn / 16 * kSpillMin));
    n += (size_t)(win + sl.spill_cap[w]);
  }
  return sizeof(int32_t) * n + 3 * kRegions * sizeof(int64_t) * (size_t)kn + 64;
}

__global__ void k_set_layout(StageLayout v, StageLayout* out) { *out = v; }

int64_t walk_levels(Ctx& c, int lev_first, int lev_last, const std::vector<int32_t>& lo,
                    const std::vector<int32_t>& hi, int64_t& far_base, int64_t& near_base) {
  TreeView t{(const WalkRec*)c.walkrec.p, c.theta, c.walk_abs_tol, c.walk_mode, c.opt.error_tol,
             c.opt.theta_max, c.opt.theta_max * c.opt.theta_max, (const float*)c.model.p, c.opt.learned_min_work,
             c.walk_mode != 0 ? (const double*)c.gmin.p + 3 * (size_t)c.ncells : nullptr, nullptr};
  static const bool debug_env = getenv("AMFMM_DEBUG_WALK") != nullptr;
  const bool debug = debug_env && !c.arena;  // no events in an allocation-free solve
  const int ext = c.walk_mode == 2 ? kExtLearned : (c.walk_mode == 3 ? kExtMultipole : kExtBase);
  // per-level ratios of terminal pairs to entries, kept while the rule stays the same
  const double key[4] = {(double)c.walk_mode, c.theta, c.opt.error_tol, c.opt.theta_max};
  if (!std::equal(key, key + 4, c.walk_ratio_key) || c.walk_ratio.size() < 3 * lo.size()) {
    std::copy(key, key + 4, c.walk_ratio_key);
    c.walk_ratio.assign(3 * lo.size(), -1.0);
  }
  // staging room: a third of the free device memory, at most 64 GiB
  const size_t fr = free_device_bytes(c);
  // (the staging buffer of an earlier walk is given back when it grows; in an
  // arena its block need not join the largest free one)
  const size_t stage_limit = std::min<size_t>(fr / 3 + (c.arena ? 0 : c.stage.cap), size_t(64) << 30);
  // global work queues: at most kGlobalQueueBytes, an eighth of an arena
  const int64_t queue_limit = c.arena ? (int64_t)(fr / 8) : kGlobalQueueBytes;
  double prev[3];
  bool have_prev = false;
  int64_t cand = 0;  // candidate pairs, counted once the levels are done (a batch over budget is walked again)
  int64_t F = c.frontier;
  int64_t* tot_host = c.pinned;
  for (int lev = lev_first; lev <= lev_last && F > 0; ++lev) {
    const int32_t c0 = lo[lev], nl = hi[lev] - lo[lev];
    const int32_t c0n = lev + 1 < (int)lo.size() ? lo[lev + 1] : 0;
    const size_t L = (size_t)nl + 1;
    // enough waves to fill the chip (small frontiers: one entry per wave),
    // few enough that dispatch does not dominate
    const int32_t chunk = (int32_t)std::min<int64_t>(kChunkMax, std::max<int64_t>(1, (F + kWavesPerLevel - 1) / kWavesPerLevel));
    const int64_t kmax = F / chunk + nl + 1;  // upper bound on the chunks
    const size_t K = (size_t)kmax + 1;
    int64_t *gbeg, *gbeg_n;
    int32_t *gcnt, *gcnt_n;
    group_ptrs(c, c.grp_cur, &gbeg, &gcnt);
    group_ptrs(c, 1 - c.grp_cur, &gbeg_n, &gcnt_n);
    int64_t* w = (int64_t*)ensure(c, c.scratch2, sizeof(int64_t) * (4 * L + 9 * K + 48));
    int64_t *nck = w, *cbase = nck + L, *ns = cbase + L, *nbase = ns + L;
    int64_t *km = nbase + L, *kp = km + K, *kq = kp + K, *mex = kq + K, *pex = mex + K, *qex = pex + K;
    int32_t* kov = (int32_t*)(qex + K);
    int64_t *kd = qex + 2 * K, *kdex = kd + K;  // candidate pairs per chunk, and their scan
    // [0..3] totals, [4] chunks out of room, [5] candidate pairs, [8..10] spill
    // used, [12..16] debug counters, [20..] the staging layout
    int64_t* tot = qex + 4 * K;
    const int32_t* fy = as<int32_t>(c.fy);
    hipLaunchKernelGGL(k_chunk_counts, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, nl, (const int32_t*)gcnt,
                       chunk, nck);
    AMFMM_HIP(hipGetLastError());
    scan_i64(c, nck, cbase, nl);
    AMFMM_HIP(hipMemcpyAsync(tot_host, cbase + nl, sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
    AMFMM_HIP(hipStreamSynchronize(c.stream));
    const int64_t kn = tot_host[0];
    int32_t* kcell = (int32_t*)ensure(c, c.fx, sizeof(int32_t) * (kn + 1));
    hipLaunchKernelGGL(k_chunk_map, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, nl, (const int64_t*)cbase,
                       kcell);
    const unsigned kgrid = blocks_for(kn, kBS / 64);
    // few chunks: a larger work queue per wave, in global memory
    int32_t* gq = nullptr;
    int32_t qcap = kQ;
    {
      int64_t g = kGlobalQueueMax;
      while (g > 4 * kQ && (int64_t)sizeof(int32_t) * g * kn > queue_limit) g >>= 1;
      if ((int64_t)sizeof(int32_t) * g * kn <= queue_limit) {
        qcap = (int32_t)g;
        gq = (int32_t*)ensure(c, c.gqueue, sizeof(int32_t) * (size_t)kn * qcap);
      }
    }
    StageLayout sl{};
    const size_t stage_bytes = stage_layout(c, lev, F, kn, have_prev ? prev : nullptr, stage_limit, sl);
    {
      int64_t* st64 = (int64_t*)ensure(c, c.stage, stage_bytes);
      sl.ksec = st64;
      int32_t* st = (int32_t*)(st64 + 3 * kRegions * kn);
      for (int w = 0; w < 3; ++w) {
        sl.win[w] = st;
        st += ((sl.cap16[w] * F) >> 4) + kn * sl.slack[w] + 1;
        sl.spill[w] = st;
        st += sl.spill_cap[w];
      }
    }
    unsigned long long* nov = (unsigned long long*)(tot + 4);
    sl.used = (unsigned long long*)(tot + 8);
    unsigned long long* dbg = debug ? (unsigned long long*)(tot + 12) : nullptr;
    StageLayout* sl_dev = (StageLayout*)(tot + 20);
    static_assert(20 + sizeof(StageLayout) / sizeof(int64_t) <= 48, "walk totals");
    zero_u64(c, nov, 16);
    hipLaunchKernelGGL(k_set_layout, dim3(1), dim3(1), 0, c.stream, sl, sl_dev);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (debug) {
      AMFMM_HIP(hipEventCreate(&e0));
      AMFMM_HIP(hipEventCreate(&e1));
      AMFMM_HIP(hipEventRecord(e0, c.stream));
    }
    mark(c, kPhWalkPass);
    hipLaunchKernelGGL(ext == kExtLearned     ? k_walk_stage<kExtLearned>
                       : ext == kExtMultipole ? k_walk_stage<kExtMultipole>
                                              : k_walk_stage<kExtBase>,
                       dim3(kgrid), dim3(kBS), 0, c.stream, t, c0, kn, chunk, (const int32_t*)kcell,
                       (const int64_t*)cbase, (const int64_t*)gbeg, (const int32_t*)gcnt, fy,
                       (const StageLayout*)sl_dev, km, kp, kq, kov, kd, nov, gq, qcap, dbg);
    ++c.pass_launches;
    mark(c, kPhWalk);
    AMFMM_HIP(hipGetLastError());
    if (debug) AMFMM_HIP(hipEventRecord(e1, c.stream));
    scan_i64(c, km, mex, kn);
    scan_i64(c, kp, pex, kn);
    scan_i64(c, kq, qex, kn);
    scan_i64(c, kd, kdex, kn);
    hipLaunchKernelGGL(k_walk_cells, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, t, c0, nl, c0n,
                       (const int64_t*)cbase, (const int64_t*)mex, (const int64_t*)pex, (const int64_t*)qex, far_base,
                       near_base, (int64_t*)c.far_start.p, (int32_t*)c.far_count.p, (int64_t*)c.near_start.p,
                       (int32_t*)c.near_count.p, ns);
    AMFMM_HIP(hipGetLastError());
    scan_i64(c, ns, nbase, nl);
    hipLaunchKernelGGL(k_walk_groups, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, t, c0, nl, c0n,
                       (const int64_t*)cbase, (const int64_t*)qex, (const int64_t*)nbase, gbeg_n, gcnt_n);
    hipLaunchKernelGGL(k_gather_totals, dim3(1), dim3(1), 0, c.stream, (const int64_t*)mex, (const int64_t*)pex,
                       (const int64_t*)qex, (const int64_t*)nbase, (const int64_t*)kdex, kn, nl, tot);
    AMFMM_HIP(hipGetLastError());
    AMFMM_HIP(hipMemcpyAsync(tot_host, tot, sizeof(int64_t) * 6, hipMemcpyDeviceToHost, c.stream));
    AMFMM_HIP(hipStreamSynchronize(c.stream));
    const int64_t mt = tot_host[0], pt = tot_host[1], Fn = tot_host[2], qt = tot_host[3], novh = tot_host[4];
    cand += tot_host[5];
    if (debug) {
      unsigned long long h[5];
      AMFMM_HIP(hipMemcpy(h, dbg, sizeof(h), hipMemcpyDeviceToHost));
      float ms = 0.f;
      AMFMM_HIP(hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      fprintf(stderr,
              "walk level %d: cells %d entries %lld chunks %lld (x%d) far %lld near %lld next %lld | staging pass "
              "%.3f ms, steps %llu, pairs %llu, deep %llu, asked %llu in %llu steps, overflowed %lld\n",
              lev, nl, (long long)F, (long long)kn, chunk, (long long)mt, (long long)pt, (long long)Fn, ms, h[0],
              h[2], h[1], h[3], h[4], (long long)novh);
    }
    prev[0] = (double)mt / (double)F;
    prev[1] = (double)pt / (double)F;
    prev[2] = (double)qt / (double)F;
    have_prev = true;
    if ((size_t)lev < lo.size()) std::copy(prev, prev + 3, c.walk_ratio.begin() + 3 * (size_t)lev);
    if (Fn >= (int64_t(1) << 34)) throw BudgetExceeded();
    if (c.walk_budget &&
        (double)sizeof(int32_t) * (double)(far_base + mt + near_base + pt + 2 * Fn) > (double)c.walk_budget)
      throw BudgetExceeded();
    int32_t* far_src = (int32_t*)ensure_keep(c, c.far_src, sizeof(int32_t) * (far_base + mt + 1),
                                             sizeof(int32_t) * far_base);
    int32_t* near_src = (int32_t*)ensure_keep(c, c.near_src, sizeof(int32_t) * (near_base + pt + 1),
                                              sizeof(int32_t) * near_base);
    int32_t* fy_n = (int32_t*)ensure(c, c.fy2, sizeof(int32_t) * (Fn + 1));
    if (novh < kn)
      hipLaunchKernelGGL(k_walk_compact, dim3(blocks_for(kn, kBS / 64)), dim3(kBS), 0, c.stream, t, c0, kn, chunk,
                         (const int32_t*)kcell, (const int64_t*)cbase, (const int64_t*)gbeg, (const int32_t*)gcnt,
                         (const StageLayout*)sl_dev, (const int64_t*)mex,
                         (const int64_t*)pex, (const int64_t*)qex, (const int64_t*)nbase, (const int32_t*)kov,
                         far_base, near_base, far_src, near_src, fy_n);
    if (novh > 0)
      hipLaunchKernelGGL(ext == kExtLearned     ? k_walk_emit<kExtLearned>
                         : ext == kExtMultipole ? k_walk_emit<kExtMultipole>
                                                : k_walk_emit<kExtBase>,
                         dim3(kgrid), dim3(kBS), 0, c.stream, t, c0, kn, chunk, (const int32_t*)kcell,
                         (const int64_t*)cbase, (const int64_t*)gbeg, (const int32_t*)gcnt, fy, (const int64_t*)mex,
                         (const int64_t*)pex, (const int64_t*)qex, (const int64_t*)nbase, (const int32_t*)kov,
                         far_base, near_base, far_src, near_src, fy_n, gq, qcap);
    AMFMM_HIP(hipGetLastError());
    far_base += mt;
    near_base += pt;
    std::swap(c.fy, c.fy2);
    c.grp_cur = 1 - c.grp_cur;
    F = Fn;
  }
  c.frontier = F;
  c.walk_candidates += cand;
  return F;
}

void dual_walk(Ctx& c, double theta) {
  walk_prepare(c, theta);
  walk_start(c);
  std::vector<int32_t> lo(c.level_start.begin(), c.level_start.end() - 1),
      hi(c.level_start.begin() + 1, c.level_start.end());
  int64_t far_base = 0, near_base = 0;
  walk_levels(c, 0, c.depth, lo, hi, far_base, near_base);
  c.n_far = far_base;
  c.n_near = near_base;
  c.have_lists = true;
}

}  // namespace amfmm
