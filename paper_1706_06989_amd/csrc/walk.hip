// Interaction selection (Sec. 2): symmetric dual walk under the opening
// criterion |Z_A - Z_B| >= (R_A + R_B)/theta, organised by target cell.
//
// The walk of cell pairs is reproduced pair for pair, but every visited pair
// is held twice, once by each of its cells (directed entries (X, Y)), and the
// frontier is processed one tree level of X at a time, grouped by X.  For an
// entry (X, Y) a thread runs a depth-first descent into Y's subtree while the
// symmetric split rule opens Y; each terminal pair ends as
//   * a far-field entry X <- Y when accepted,
//   * a near-field entry X <- Y when both are leaves,
//   * a "split X" base that hands (X_c, Y) to every child X_c of X.
// A self entry (X, X) of a split cell hands (X_c, X_c') to every child for all
// children X_c' (self included); of a leaf it becomes the near-field entry X<-X.
// The decision on a pair depends only on the unordered pair (the criterion is
// symmetric and the split rule picks the larger R_max, ties to the lower
// index, and the non-leaf when one is a leaf), so both cells of a pair make
// the same decision and every directed list comes out grouped by target with
// no sort: count pass -> scans -> emit pass, deterministic.
//
// Compiled with -ffp-contract=off: the criterion must round exactly as the
// plain definition does.
#include <cstdio>
#include <cstdlib>

#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;

enum : int { kAccept = 0, kNear = 1, kSplitX = 2, kSplitY = 3 };

// per cell, everything a walk step reads, in one 48-byte record
struct alignas(16) WalkCell {
  double gx, gy, gz, gw;  // centre of mass, R_max
  int32_t ch0;    // first child (-1 for leaves)
  int32_t nch;    // child count
  int32_t par;    // parent
  int32_t next;   // next sibling, -1 for the last child
};

struct TreeView {
  const WalkCell* rec;
  double theta;
};

__device__ inline WalkCell load_cell(const WalkCell* __restrict__ r, int32_t c) {
  const double2* p = reinterpret_cast<const double2*>(r + c);
  const int4* q = reinterpret_cast<const int4*>(reinterpret_cast<const char*>(r + c) + 32);
  WalkCell w;
  const double2 p0 = p[0], p1 = p[1];
  w.gx = p0.x;
  w.gy = p0.y;
  w.gz = p1.x;
  w.gw = p1.y;
  int4 v = q[0];
  w.ch0 = v.x;
  w.nch = v.y;
  w.par = v.z;
  w.next = v.w;
  return w;
}

__device__ inline int decide(const TreeView& t, int32_t X, const WalkCell& a, int32_t Y, const WalkCell& b) {
  const double dx = a.gx - b.gx, dy = a.gy - b.gy, dz = a.gz - b.gz;
  const double d = sqrt((dx * dx + dy * dy) + dz * dz);
  const double rhs = (a.gw + b.gw) / t.theta;
  if (d > 0.0 && d >= rhs) return kAccept;
  const bool lx = a.nch == 0, ly = b.nch == 0;
  if (lx && ly) return kNear;
  if (lx) return kSplitY;
  if (ly) return kSplitX;
  if (a.gw > b.gw) return kSplitX;
  if (a.gw < b.gw) return kSplitY;
  return X < Y ? kSplitX : kSplitY;
}

// Visits the terminal pairs of entry (X, Y) in depth-first order (children of
// Y in octant order) and calls f(kind, Y') for each.
template <typename F>
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
    int d = decide(t, X, a, cur, b);
    if (d == kSplitY) {
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
                                                    const int32_t* __restrict__ ch0, const int32_t* __restrict__ nch,
                                                    const int32_t* __restrict__ par, WalkCell* __restrict__ rec) {
  int32_t c = blockIdx.x * kBS + threadIdx.x;
  if (c >= nc) return;
  WalkCell w;
  const double4 g = geo[c];
  w.gx = g.x;
  w.gy = g.y;
  w.gz = g.z;
  w.gw = g.w;
  w.ch0 = nch[c] ? ch0[c] : -1;
  w.nch = nch[c];
  const int32_t p = par[c];
  w.par = p;
  w.next = (p >= 0 && c + 1 < ch0[p] + nch[p]) ? c + 1 : -1;
  rec[c] = w;
}

__device__ inline int32_t wave_excl_scan(int32_t v, int32_t* total) {
  const int lane = threadIdx.x & 63;
  int32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  *total = __shfl(inc, 63, 64);
  return inc - v;
}

__device__ inline int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

constexpr int kQ = 1024;  // per-wave LDS work queue (power of two)

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct EmitDst {
  int64_t fo, no, nb, S;
  int32_t* far_src;
  int32_t* near_src;
  int32_t* fy_n;
};

// All pairs held by target cell X at this level, processed by one wave
// breadth-first: each step gives every lane one pair (taken first from the
// wave's queue, else from X's frontier entries); a pair whose rule opens Y
// pushes Y's children to the queue; when the queue is full the lane descends
// Y's subtree itself.  The order is a fixed function of the inputs, so the
// counting run and the emitting run visit the same pairs in the same order.
template <bool EMIT>
__device__ inline void wave_walk(const TreeView& t, int32_t X, const WalkCell& cx, const int32_t* __restrict__ fy,
                                 int64_t b, int32_t n, int32_t* qbuf, int64_t& tm, int64_t& tp, int64_t& tq,
                                 EmitDst dst) {
  const int lane = threadIdx.x & 63;
  int32_t head = 0, tail = 0, fpos = 0;
  int64_t fo = dst.fo, no = dst.no, B = 0;
  while (head < tail || fpos < n) {
    int32_t Y = -1;
    if (head < tail) {
      const int k = min(64, tail - head);
      if (lane < k) Y = qbuf[(head + lane) & (kQ - 1)];
      head += k;
    } else {
      const int k = min(64, n - fpos);
      if (lane < k) Y = fy[b + fpos + lane];
      fpos += k;
    }
    wave_sync();  // queue slots just read may be reused by this step's pushes
    int32_t m = 0, p = 0, q = 0, push = 0, ych0 = 0;
    bool self = false;
    if (Y >= 0) {
      if (Y == X) {
        self = true;
        if (cx.nch == 0) p = 1;
        else q = cx.nch;
      } else {
        const WalkCell cy = load_cell(t.rec, Y);
        const int d = decide(t, X, cx, Y, cy);
        m = d == kAccept;
        p = d == kNear;
        q = d == kSplitX;
        if (d == kSplitY) {
          push = cy.nch;
          ych0 = cy.ch0;
        }
      }
    }
    int32_t ptot;
    const int32_t poff = wave_excl_scan(push, &ptot);
    const int32_t freeq = kQ - (tail - head);
    const bool fits = poff + push <= freeq;
    const uint64_t over = __ballot(push > 0 && !fits);
    const int32_t pushed = over ? __shfl(poff, __ffsll((unsigned long long)over) - 1, 64) : ptot;
    if (push > 0 && fits)
      for (int32_t j = 0; j < push; ++j) qbuf[(tail + poff + j) & (kQ - 1)] = ych0 + j;
    tail += pushed;
    wave_sync();
    const bool deep = push > 0 && !fits;  // queue full: descend in this lane
    if (deep)
      traverse(t, X, Y, [&](int d, int32_t) {
        m += d == kAccept;
        p += d == kNear;
        q += d == kSplitX;
      });
    if (!EMIT) {
      tm += m;
      tp += p;
      tq += q;
    } else {
      int32_t Tm, Tp, Tq;
      const int32_t om = wave_excl_scan(m, &Tm);
      const int32_t op = wave_excl_scan(p, &Tp);
      const int32_t oq = wave_excl_scan(q, &Tq);
      if (deep) {
        int64_t f = fo + om, g = no + op, bb = B + oq;
        traverse(t, X, Y, [&](int d, int32_t Z) {
          if (d == kAccept) {
            dst.far_src[f++] = Z;
          } else if (d == kNear) {
            dst.near_src[g++] = Z;
          } else {
            for (int32_t r = 0; r < cx.nch; ++r) dst.fy_n[dst.nb + r * dst.S + bb] = Z;
            ++bb;
          }
        });
      } else if (self) {
        if (p) dst.near_src[no + op] = X;
        for (int32_t j = 0; j < q; ++j)
          for (int32_t r = 0; r < cx.nch; ++r) dst.fy_n[dst.nb + r * dst.S + B + oq + j] = cx.ch0 + j;
      } else if (m) {
        dst.far_src[fo + om] = Y;
      } else if (p) {
        dst.near_src[no + op] = Y;
      } else if (q) {
        for (int32_t r = 0; r < cx.nch; ++r) dst.fy_n[dst.nb + r * dst.S + B + oq] = Y;
      }
      fo += Tm;
      no += Tp;
      B += Tq;
    }
  }
}

__global__ void __launch_bounds__(kBS) k_walk_count(TreeView t, int32_t c0, int32_t nl,
                                                    const int64_t* __restrict__ gbeg, const int32_t* __restrict__ gcnt,
                                                    const int32_t* __restrict__ fy, int64_t* __restrict__ cm,
                                                    int64_t* __restrict__ cp, int64_t* __restrict__ cq,
                                                    int64_t* __restrict__ ns) {
  __shared__ int32_t queue[kBS / 64][kQ];
  const int lane = threadIdx.x & 63;
  const int32_t i = blockIdx.x * (kBS / 64) + (threadIdx.x >> 6);
  if (i >= nl) return;
  const int32_t X = c0 + i;
  const WalkCell cx = load_cell(t.rec, X);
  int64_t tm = 0, tp = 0, tq = 0;
  wave_walk<false>(t, X, cx, fy, gbeg[i], gcnt[i], queue[threadIdx.x >> 6], tm, tp, tq, EmitDst{});
  tm = wave_sum64(tm);
  tp = wave_sum64(tp);
  tq = wave_sum64(tq);
  if (lane == 0) {
    cm[i] = tm;
    cp[i] = tp;
    cq[i] = tq;
    ns[i] = (int64_t)cx.nch * tq;
  }
}

__global__ void __launch_bounds__(kBS) k_walk_emit(TreeView t, int32_t c0, int32_t nl, int32_t c0n,
                                                   const int64_t* __restrict__ gbeg, const int32_t* __restrict__ gcnt,
                                                   const int32_t* __restrict__ fy, const int64_t* __restrict__ cm,
                                                   const int64_t* __restrict__ cp, const int64_t* __restrict__ cq,
                                                   const int64_t* __restrict__ mex, const int64_t* __restrict__ pex,
                                                   const int64_t* __restrict__ nbase, int64_t far_base,
                                                   int64_t near_base, int64_t* __restrict__ far_start,
                                                   int32_t* __restrict__ far_count, int64_t* __restrict__ near_start,
                                                   int32_t* __restrict__ near_count, int32_t* __restrict__ far_src,
                                                   int32_t* __restrict__ near_src, int64_t* __restrict__ gbeg_n,
                                                   int32_t* __restrict__ gcnt_n, int32_t* __restrict__ fy_n) {
  __shared__ int32_t queue[kBS / 64][kQ];
  const int lane = threadIdx.x & 63;
  const int32_t i = blockIdx.x * (kBS / 64) + (threadIdx.x >> 6);
  if (i >= nl) return;
  const int32_t X = c0 + i;
  const WalkCell cx = load_cell(t.rec, X);
  const int64_t S = cq[i], nb = nbase[i];
  if (lane == 0) {
    far_start[X] = far_base + mex[i];
    far_count[X] = (int32_t)cm[i];
    near_start[X] = near_base + pex[i];
    near_count[X] = (int32_t)cp[i];
  }
  for (int32_t r = lane; r < cx.nch; r += 64) {
    gbeg_n[cx.ch0 + r - c0n] = nb + r * S;
    gcnt_n[cx.ch0 + r - c0n] = (int32_t)S;
  }
  int64_t tm = 0, tp = 0, tq = 0;
  EmitDst dst{far_base + mex[i], near_base + pex[i], nb, S, far_src, near_src, fy_n};
  wave_walk<true>(t, X, cx, fy, gbeg[i], gcnt[i], queue[threadIdx.x >> 6], tm, tp, tq, dst);
}

__global__ void k_walk_init(int64_t* gbeg, int32_t* gcnt, int32_t* fy) {
  gbeg[0] = 0;
  gcnt[0] = 1;
  fy[0] = 0;
}

__global__ void k_gather_totals(const int64_t* mex, const int64_t* pex, const int64_t* nbase, int32_t nl,
                                int64_t* out) {
  out[0] = mex[nl];
  out[1] = pex[nl];
  out[2] = nbase[nl];
}

}  // namespace

void walk_prepare(Ctx& c, double theta) {
  const int32_t nc = c.ncells;
  WalkCell* rec = (WalkCell*)ensure(c, c.walkrec, sizeof(WalkCell) * (size_t)nc);
  hipLaunchKernelGGL(k_pack_cells, dim3(blocks_for(nc, kBS)), dim3(kBS), 0, c.stream, nc, (const double4*)c.geo.p,
                     as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild), as<int32_t>(c.c_parent), rec);
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
}

int64_t walk_levels(Ctx& c, int lev_first, int lev_last, const std::vector<int32_t>& lo,
                    const std::vector<int32_t>& hi, int64_t& far_base, int64_t& near_base) {
  TreeView t{(const WalkCell*)c.walkrec.p, c.theta};
  static const bool debug = getenv("AMFMM_DEBUG_WALK") != nullptr;
  int64_t F = c.frontier;
  int64_t* tot_host = c.pinned;
  for (int lev = lev_first; lev <= lev_last && F > 0; ++lev) {
    const int32_t c0 = lo[lev], nl = hi[lev] - lo[lev];
    const int32_t c0n = lev + 1 < (int)lo.size() ? lo[lev + 1] : 0;
    const size_t L = (size_t)nl + 1;
    int64_t *gbeg, *gbeg_n;
    int32_t *gcnt, *gcnt_n;
    group_ptrs(c, c.grp_cur, &gbeg, &gcnt);
    group_ptrs(c, 1 - c.grp_cur, &gbeg_n, &gcnt_n);
    int64_t* w = (int64_t*)ensure(c, c.scratch2, sizeof(int64_t) * (7 * L + 4));
    int64_t *cm = w, *cp = cm + L, *cq = cp + L, *ns = cq + L, *mex = ns + L, *pex = mex + L, *nbase = pex + L;
    int64_t* tot = nbase + L;
    const int32_t* fy = as<int32_t>(c.fy);
    const unsigned grid = blocks_for(nl, kBS / 64);
    hipLaunchKernelGGL(k_walk_count, dim3(grid), dim3(kBS), 0, c.stream, t, c0, nl, (const int64_t*)gbeg,
                       (const int32_t*)gcnt, fy, cm, cp, cq, ns);
    AMFMM_HIP(hipGetLastError());
    scan_i64(c, cm, mex, nl);
    scan_i64(c, cp, pex, nl);
    scan_i64(c, ns, nbase, nl);
    hipLaunchKernelGGL(k_gather_totals, dim3(1), dim3(1), 0, c.stream, (const int64_t*)mex, (const int64_t*)pex,
                       (const int64_t*)nbase, nl, tot);
    AMFMM_HIP(hipGetLastError());
    AMFMM_HIP(hipMemcpyAsync(tot_host, tot, sizeof(int64_t) * 3, hipMemcpyDeviceToHost, c.stream));
    AMFMM_HIP(hipStreamSynchronize(c.stream));
    const int64_t mt = tot_host[0], pt = tot_host[1], Fn = tot_host[2];
    if (debug)
      fprintf(stderr, "walk level %d: cells %d entries %lld far %lld near %lld next %lld\n", lev, nl, (long long)F,
              (long long)mt, (long long)pt, (long long)Fn);
    if (Fn >= (int64_t)INT32_MAX) throw Error(AMFMM_E_OOM, "walk frontier exceeds 2^31 entries");
    int32_t* far_src = (int32_t*)ensure_keep(c, c.far_src, sizeof(int32_t) * (far_base + mt + 1),
                                             sizeof(int32_t) * far_base);
    int32_t* near_src = (int32_t*)ensure_keep(c, c.near_src, sizeof(int32_t) * (near_base + pt + 1),
                                              sizeof(int32_t) * near_base);
    int32_t* fy_n = (int32_t*)ensure(c, c.fy2, sizeof(int32_t) * (Fn + 1));
    hipLaunchKernelGGL(k_walk_emit, dim3(grid), dim3(kBS), 0, c.stream, t, c0, nl, c0n, (const int64_t*)gbeg,
                       (const int32_t*)gcnt, fy, (const int64_t*)cm, (const int64_t*)cp, (const int64_t*)cq,
                       (const int64_t*)mex, (const int64_t*)pex, (const int64_t*)nbase, far_base, near_base,
                       (int64_t*)c.far_start.p, (int32_t*)c.far_count.p, (int64_t*)c.near_start.p,
                       (int32_t*)c.near_count.p, far_src, near_src, gbeg_n, gcnt_n, fy_n);
    AMFMM_HIP(hipGetLastError());
    far_base += mt;
    near_base += pt;
    std::swap(c.fy, c.fy2);
    c.grp_cur = 1 - c.grp_cur;
    F = Fn;
  }
  c.frontier = F;
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
