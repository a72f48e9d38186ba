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
#include "internal.h"

namespace amfmm {
namespace {

constexpr int kBS = 256;

enum : int { kAccept = 0, kNear = 1, kSplitX = 2, kSplitY = 3 };

struct TreeView {
  const double4* geo;
  const int32_t* ch0;
  const int32_t* nch;
  const int32_t* par;
  double theta;
};

__device__ inline int decide(const TreeView& t, int32_t X, int32_t Y) {
  const double4 a = t.geo[X], b = t.geo[Y];
  const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  const double d = sqrt((dx * dx + dy * dy) + dz * dz);
  const double rhs = (a.w + b.w) / t.theta;
  if (d > 0.0 && d >= rhs) return kAccept;
  const bool lx = t.nch[X] == 0, ly = t.nch[Y] == 0;
  if (lx && ly) return kNear;
  if (lx) return kSplitY;
  if (ly) return kSplitX;
  if (a.w > b.w) return kSplitX;
  if (a.w < b.w) return kSplitY;
  return X < Y ? kSplitX : kSplitY;
}

// Visits the terminal pairs of entry (X, Y) in depth-first order (children of
// Y in octant order) and calls f(kind, Y') for each.
template <typename F>
__device__ inline void traverse(const TreeView& t, int32_t X, int32_t Y, F&& f) {
  if (X == Y) {
    if (t.nch[X] == 0) {
      f(kNear, X);
    } else {
      const int32_t c0 = t.ch0[X], k = t.nch[X];
      for (int32_t j = 0; j < k; ++j) f(kSplitX, c0 + j);
    }
    return;
  }
  int32_t cur = Y;
  for (;;) {
    int d = decide(t, X, cur);
    if (d == kSplitY) {
      cur = t.ch0[cur];
      continue;
    }
    f(d, cur);
    for (;;) {
      if (cur == Y) return;
      int32_t p = t.par[cur];
      if (cur + 1 < t.ch0[p] + t.nch[p]) {
        ++cur;
        break;
      }
      cur = p;
    }
  }
}

__global__ void __launch_bounds__(kBS) k_walk_count(TreeView t, const int32_t* __restrict__ fx,
                                                    const int32_t* __restrict__ fy, int64_t F,
                                                    int64_t* __restrict__ cm, int64_t* __restrict__ cp,
                                                    int64_t* __restrict__ cq, int32_t c0,
                                                    int32_t* __restrict__ gbeg, int32_t* __restrict__ gend) {
  int64_t e = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (e >= F) return;
  const int32_t X = fx[e];
  int32_t m = 0, p = 0, q = 0;
  traverse(t, X, fy[e], [&](int d, int32_t) {
    m += d == kAccept;
    p += d == kNear;
    q += d == kSplitX;
  });
  cm[e] = m;
  cp[e] = p;
  cq[e] = q;
  if (e == 0 || fx[e - 1] != X) gbeg[X - c0] = (int32_t)e;
  if (e == F - 1 || fx[e + 1] != X) gend[X - c0] = (int32_t)(e + 1);
}

// per cell of the level: list extents, and the size of its children's entries
__global__ void __launch_bounds__(kBS) k_walk_cells(int32_t c0, int32_t nl, const int32_t* __restrict__ gbeg,
                                                    const int32_t* __restrict__ gend, const int64_t* __restrict__ sm,
                                                    const int64_t* __restrict__ sp, const int64_t* __restrict__ sq,
                                                    const int32_t* __restrict__ nch, int64_t far_base,
                                                    int64_t near_base, int64_t* __restrict__ far_start,
                                                    int32_t* __restrict__ far_count,
                                                    int64_t* __restrict__ near_start,
                                                    int32_t* __restrict__ near_count, int64_t* __restrict__ gq0,
                                                    int64_t* __restrict__ gS, int64_t* __restrict__ nsize) {
  int32_t i = blockIdx.x * kBS + threadIdx.x;
  if (i >= nl) return;
  const int32_t X = c0 + i;
  const int32_t b = gbeg[i], e = gend[i];
  far_start[X] = far_base + sm[b];
  far_count[X] = (int32_t)(sm[e] - sm[b]);
  near_start[X] = near_base + sp[b];
  near_count[X] = (int32_t)(sp[e] - sp[b]);
  const int64_t S = sq[e] - sq[b];
  gq0[i] = sq[b];
  gS[i] = S;
  nsize[i] = nch[X] * S;
}

__global__ void __launch_bounds__(kBS) k_walk_emit(TreeView t, const int32_t* __restrict__ fx,
                                                   const int32_t* __restrict__ fy, int64_t F, int32_t c0,
                                                   const int64_t* __restrict__ sm, const int64_t* __restrict__ sp,
                                                   const int64_t* __restrict__ sq, const int64_t* __restrict__ gq0,
                                                   const int64_t* __restrict__ gS, const int64_t* __restrict__ nbase,
                                                   int32_t* __restrict__ far_src, int64_t far_base,
                                                   int32_t* __restrict__ near_src, int64_t near_base,
                                                   int32_t* __restrict__ nx, int32_t* __restrict__ ny) {
  int64_t e = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (e >= F) return;
  const int32_t X = fx[e];
  const int32_t i = X - c0;
  int64_t fo = far_base + sm[e];
  int64_t no = near_base + sp[e];
  int64_t B = sq[e] - gq0[i];  // rank of the next base inside X's group
  const int64_t S = gS[i], nb = nbase[i];
  const int32_t k = t.nch[X], first = t.ch0[X];
  traverse(t, X, fy[e], [&](int d, int32_t Y) {
    if (d == kAccept) {
      far_src[fo++] = Y;
    } else if (d == kNear) {
      near_src[no++] = Y;
    } else {
      for (int32_t r = 0; r < k; ++r) {
        int64_t pos = nb + r * S + B;
        nx[pos] = first + r;
        ny[pos] = Y;
      }
      ++B;
    }
  });
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_walk_init(int32_t* fx, int32_t* fy) {
  fx[0] = 0;
  fy[0] = 0;
}

__global__ void k_gather_totals(const int64_t* sm, const int64_t* sp, const int64_t* ns, int64_t F, int32_t nl,
                                int64_t* out) {
  out[0] = sm[F];
  out[1] = sp[F];
  out[2] = ns[nl];
}

}  // namespace

void dual_walk(Ctx& c, double theta) {
  const int32_t nc = c.ncells;
  TreeView t{(const double4*)c.geo.p, as<int32_t>(c.c_child0), as<int32_t>(c.c_nchild), as<int32_t>(c.c_parent),
             theta};
  int64_t* far_start = (int64_t*)ensure(c, c.far_start, sizeof(int64_t) * nc);
  int32_t* far_count = (int32_t*)ensure(c, c.far_count, sizeof(int32_t) * nc);
  int64_t* near_start = (int64_t*)ensure(c, c.near_start, sizeof(int64_t) * nc);
  int32_t* near_count = (int32_t*)ensure(c, c.near_count, sizeof(int32_t) * nc);
  int64_t F = 1;
  ensure(c, c.fx, sizeof(int32_t) * 16);
  ensure(c, c.fy, sizeof(int32_t) * 16);
  hipLaunchKernelGGL(k_walk_init, dim3(1), dim3(1), 0, c.stream, as<int32_t>(c.fx), as<int32_t>(c.fy));
  AMFMM_HIP(hipGetLastError());
  int64_t far_base = 0, near_base = 0;
  int64_t* tot_host = nullptr;
  AMFMM_HIP(hipHostMalloc((void**)&tot_host, sizeof(int64_t) * 4, hipHostMallocDefault));
  try {
    for (int lev = 0; lev <= c.depth && F > 0; ++lev) {
      const int32_t c0 = c.level_start[lev], nl = c.level_start[lev + 1] - c0;
      if (F >= (int64_t)INT32_MAX) throw Error(AMFMM_E_OOM, "walk frontier exceeds 2^31 entries");
      // per-entry counts and their scans (n+1 each), per-cell group data
      const size_t E = (size_t)F + 1, L = (size_t)nl + 1;
      int64_t* w = (int64_t*)ensure(c, c.fcnt, sizeof(int64_t) * (6 * E + 5 * L + 4));
      int64_t *cm = w, *cp = cm + E, *cq = cp + E, *sm = cq + E, *sp = sm + E, *sq = sp + E;
      int64_t *gq0 = sq + E, *gS = gq0 + L, *nsize = gS + L, *nbase = nsize + L, *tot = nbase + L;
      int32_t* gbeg = (int32_t*)ensure(c, c.grp, sizeof(int32_t) * 2 * L);
      int32_t* gend = gbeg + L;
      const int32_t* fx = as<int32_t>(c.fx);
      const int32_t* fy = as<int32_t>(c.fy);
      hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(2 * L, kBS)), dim3(kBS), 0, c.stream, gbeg, (int64_t)(2 * L), 0);
      hipLaunchKernelGGL(k_walk_count, dim3(blocks_for(F, kBS)), dim3(kBS), 0, c.stream, t, fx, fy, F, cm, cp, cq,
                         c0, gbeg, gend);
      AMFMM_HIP(hipGetLastError());
      scan_i64(c, cm, sm, F);
      scan_i64(c, cp, sp, F);
      scan_i64(c, cq, sq, F);
      hipLaunchKernelGGL(k_walk_cells, dim3(blocks_for(nl, kBS)), dim3(kBS), 0, c.stream, c0, nl,
                         (const int32_t*)gbeg, (const int32_t*)gend, (const int64_t*)sm, (const int64_t*)sp,
                         (const int64_t*)sq, as<int32_t>(c.c_nchild), far_base, near_base, far_start, far_count,
                         near_start, near_count, gq0, gS, nsize);
      AMFMM_HIP(hipGetLastError());
      scan_i64(c, nsize, nbase, nl);
      hipLaunchKernelGGL(k_gather_totals, dim3(1), dim3(1), 0, c.stream, (const int64_t*)sm, (const int64_t*)sp,
                         (const int64_t*)nbase, F, nl, tot);
      AMFMM_HIP(hipGetLastError());
      AMFMM_HIP(hipMemcpyAsync(tot_host, tot, sizeof(int64_t) * 3, hipMemcpyDeviceToHost, c.stream));
      AMFMM_HIP(hipStreamSynchronize(c.stream));
      const int64_t mt = tot_host[0], pt = tot_host[1], Fn = tot_host[2];
      int32_t* far_src = (int32_t*)ensure_keep(c, c.far_src, sizeof(int32_t) * (far_base + mt + 1),
                                               sizeof(int32_t) * far_base);
      int32_t* near_src = (int32_t*)ensure_keep(c, c.near_src, sizeof(int32_t) * (near_base + pt + 1),
                                                sizeof(int32_t) * near_base);
      int32_t* nx = (int32_t*)ensure(c, c.fx2, sizeof(int32_t) * (Fn + 1));
      int32_t* ny = (int32_t*)ensure(c, c.fy2, sizeof(int32_t) * (Fn + 1));
      hipLaunchKernelGGL(k_walk_emit, dim3(blocks_for(F, kBS)), dim3(kBS), 0, c.stream, t, fx, fy, F, c0,
                         (const int64_t*)sm, (const int64_t*)sp, (const int64_t*)sq, (const int64_t*)gq0,
                         (const int64_t*)gS, (const int64_t*)nbase, far_src, far_base, near_src, near_base, nx, ny);
      AMFMM_HIP(hipGetLastError());
      far_base += mt;
      near_base += pt;
      std::swap(c.fx, c.fx2);
      std::swap(c.fy, c.fy2);
      F = Fn;
    }
  } catch (...) {
    (void)hipHostFree(tot_host);
    throw;
  }
  AMFMM_HIP(hipHostFree(tot_host));
  c.n_far = far_base;
  c.n_near = near_base;
  c.theta = theta;
  c.have_lists = true;
}

}  // namespace amfmm
