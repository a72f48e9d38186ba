// C ABI of libamfmm_hip.so: context, scratch arena, phase sequencing,
// timing and introspection.  Internal errors are C++ exceptions that never
// cross the ABI: every entry point turns them into an amfmm_status.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>

#include "internal.h"

struct amfmm_ctx {
  amfmm::Ctx c;
};

namespace amfmm {

static bool in_arena(const Ctx& c, const void* p) {
  return c.arena && (const char*)p >= c.arena && (const char*)p < c.arena + c.arena_cap;
}

constexpr size_t kArenaAlign = 256;

// give an arena block back, merged with free neighbours
static void arena_release(Ctx& c, size_t off, size_t bytes) {
  auto next = c.arena_free.lower_bound(off);
  if (next != c.arena_free.end() && off + bytes == next->first) {
    bytes += next->second;
    next = c.arena_free.erase(next);
  }
  if (next != c.arena_free.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += bytes;
      return;
    }
  }
  c.arena_free.emplace(off, bytes);
}

static void release(Ctx& c, DevBuf& b) {
  if (b.p) {
    if (in_arena(c, b.p)) {
      arena_release(c, (size_t)((char*)b.p - c.arena), b.cap);
    } else {
      (void)hipFree(b.p);
      c.bytes -= b.cap;
    }
    b.p = nullptr;
    b.cap = 0;
  }
}

// an arena block of `bytes` (a multiple of kArenaAlign): the first free block
// that holds it
static void* arena_alloc(Ctx& c, size_t bytes) {
  for (auto it = c.arena_free.begin(); it != c.arena_free.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t off = it->first, rest = it->second - bytes;
    c.arena_free.erase(it);
    if (rest) c.arena_free.emplace(off + bytes, rest);
    return c.arena + off;
  }
  size_t largest = 0, total = 0;
  for (const auto& f : c.arena_free) {
    largest = std::max(largest, f.second);
    total += f.second;
  }
  throw Error(AMFMM_E_OOM, "allocation-free solve: its scratch needs more than the " +
                               std::to_string(c.arena_cap >> 20) + " MiB static array (request of " +
                               std::to_string(bytes) + " bytes; " + std::to_string(total) + " bytes free, " +
                               "largest block " + std::to_string(largest) + ")");
}

static void* alloc(Ctx& c, size_t bytes) {
  if (c.arena) return arena_alloc(c, bytes);
  if (c.opt.max_bytes > 0 && (int64_t)(c.bytes + bytes) > c.opt.max_bytes)
    throw Error(AMFMM_E_OOM, "device scratch would exceed max_bytes (" + std::to_string(c.bytes + bytes) + " bytes)");
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(AMFMM_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  c.bytes += bytes;
  return p;
}

size_t free_device_bytes(Ctx& c) {
  if (c.arena) {
    size_t largest = 0;
    for (const auto& f : c.arena_free) largest = std::max(largest, f.second);
    return largest;
  }
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    fr = size_t(16) << 30;
  }
  return fr;
}

void* ensure(Ctx& c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return b.p;
  release(c, b);
  // headroom for regrowth, except in the arena (exact blocks: buffers sized
  // from the free space would otherwise outgrow it)
  size_t want = bytes + bytes / 4;
  if (c.arena) want = (bytes + kArenaAlign - 1) & ~(kArenaAlign - 1);
  b.p = alloc(c, want);
  b.cap = want;
  return b.p;
}

void* ensure_keep(Ctx& c, DevBuf& b, size_t bytes, size_t keep) {
  if (bytes == 0) bytes = 8;
  if (b.cap >= bytes) return b.p;
  size_t want = bytes + bytes / 4;
  if (c.arena) {
    want = (want + kArenaAlign - 1) & ~(kArenaAlign - 1);
    // an arena block followed by a large enough free block grows in place
    if (b.p && in_arena(c, b.p)) {
      const size_t end = (size_t)((char*)b.p - c.arena) + b.cap, more = want - b.cap;
      auto it = c.arena_free.find(end);
      if (it != c.arena_free.end() && it->second >= more) {
        const size_t rest = it->second - more;
        c.arena_free.erase(it);
        if (rest) c.arena_free.emplace(end + more, rest);
        b.cap = want;
        return b.p;
      }
    }
  }
  void* p = alloc(c, want);
  if (b.p && keep) AMFMM_HIP(hipMemcpyAsync(p, b.p, std::min(keep, b.cap), hipMemcpyDeviceToDevice, c.stream));
  if (b.p) {
    AMFMM_HIP(hipStreamSynchronize(c.stream));
    release(c, b);
  }
  b.p = p;
  b.cap = want;
  return b.p;
}

void sync(Ctx& c) { AMFMM_HIP(hipStreamSynchronize(c.stream)); }

static DevBuf* all_bufs(Ctx& c, int i) {
  DevBuf* v[] = {&c.pos4, &c.keys, &c.perm, &c.keys2, &c.perm2, &c.bbox, &c.scratch, &c.scratch2, &c.hist,
                 &c.c_begin, &c.c_count, &c.c_parent, &c.c_child0, &c.c_nchild, &c.leaves, &c.geo, &c.mom,
                 &c.msum, &c.loc, &c.far_start, &c.far_count, &c.far_src, &c.near_start, &c.near_count,
                 &c.near_src, &c.fx, &c.fy, &c.fx2, &c.fy2, &c.fcnt, &c.grp, &c.walkrec, &c.fsave, &c.gsave, &c.counters, &c.gqueue, &c.stage, &c.farrec, &c.gmin, &c.model, &c.mlp_tmp, &c.mlp_part,
                 &c.mlp_grad, &c.mono, &c.locg};
  const int nv = (int)(sizeof(v) / sizeof(v[0]));
  return i < nv ? v[i] : nullptr;
}

void mark(Ctx& c, int phase) {
  if (c.arena) return;  // the allocation-free solve creates no events
  if (c.ev_used == c.ev_pool.size()) {
    hipEvent_t e;
    AMFMM_HIP(hipEventCreate(&e));
    c.ev_pool.push_back(e);
    c.ev_phase.push_back(0);
  }
  AMFMM_HIP(hipEventRecord(c.ev_pool[c.ev_used], c.stream));
  c.ev_phase[c.ev_used] = phase;
  ++c.ev_used;
}

// Scratch of the allocation-free solve: one array in the library's code
// object, so every device the library runs on holds its own copy of it until
// the process ends.  Host code never passes the array's name to a kernel or a
// copy: it looks up each device's copy once (hipGetSymbolAddress with that
// device current, in amfmm_create) and uses that address.
constexpr size_t kNoAllocBytes = size_t(256) << 20;
constexpr int64_t kNoAllocMaxN = int64_t(1) << 18;
__device__ __align__(256) char scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static std::vector<char*> g_scratch_ptr;  // per device; nullptr until looked up

// The device address of the scratch array on `device`, which must be the
// current device: looked up on the first call for that device.
static char* device_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  if (!g_scratch_ptr[(size_t)device]) {
    char* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      throw Error(AMFMM_E_HIP, std::string("hipGetSymbolAddress of the allocation-free scratch failed: ") +
                                   hipGetErrorString(e));
    }
    g_scratch_ptr[(size_t)device] = ptr;
  }
  return g_scratch_ptr[(size_t)device];
}

}  // namespace amfmm

using amfmm::Ctx;
using amfmm::Error;

template <typename F>
static int guarded(amfmm_ctx* ctx, F&& f) {
  if (!ctx) return AMFMM_E_INVALID;
  try {
    return f(ctx->c);
  } catch (const Error& e) {
    ctx->c.last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->c.last_error = e.what();
    return AMFMM_E_HIP;
  }
}

template <typename T>
static std::vector<T> fetch(Ctx& c, const void* dev, size_t count) {
  std::vector<T> h(count);
  if (count) AMFMM_HIP(hipMemcpyAsync(h.data(), dev, sizeof(T) * count, hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
  return h;
}

static void build_near_pairs(Ctx& c);

namespace {

// Unordered near-field leaf pairs (x, o), x <= o, behind the near lists (the
// pairs amfmm_get_lists returns): one thread per target cell x, a walk over
// each entry's subtree by first child, next sibling and parent (no stack),
// summed per wave and added to *total.
__global__ void __launch_bounds__(256) k_count_near_pairs(int32_t nc, const int64_t* __restrict__ start,
                                                           const int32_t* __restrict__ count,
                                                           const int32_t* __restrict__ src,
                                                           const int32_t* __restrict__ ch0,
                                                           const int32_t* __restrict__ nch,
                                                           const int32_t* __restrict__ par,
                                                           unsigned long long* __restrict__ total) {
  const int32_t x = blockIdx.x * 256 + threadIdx.x;
  unsigned long long k = 0;
  if (x < nc) {
    for (int32_t j = 0; j < count[x]; ++j) {
      const int32_t y = src[start[x] + j];
      int32_t o = y;
      for (;;) {
        if (nch[o] > 0) {
          o = ch0[o];
          continue;
        }
        k += (x <= o) ? 1ull : 0ull;
        // next leaf: the next sibling of o or of its nearest ancestor below y
        while (o != y) {
          const int32_t p = par[o];
          if (o + 1 < ch0[p] + nch[p]) {
            ++o;
            break;
          }
          o = p;
        }
        if (o == y) break;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) k += __shfl_down(k, off, 64);
  if ((threadIdx.x & 63) == 0 && k) atomicAdd(total, k);
}

}  // namespace

// the number of pairs build_near_pairs would list, counted on the device
static int64_t count_near_pairs(Ctx& c) {
  if (c.near_pairs_valid) return (int64_t)c.near_pairs_host.size();
  unsigned long long* t = (unsigned long long*)amfmm::ensure(c, c.counters, 64) + 1;
  amfmm::zero_u64(c, t, 1);
  hipLaunchKernelGGL(k_count_near_pairs, dim3(amfmm::blocks_for(c.ncells, 256)), dim3(256), 0, c.stream,
                     c.ncells, (const int64_t*)c.near_start.p, (const int32_t*)c.near_count.p,
                     (const int32_t*)c.near_src.p, (const int32_t*)c.c_child0.p, (const int32_t*)c.c_nchild.p,
                     (const int32_t*)c.c_parent.p, t);
  AMFMM_HIP(hipGetLastError());
  unsigned long long h = 0;
  AMFMM_HIP(hipMemcpyAsync(&h, t, sizeof(h), hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
  return (int64_t)h;
}

static int fail(Ctx& c, int code, const char* msg) {
  c.last_error = msg;
  return code;
}

extern "C" {

int amfmm_default_options(amfmm_options* o) {
  if (!o) return AMFMM_E_INVALID;
  o->n_crit = 25;
  o->variant = AMFMM_TC;
  o->precision = AMFMM_FP64;
  o->criterion = AMFMM_GEOMETRIC;
  o->G = 1.0;
  o->error_tol = 1e-4;
  o->theta_max = 1.0;
  o->learned_min_work = 262144;
  o->max_bytes = 0;
  o->list_bytes = 0;
  o->softening = 0.0;
  o->order = 3;
  return AMFMM_OK;
}

static int check_options(const amfmm_options* o) {
  if (o->n_crit < 1 || o->n_crit > 4096) return AMFMM_E_INVALID;
  if (o->variant < AMFMM_UC || o->variant > AMFMM_TCO) return AMFMM_E_INVALID;
  if (o->precision != AMFMM_FP64 && o->precision != AMFMM_MIXED) return AMFMM_E_INVALID;
  if (o->criterion < AMFMM_GEOMETRIC || o->criterion > AMFMM_MULTIPOLE) return AMFMM_E_INVALID;
  if (!(o->G == o->G) || o->max_bytes < 0 || o->list_bytes < 0 || o->learned_min_work < 0) return AMFMM_E_INVALID;
  if (!(o->softening >= 0.0) || !std::isfinite(o->softening)) return AMFMM_E_INVALID;
  if (o->order != 3 && (o->order != 4 || o->variant == AMFMM_TCO))
    return AMFMM_E_INVALID;
  return AMFMM_OK;
}

int amfmm_create(const amfmm_options* opt, void* stream, amfmm_ctx** out) {
  if (!out) return AMFMM_E_INVALID;
  *out = nullptr;
  amfmm_options o;
  amfmm_default_options(&o);
  if (opt) o = *opt;
  if (check_options(&o) != AMFMM_OK) return AMFMM_E_INVALID;
  amfmm_ctx* ctx = new amfmm_ctx();
  ctx->c.opt = o;
  ctx->c.stream = (hipStream_t)stream;
  if (hipGetDevice(&ctx->c.device) != hipSuccess) {
    delete ctx;
    return AMFMM_E_HIP;
  }
  if (hipHostMalloc((void**)&ctx->c.pinned, 8 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return AMFMM_E_HIP;
  }
  try {
    (void)amfmm::device_scratch(ctx->c.device);  // the allocation-free solve's array on this device
  } catch (const Error&) {
    (void)hipHostFree(ctx->c.pinned);
    delete ctx;
    return AMFMM_E_HIP;
  }
  *out = ctx;
  return AMFMM_OK;
}

int amfmm_destroy(amfmm_ctx* ctx) {
  if (!ctx) return AMFMM_E_INVALID;
  Ctx& c = ctx->c;
  (void)hipStreamSynchronize(c.stream);
  for (int i = 0; amfmm::all_bufs(c, i); ++i) amfmm::release(c, *amfmm::all_bufs(c, i));
  for (auto& e : c.ev_pool) (void)hipEventDestroy(e);
  if (c.pinned) (void)hipHostFree(c.pinned);
  delete ctx;
  return AMFMM_OK;
}

int amfmm_set_field_estimate(amfmm_ctx* ctx, const double* gx, const double* gy, const double* gz) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if ((gy == nullptr) != (gz == nullptr)) return fail(c, AMFMM_E_INVALID, "give magnitudes or all three components");
    c.field = gx;
    c.field_y = gx ? gy : nullptr;
    c.field_z = gx ? gz : nullptr;
    return AMFMM_OK;
  });
}

int amfmm_set_model(amfmm_ctx* ctx, const float* model) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (!model) {
      amfmm::release(c, c.model);
      return AMFMM_OK;
    }
    for (int i = 0; i < AMFMM_MLP_MODEL; ++i)
      if (!std::isfinite(model[i]) && !(i >= 4817 && std::isinf(model[i])))
        return fail(c, AMFMM_E_NONFINITE, "model holds a NaN or an infinite weight");
    float* tmp = (float*)amfmm::ensure(c, c.mlp_tmp, sizeof(float) * AMFMM_MLP_MODEL);
    float* dst = (float*)amfmm::ensure(c, c.model, sizeof(float) * AMFMM_MLP_MODEL);
    AMFMM_HIP(hipMemcpyAsync(tmp, model, sizeof(float) * AMFMM_MLP_MODEL, hipMemcpyHostToDevice, c.stream));
    amfmm::round_model(c, tmp, dst);
    amfmm::sync(c);
    c.hint_n = 0;  // decisions change: forget the batch size of earlier solves
    return AMFMM_OK;
  });
}

int amfmm_pair_features(amfmm_ctx* ctx, int64_t np, const int32_t* pairs, float* feats) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (np < 0 || (np > 0 && (!pairs || !feats))) return fail(c, AMFMM_E_INVALID, "bad pair arguments");
    amfmm::compute_pair_features(c, np, pairs, feats);
    return AMFMM_OK;
  });
}

int amfmm_pair_labels(amfmm_ctx* ctx, int32_t variant, int64_t np, const int32_t* pairs, double* labels) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (np < 0 || (np > 0 && (!pairs || !labels))) return fail(c, AMFMM_E_INVALID, "bad pair arguments");
    if (variant < AMFMM_UC || variant > AMFMM_TCO) return fail(c, AMFMM_E_INVALID, "bad variant");
    amfmm::compute_pair_labels(c, variant, np, pairs, labels);
    return AMFMM_OK;
  });
}

int amfmm_mlp_predict(amfmm_ctx* ctx, int64_t n, const float* model, const float* feats, float* y) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (n < 0 || !model || (n > 0 && (!feats || !y))) return fail(c, AMFMM_E_INVALID, "bad arguments");
    amfmm::mlp_predict(c, n, model, feats, y);
    return AMFMM_OK;
  });
}

int amfmm_mlp_grad(amfmm_ctx* ctx, int64_t n, const float* model, const float* feats, const float* labels,
                   double tau, float* grad, double* loss) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (n < 1 || n >= (int64_t)INT32_MAX || !model || !feats || !labels || !grad)
      return fail(c, AMFMM_E_INVALID, "bad arguments");
    if (!(tau > 0.0 && tau < 1.0)) return fail(c, AMFMM_E_INVALID, "tau must lie in (0, 1)");
    const double l = amfmm::mlp_grad(c, n, model, feats, labels, tau, grad);
    if (loss) *loss = l;
    return AMFMM_OK;
  });
}

int amfmm_mlp_train(amfmm_ctx* ctx, int64_t n, const float* feats, const float* labels, float* model,
                    float* adam_m, float* adam_v, int64_t step0, int32_t steps, int32_t batch, double lr,
                    double tau, double* last_loss) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (n < 1 || n >= (int64_t)INT32_MAX || !feats || !labels || !model || !adam_m || !adam_v)
      return fail(c, AMFMM_E_INVALID, "bad arguments");
    if (step0 < 0 || steps < 0 || batch < 1 || batch > (1 << 20) || !(lr > 0.0))
      return fail(c, AMFMM_E_INVALID, "bad training schedule");
    if (!(tau > 0.0 && tau < 1.0)) return fail(c, AMFMM_E_INVALID, "tau must lie in (0, 1)");
    const double l = amfmm::mlp_train(c, n, feats, labels, model, adam_m, adam_v, step0, steps, batch, lr, tau);
    if (last_loss) *last_loss = l;
    return AMFMM_OK;
  });
}

int amfmm_set_stream(amfmm_ctx* ctx, void* stream) {
  return guarded(ctx, [&](Ctx& c) -> int {
    c.stream = (hipStream_t)stream;
    return AMFMM_OK;
  });
}

static int build_tree_impl(Ctx& c, int64_t n, const double* x, const double* y, const double* z,
                           const double* m) {
  if (n < 1 || n >= (int64_t)INT32_MAX) return fail(c, AMFMM_E_INVALID, "n must be in [1, 2^31)");
  if (!x || !y || !z || !m) return fail(c, AMFMM_E_INVALID, "null input pointer");
  c.have_tree = c.have_moments = c.have_lists = false;
  c.ev_used = 0;
  amfmm::mark(c, amfmm::kPhValidate);
  int st = amfmm::bbox_validate(c, x, y, z, m, n);
  if (st == AMFMM_E_NONFINITE) return fail(c, st, "non-finite position or mass");
  if (st != AMFMM_OK) return fail(c, st, "masses must be positive");
  amfmm::mark(c, amfmm::kPhSort);
  amfmm::build_keys_sort(c, x, y, z, m, n);
  amfmm::mark(c, amfmm::kPhTree);
  amfmm::build_levels(c);
  amfmm::mark(c, amfmm::kPhEnd);
  c.have_tree = true;
  return AMFMM_OK;
}

int amfmm_build_tree(amfmm_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                     const double* m) {
  return guarded(ctx, [&](Ctx& c) -> int { return build_tree_impl(c, n, x, y, z, m); });
}

static int moments_impl(Ctx& c) {
  if (!c.have_tree) return fail(c, AMFMM_E_STATE, "compute_moments needs build_tree");
  if (c.ev_used) --c.ev_used;  // continue the timeline of the tree build
  amfmm::mark(c, amfmm::kPhMoments);
  amfmm::upward_pass(c);
  if (c.opt.order != 3) amfmm::order_upward(c);
  amfmm::far_prepare(c);
  amfmm::mark(c, amfmm::kPhEnd);
  return AMFMM_OK;
}

int amfmm_compute_moments(amfmm_ctx* ctx) {
  return guarded(ctx, [&](Ctx& c) -> int { return moments_impl(c); });
}

static int walk_impl(Ctx& c, double theta) {
  if (!(theta > 0.0 && theta <= 1.0)) return fail(c, AMFMM_E_INVALID, "theta must lie in (0, 1]");
  if (!c.have_moments) return fail(c, AMFMM_E_STATE, "walk needs compute_moments");
  if (c.ev_used) --c.ev_used;
  amfmm::mark(c, amfmm::kPhWalk);
  amfmm::dual_walk(c, theta);
  c.near_pairs_valid = false;
  amfmm::mark(c, amfmm::kPhEnd);
  c.batched = false;
  c.far_evals = c.n_far;
  return AMFMM_OK;
}

int amfmm_walk(amfmm_ctx* ctx, double theta) {
  return guarded(ctx, [&](Ctx& c) -> int { return walk_impl(c, theta); });
}

// counters of an evaluation: near interactions (counters[0]) and launches
// (the walk's own are reset when a walk starts)
static void zero_counters(Ctx& c) {
  c.far_launches = c.near_launches = 0;
  void* p = amfmm::ensure(c, c.counters, 64);
  amfmm::zero_u64(c, (unsigned long long*)p, 1);
}

// far field, push-down and near field over all cells, from kept lists
static void evaluate_all(Ctx& c, double* ax, double* ay, double* az, double* pot) {
  using namespace amfmm;
  mark(c, kPhFar);
  far_field(c, 0, c.ncells);
  mark(c, kPhPush);
  for (int l = 1; l <= c.depth; ++l) push_down(c, c.level_start[l], c.level_start[l + 1]);
  mark(c, kPhNear);
  near_field(c, (const int32_t*)c.leaves.p, 0, c.nleaves, ax, ay, az, pot);
  mark(c, kPhEnd);
}

static int evaluate_impl(Ctx& c, double* ax, double* ay, double* az, double* pot) {
  if (!c.have_lists) return fail(c, AMFMM_E_STATE, "evaluate needs walk");
  if (!ax || !ay || !az) return fail(c, AMFMM_E_INVALID, "null output pointer");
  if (c.ev_used) --c.ev_used;
  zero_counters(c);
  evaluate_all(c, ax, ay, az, pot);
  return AMFMM_OK;
}

// Device bytes the lists and the walk frontier take per particle at this
// theta: measured on Plummer spheres (about 320 B at theta = 0.5), growing as
// theta^-3 like the number of interacting pairs.
static double list_bytes_per_particle(double theta) {
  const double r = 0.5 / theta;
  return 320.0 * r * r * r;
}

// List bytes a walk may take.  A list that grows is copied, so its old and
// new blocks coexist for a moment, and each block carries a quarter of
// headroom: lists within b bytes peak below 2.25 b.  Outside an arena the
// lists and the staging room this context already holds are reused by the
// next walk and count as free, and b is two fifths of that: the whole walk
// of a large problem fits in one pass when the device has the memory (one
// evaluation launch per phase instead of one per batch).  In an arena: a
// quarter of its largest free block.
static size_t list_budget(Ctx& c) {
  if (c.opt.list_bytes > 0) return (size_t)c.opt.list_bytes;
  size_t fr = amfmm::free_device_bytes(c);
  if (!c.arena) fr += c.far_src.cap + c.near_src.cap + c.fy.cap + c.fy2.cap + c.stage.cap;
  size_t b = c.arena ? fr / 4 : fr / 5 * 2;
  if (c.opt.max_bytes > 0) b = std::min<size_t>(b, (size_t)c.opt.max_bytes / 2);
  return c.arena ? b : std::max<size_t>(b, size_t(64) << 20);
}

// a device allocation that failed outside an arena: the walk that needed it
// can go batch by batch instead
static bool out_of_device_memory(const Ctx& c, const amfmm::Error& e) {
  return !c.arena && e.code == AMFMM_E_OOM && c.opt.max_bytes == 0;
}

// Walk and evaluation one batch of subtrees at a time, so that the lists of
// the whole tree never have to exist at once (small theta, large N).  The top
// levels are walked and evaluated for all cells; below the split level the
// cells are cut into contiguous batches of subtrees, each walked to the
// leaves, evaluated (far field, push-down, near field) and released.  The
// pairs are the same as those of the whole walk; the results agree up to
// rounding (how a level's frontier is cut into work chunks depends on its
// size, and with it the order in which a cell's pairs are listed and summed).
static void solve_batched(Ctx& c, double theta, double* ax, double* ay, double* az, double* pot) {
  using namespace amfmm;
  const double bpp = list_bytes_per_particle(theta);
  const double budget = (double)list_budget(c);
  const int64_t pmax = std::max<int64_t>(1, (int64_t)(budget / bpp));
  // particle ranges of all cells (host copy), to pick the split level and cut batches
  std::vector<int32_t> hb(c.ncells), hc(c.ncells);
  AMFMM_HIP(hipMemcpyAsync(hb.data(), c.c_begin.p, sizeof(int32_t) * c.ncells, hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipMemcpyAsync(hc.data(), c.c_count.p, sizeof(int32_t) * c.ncells, hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
  // split level: the first level with many cells none of which is too large a
  // share of the particles (dense cores make cells of one level very unequal)
  const int64_t cap = std::max<int64_t>(4096, c.n / 1024);
  int Ls = 1;
  for (; Ls < c.depth; ++Ls) {
    const int32_t a = c.level_start[Ls], b = c.level_start[Ls + 1];
    if (b - a < 4096) continue;
    int32_t big = 0;
    for (int32_t q = a; q < b; ++q) big = std::max(big, hc[q]);
    if (big <= cap) break;
  }
  c.walk_budget = 0;  // the top levels are walked whole
  mark(c, kPhWalk);
  walk_prepare(c, theta);
  walk_start(c);
  std::vector<int32_t> lo(c.level_start.begin(), c.level_start.end() - 1),
      hi(c.level_start.begin() + 1, c.level_start.end());
  int64_t fb = 0, nb = 0;
  walk_levels(c, 0, Ls - 1, lo, hi, fb, nb);
  c.far_evals = fb;
  mark(c, kPhFar);
  far_field(c, 0, c.level_start[Ls]);
  mark(c, kPhPush);
  for (int l = 1; l < Ls; ++l) push_down(c, c.level_start[l], c.level_start[l + 1]);
  mark(c, kPhNear);
  for (int l = 0; l < Ls; ++l) near_field(c, nullptr, lo[l], hi[l] - lo[l], ax, ay, az, pot);
  // keep the level-Ls frontier and its groups
  const int64_t FL = c.frontier;
  const int32_t nL = c.level_start[Ls + 1] - c.level_start[Ls];
  int64_t* gbeg;
  int32_t* gcnt;
  group_arrays(c, &gbeg, &gcnt);
  std::vector<int64_t> hbeg(nL);
  std::vector<int32_t> hcnt(nL);
  AMFMM_HIP(hipMemcpyAsync(hbeg.data(), gbeg, sizeof(int64_t) * nL, hipMemcpyDeviceToHost, c.stream));
  AMFMM_HIP(hipMemcpyAsync(hcnt.data(), gcnt, sizeof(int32_t) * nL, hipMemcpyDeviceToHost, c.stream));
  int32_t* fsave = (int32_t*)ensure(c, c.fsave, sizeof(int32_t) * (FL + 1));
  AMFMM_HIP(hipMemcpyAsync(fsave, c.fy.p, sizeof(int32_t) * FL, hipMemcpyDeviceToDevice, c.stream));
  AMFMM_HIP(hipStreamSynchronize(c.stream));
  const int32_t L0 = c.level_start[Ls];
  std::vector<int64_t> bbeg(nL);
  c.walk_budget = (size_t)budget;
  int32_t x0 = 0;
  // batch size in particles: the last solve's, never above 9/10 of a size
  // that has exceeded the budget for this problem
  auto capped = [&](int64_t v) {
    v = std::min(v, pmax);
    return c.batch_fail > 0 ? std::max<int64_t>(1, std::min(v, c.batch_fail - c.batch_fail / 10)) : v;
  };
  int64_t plim = capped(c.batch_hint > 0 ? c.batch_hint : pmax);
  while (x0 < nL) {
    int32_t x1 = x0;
    int64_t parts = 0;
    while (x1 < nL && (x1 == x0 || parts + hc[L0 + x1] <= plim)) parts += hc[L0 + x1++];
    // this batch's groups, relative to its first entry, and its entries
    const int64_t base = hbeg[x0];
    int64_t F = 0;
    for (int32_t i = x0; i < x1; ++i) {
      bbeg[i - x0] = hbeg[i] - base;
      F += hcnt[i];
    }
    mark(c, kPhWalk);
    group_arrays(c, &gbeg, &gcnt);
    AMFMM_HIP(hipMemcpyAsync(gbeg, bbeg.data(), sizeof(int64_t) * (x1 - x0), hipMemcpyHostToDevice, c.stream));
    AMFMM_HIP(hipMemcpyAsync(gcnt, hcnt.data() + x0, sizeof(int32_t) * (x1 - x0), hipMemcpyHostToDevice, c.stream));
    int32_t* fy = (int32_t*)ensure(c, c.fy, sizeof(int32_t) * (F + 1));
    AMFMM_HIP(hipMemcpyAsync(fy, fsave + base, sizeof(int32_t) * F, hipMemcpyDeviceToDevice, c.stream));
    c.frontier = F;
    // the batch's cells on each level: those whose particles lie in its range
    const int32_t pb = hb[L0 + x0], pe = hb[L0 + x1 - 1] + hc[L0 + x1 - 1];
    std::vector<int32_t> blo(lo), bhi(hi);
    for (int l = Ls; l <= c.depth; ++l) {
      const int32_t* first = hb.data() + c.level_start[l];
      const int32_t* last = hb.data() + c.level_start[l + 1];
      blo[l] = (int32_t)(std::lower_bound(first, last, pb) - hb.data());
      bhi[l] = (int32_t)(std::lower_bound(first, last, pe) - hb.data());
    }
    int64_t bfb = 0, bnb = 0;
    bool over = false;
    try {
      walk_levels(c, Ls, c.depth, blo, bhi, bfb, bnb);
    } catch (const BudgetExceeded&) {
      over = true;
    } catch (const Error& e) {
      if (!out_of_device_memory(c, e)) throw;
      over = true;
    }
    if (over) {
      // too many pairs for one batch (or for the device): halve it (a single
      // cell that does not fit is reported as out of memory)
      if (x1 - x0 == 1) throw Error(AMFMM_E_OOM, "one subtree's interaction lists exceed the list budget");
      c.batch_fail = c.batch_fail > 0 ? std::min(c.batch_fail, parts) : parts;
      plim = std::max<int64_t>(1, parts / 2);
      continue;
    }
    c.batch_hint = plim;
    plim = capped(plim + plim / 4);
    c.far_evals += bfb;
    mark(c, kPhFar);
    for (int l = Ls; l <= c.depth; ++l) far_field(c, blo[l], bhi[l]);
    mark(c, kPhPush);
    for (int l = Ls; l <= c.depth; ++l) push_down(c, blo[l], bhi[l]);
    mark(c, kPhNear);
    for (int l = Ls; l <= c.depth; ++l) near_field(c, nullptr, blo[l], bhi[l] - blo[l], ax, ay, az, pot);
    x0 = x1;
  }
  mark(c, kPhEnd);
  c.have_lists = false;  // lists of the last batch only: not kept
  c.batched = true;
}

int amfmm_evaluate(amfmm_ctx* ctx, double* ax, double* ay, double* az, double* pot) {
  return guarded(ctx, [&](Ctx& c) -> int { return evaluate_impl(c, ax, ay, az, pot); });
}

static int solve_impl(Ctx& c, int64_t n, const double* x, const double* y, const double* z, const double* m,
                      double theta, double* ax, double* ay, double* az, double* pot) {
  {
    if (!(theta > 0.0 && theta <= 1.0)) return fail(c, AMFMM_E_INVALID, "theta must lie in (0, 1]");
    if (!ax || !ay || !az) return fail(c, AMFMM_E_INVALID, "null output pointer");
    int st = build_tree_impl(c, n, x, y, z, m);
    if (st) return st;
    if ((st = moments_impl(c))) return st;
    if (c.ev_used) --c.ev_used;
    zero_counters(c);
    const double need = list_bytes_per_particle(theta) * (double)n;
    const size_t budget = list_budget(c);
    // a context that needed batches for this size and criterion goes straight to them
    const bool same = c.hint_n == n && c.hint_theta == theta && c.hint_mode == c.opt.criterion &&
                      c.hint_tol == c.opt.error_tol;
    if (!same) c.batch_hint = c.batch_fail = 0;
    bool whole = (need <= (double)budget || c.depth < 3) && !(same && c.batch_hint > 0);
    if (whole) {
      amfmm::mark(c, amfmm::kPhWalk);
      c.walk_budget = c.depth < 3 ? 0 : budget;
      try {
        amfmm::dual_walk(c, theta);
      } catch (const amfmm::BudgetExceeded&) {
        whole = false;  // the estimate was too low: walk batch by batch
      } catch (const amfmm::Error& e) {
        if (!out_of_device_memory(c, e)) throw;
        // the lists did not fit the device after all: give back what the
        // walk grew and go batch by batch, at most half the particles a batch
        release(c, c.far_src);
        release(c, c.near_src);
        release(c, c.stage);
        c.batch_fail = std::max<int64_t>(1, n / 2);
        whole = false;
      }
      c.walk_budget = 0;
    }
    if (whole) {
      c.near_pairs_valid = false;
      c.batched = false;
      c.far_evals = c.n_far;
      evaluate_all(c, ax, ay, az, pot);
    } else {
      solve_batched(c, theta, ax, ay, az, pot);
      c.walk_budget = 0;
    }
    c.hint_n = n;
    c.hint_theta = theta;
    c.hint_mode = c.opt.criterion;
    c.hint_tol = c.opt.error_tol;
    return AMFMM_OK;
  }
}

int amfmm_solve_gravity(amfmm_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                        const double* m, double theta, double* ax, double* ay, double* az, double* pot) {
  return guarded(ctx, [&](Ctx& c) -> int { return solve_impl(c, n, x, y, z, m, theta, ax, ay, az, pot); });
}

int amfmm_leapfrog(amfmm_ctx* ctx, int64_t n, double* x, double* y, double* z, double* vx, double* vy, double* vz,
                   const double* m, double theta, double dt, int32_t steps, double* ax, double* ay, double* az) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (!vx || !vy || !vz || !ax || !ay || !az) return fail(c, AMFMM_E_INVALID, "null pointer");
    if (steps < 0 || !std::isfinite(dt)) return fail(c, AMFMM_E_INVALID, "bad steps or dt");
    if (!(theta > 0.0 && theta <= 1.0)) return fail(c, AMFMM_E_INVALID, "theta must lie in (0, 1]");
    if (n < 1 || n >= (int64_t)INT32_MAX) return fail(c, AMFMM_E_INVALID, "n must be in [1, 2^31)");
    for (int32_t s = 0; s < steps; ++s) {
      amfmm::kick(c, n, 0.5 * dt, ax, ay, az, vx, vy, vz);
      amfmm::drift(c, n, dt, vx, vy, vz, x, y, z);
      const int st = solve_impl(c, n, x, y, z, m, theta, ax, ay, az, nullptr);
      if (st) return st;
      amfmm::kick(c, n, 0.5 * dt, ax, ay, az, vx, vy, vz);
    }
    return AMFMM_OK;
  });
}

// The solve with every device buffer carved from this device's scratch array.
// The context's own buffers, batch hints and timing are set aside for the
// call and restored after it (so its tree, lists and phase times are not
// kept: introspection calls see no tree afterwards); the learned model stays
// in place (read only).
int amfmm_solve_gravity_noalloc(amfmm_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                                const double* m, double theta, double* ax, double* ay, double* az, double* pot) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (n > amfmm::kNoAllocMaxN)
      return fail(c, AMFMM_E_INVALID, "allocation-free solve: n exceeds its maximum of 2^18 particles");
    if (c.arena) return fail(c, AMFMM_E_STATE, "allocation-free solve already running on this context");
    if (c.opt.order != 3) return fail(c, AMFMM_E_INVALID, "allocation-free solve: expansion order 3 only");
    struct Saved {
      Ctx& c;
      std::vector<amfmm::DevBuf> bufs;
      int64_t batch_hint, hint_n, batch_fail;
      double hint_theta, hint_tol;
      int hint_mode;
      explicit Saved(Ctx& cc)
          : c(cc), batch_hint(cc.batch_hint), hint_n(cc.hint_n), batch_fail(cc.batch_fail),
            hint_theta(cc.hint_theta), hint_tol(cc.hint_tol), hint_mode(cc.hint_mode) {
        for (int i = 0; amfmm::DevBuf* b = amfmm::all_bufs(c, i); ++i) {
          bufs.push_back(*b);
          if (b != &c.model) *b = amfmm::DevBuf{};
        }
        c.hint_n = 0;
      }
      ~Saved() {
        for (int i = 0; amfmm::DevBuf* b = amfmm::all_bufs(c, i); ++i) *b = bufs[(size_t)i];
        c.arena = nullptr;
        c.arena_cap = 0;
        c.arena_free.clear();
        c.have_tree = c.have_moments = c.have_lists = false;
        c.near_pairs_valid = false;
        c.batch_hint = batch_hint;
        c.hint_n = hint_n;
        c.batch_fail = batch_fail;
        c.hint_theta = hint_theta;
        c.hint_tol = hint_tol;
        c.hint_mode = hint_mode;
      }
    } saved(c);
    c.arena = amfmm::device_scratch(c.device);
    c.arena_cap = amfmm::kNoAllocBytes;
    c.arena_free.clear();
    c.arena_free.emplace(0, amfmm::kNoAllocBytes);
    c.ev_used = 0;
    return solve_impl(c, n, x, y, z, m, theta, ax, ay, az, pot);
  });
}

int amfmm_direct(amfmm_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                 const double* m, int64_t ntarget, const int64_t* targets, double* ax, double* ay,
                 double* az, double* pot, double* gabs) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (n < 1 || ntarget < 0) return fail(c, AMFMM_E_INVALID, "bad sizes");
    if (!x || !y || !z || !m || !ax || !ay || !az) return fail(c, AMFMM_E_INVALID, "null pointer");
    if (!targets && ntarget > n) return fail(c, AMFMM_E_INVALID, "ntarget > n without target indices");
    amfmm::direct_sum(c, n, x, y, z, m, ntarget, targets, ax, ay, az, pot, gabs);
    return AMFMM_OK;
  });
}

int amfmm_balance(amfmm_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                  const double* m, const double* ax, const double* ay, const double* az, double* out) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (n < 1 || !out) return fail(c, AMFMM_E_INVALID, "bad arguments");
    if (!x || !y || !z || !m || !ax || !ay || !az) return fail(c, AMFMM_E_INVALID, "null pointer");
    amfmm::balance(c, n, x, y, z, m, ax, ay, az, out);
    return AMFMM_OK;
  });
}

int amfmm_get_counts(amfmm_ctx* ctx, int64_t* counts) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (!counts) return fail(c, AMFMM_E_INVALID, "null pointer");
    counts[0] = c.have_tree ? c.ncells : 0;
    counts[1] = c.have_tree ? c.depth : 0;
    counts[2] = c.have_lists ? c.n_far / 2 : c.far_evals / 2;
    counts[3] = 0;
    if (c.have_lists) counts[3] = count_near_pairs(c);
    counts[4] = c.have_tree ? c.nleaves : 0;
    counts[5] = c.have_tree ? c.n : 0;
    counts[6] = 0;
    counts[7] = c.far_evals;
    counts[8] = c.far_launches;
    counts[9] = c.near_launches;
    counts[10] = c.walk_candidates;
    counts[11] = c.pass_launches;
    if (c.counters.p) {
      unsigned long long h = 0;
      AMFMM_HIP(hipMemcpyAsync(&h, c.counters.p, sizeof(h), hipMemcpyDeviceToHost, c.stream));
      AMFMM_HIP(hipStreamSynchronize(c.stream));
      counts[6] = (int64_t)h;
    }
    return AMFMM_OK;
  });
}

int amfmm_get_tree(amfmm_ctx* ctx, uint64_t* keys, int64_t* perm, int32_t* level, int64_t* begin,
                   int64_t* count, int32_t* parent, int32_t* child0, int32_t* nchild) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (!c.have_tree) return fail(c, AMFMM_E_STATE, "no tree");
    const size_t n = (size_t)c.n, nc = (size_t)c.ncells;
    if (keys) {
      auto k = fetch<uint64_t>(c, c.keys.p, n);
      std::memcpy(keys, k.data(), n * sizeof(uint64_t));
    }
    if (perm) {
      auto p = fetch<int32_t>(c, c.perm.p, n);
      for (size_t i = 0; i < n; ++i) perm[i] = p[i];
    }
    if (level)
      for (size_t l = 0; l + 1 < c.level_start.size(); ++l)
        for (int32_t q = c.level_start[l]; q < c.level_start[l + 1]; ++q) level[q] = (int32_t)l;
    auto cp = [&](const amfmm::DevBuf& b, auto* dst) {
      if (!dst) return;
      auto v = fetch<int32_t>(c, b.p, nc);
      for (size_t i = 0; i < nc; ++i) dst[i] = v[i];
    };
    cp(c.c_begin, begin);
    cp(c.c_count, count);
    cp(c.c_parent, parent);
    cp(c.c_child0, child0);
    cp(c.c_nchild, nchild);
    return AMFMM_OK;
  });
}

int amfmm_get_moments(amfmm_ctx* ctx, double* out21) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (!c.have_moments) return fail(c, AMFMM_E_STATE, "no moments");
    if (!out21) return fail(c, AMFMM_E_INVALID, "null pointer");
    const size_t nc = (size_t)c.ncells;
    auto g = fetch<double>(c, c.geo.p, 4 * nc);
    auto m = fetch<double>(c, c.mom.p, amfmm::kMom * nc);
    for (size_t i = 0; i < nc; ++i) {
      double* o = out21 + 21 * i;
      o[0] = m[amfmm::kMom * i];
      o[1] = g[4 * i];
      o[2] = g[4 * i + 1];
      o[3] = g[4 * i + 2];
      o[4] = g[4 * i + 3];
      for (int q = 0; q < 16; ++q) o[5 + q] = m[amfmm::kMom * i + 1 + q];
    }
    return AMFMM_OK;
  });
}

// Unordered leaf pairs of the near field.  A near entry X <- Y with a split
// cell Y stands for every leaf under Y; each directed entry contributes the
// pairs whose first cell has the lower index, so every pair appears once.
static void build_near_pairs(Ctx& c) {
  if (c.near_pairs_valid) return;
  const size_t nc = (size_t)c.ncells;
  auto s = fetch<int64_t>(c, c.near_start.p, nc);
  auto k = fetch<int32_t>(c, c.near_count.p, nc);
  auto y = fetch<int32_t>(c, c.near_src.p, (size_t)c.n_near);
  auto ch0 = fetch<int32_t>(c, c.c_child0.p, nc);
  auto nch = fetch<int32_t>(c, c.c_nchild.p, nc);
  std::vector<std::pair<int32_t, int32_t>> v;
  std::vector<int32_t> stack;
  for (size_t x = 0; x < nc; ++x)
    for (int32_t j = 0; j < k[x]; ++j) {
      stack.assign(1, y[(size_t)s[x] + j]);
      while (!stack.empty()) {
        int32_t o = stack.back();
        stack.pop_back();
        if (nch[o]) {
          for (int32_t q = ch0[o] + nch[o] - 1; q >= ch0[o]; --q) stack.push_back(q);
          continue;
        }
        if ((int32_t)x <= o) v.emplace_back((int32_t)x, o);
      }
    }
  std::sort(v.begin(), v.end());
  c.near_pairs_host.swap(v);
  c.near_pairs_valid = true;
}

int amfmm_get_lists(amfmm_ctx* ctx, int32_t* far_ab, int32_t* near_ab) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (!c.have_lists) return fail(c, AMFMM_E_STATE, "no lists");
    const size_t nc = (size_t)c.ncells;
    std::vector<std::pair<int32_t, int32_t>> v;
    if (far_ab) {
      auto s = fetch<int64_t>(c, c.far_start.p, nc);
      auto k = fetch<int32_t>(c, c.far_count.p, nc);
      auto y = fetch<int32_t>(c, c.far_src.p, (size_t)c.n_far);
      for (size_t x = 0; x < nc; ++x)
        for (int32_t j = 0; j < k[x]; ++j) {
          int32_t o = y[(size_t)s[x] + j];
          if ((int32_t)x < o) v.emplace_back((int32_t)x, o);
        }
      std::sort(v.begin(), v.end());
    }
    if (near_ab) {
      const int64_t want = count_near_pairs(c);  // what amfmm_get_counts reported
      build_near_pairs(c);
      if ((int64_t)c.near_pairs_host.size() != want)
        return fail(c, AMFMM_E_STATE, "near pair count disagrees with the lists");
    }
    // the caller sized the arrays from amfmm_get_counts: check before writing
    if (far_ab && (int64_t)v.size() != c.n_far / 2) return fail(c, AMFMM_E_STATE, "far lists are not symmetric");
    for (size_t i = 0; far_ab && i < v.size(); ++i) {
      far_ab[2 * i] = v[i].first;
      far_ab[2 * i + 1] = v[i].second;
    }
    if (near_ab) {
      const auto& w = c.near_pairs_host;
      for (size_t i = 0; i < w.size(); ++i) {
        near_ab[2 * i] = w[i].first;
        near_ab[2 * i + 1] = w[i].second;
      }
    }
    return AMFMM_OK;
  });
}

int amfmm_get_phase_times(amfmm_ctx* ctx, double* ms, int32_t cap) {
  return guarded(ctx, [&](Ctx& c) -> int {
    if (!ms || cap < 0) return fail(c, AMFMM_E_INVALID, "bad arguments");
    AMFMM_HIP(hipStreamSynchronize(c.stream));
    double t[amfmm::kPhEnd + 1] = {};
    for (size_t i = 0; i + 1 < c.ev_used; ++i) {
      float v = 0.f;
      if (hipEventElapsedTime(&v, c.ev_pool[i], c.ev_pool[i + 1]) != hipSuccess) {
        (void)hipGetLastError();
        v = 0.f;
      }
      const int ph = c.ev_phase[i];
      if (ph >= 0 && ph < amfmm::kPhEnd) t[ph] += v;
    }
    // [0..7] phases (the walk including its pass), [8] total, [9] walk pass
    const double pass = t[amfmm::kPhWalkPass];
    t[amfmm::kPhWalk] += pass;
    double out[10];
    for (int i = 0; i < 8; ++i) out[i] = t[i];
    out[8] = 0.0;
    for (int i = 0; i < 8; ++i) out[8] += t[i];
    out[9] = pass;
    int k = std::min<int32_t>(cap, 10);
    for (int i = 0; i < k; ++i) ms[i] = out[i];
    return k;
  });
}

const char* amfmm_status_string(int status) {
  switch (status) {
    case AMFMM_OK: return "ok";
    case AMFMM_E_INVALID: return "invalid argument";
    case AMFMM_E_NONFINITE: return "non-finite input";
    case AMFMM_E_OOM: return "out of device memory";
    case AMFMM_E_HIP: return "HIP runtime error";
    case AMFMM_E_STATE: return "call order violated";
    default: return "unknown status";
  }
}

const char* amfmm_last_error(amfmm_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->c.last_error.c_str();
}

}  // extern "C"
