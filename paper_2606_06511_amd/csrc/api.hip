// C ABI of libttie.so: context, workspace carve-up, argument checks, status handling.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace ttie {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of ttie_eval_static, for callers that cannot allocate: a file-scope device array
// that every GPU the library runs on holds (its own copy) until the process ends.  In host code
// its name is not a device address: ttie_create looks the address up once per device, and the
// calls use only that.
static __device__ __align__(256) unsigned char scratch[TTIE_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices];

// With `device` current: its copy's address, looked up on the first call for the device.
static hipError_t scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = p;
  return hipSuccess;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

constexpr int64_t kMaxBuckets = (int64_t)1 << kMortonBucketBits;  // buckets of the broad-phase sort

// one scan scratch serves every scan: the vertex-sized ones and the bucket counts
static int64_t scan_len(const ttie_limits& lim) { return std::max<int64_t>(lim.max_verts, kMaxBuckets) + 1; }

// eval_only: only the regions the evaluation uses get space (the others are empty)
static Layout layout_with(const ttie_limits& lim, size_t scan_bytes, bool eval_only = false) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  auto take_other = [&](size_t bytes) { return take(eval_only ? 0 : bytes); };
  const size_t H = (size_t)lim.max_hits, V = (size_t)lim.max_verts + 1, T = (size_t)std::max<int64_t>(lim.max_tris, 1);
  // bitmap words over the vertices [0, max_verts] (one bit each), plus one
  const size_t W = (size_t)lim.max_verts / 32 + 2;
  L.counters = take(sizeof(Counters));
  L.hits = take(H * sizeof(HitGeom));
  L.defer = take((size_t)lim.max_pairs * 4);
  L.full = take((size_t)lim.max_pairs * 4);  // candidates for the full screening
  L.fsig = take((size_t)lim.max_pairs * 2);  // and their plane sides
  L.nfull = take((size_t)65536 * 4 * 4);     // their number per screening unit (a wave of <= 65536 blocks, or a tile)
  L.recs = take(H * sizeof(AsmRec<double>));
  L.cnt = take(32 * W * 4);  // read a whole bitmap word's 32 counts at a time
  L.cur = take_other(V * 4);
  L.off = take_other(V * 4);  // incidence ranges per vertex (the solvers fill them)
  L.ncol = take(V * 4);
  L.inc = take(6 * H * sizeof(Incidence));
  L.colbuf = take(36 * H * 4);
  L.cstage = take(36 * H * 4 + 36 * H);  // candidate values, then one flag byte each
  L.hvbuf = take_other(18 * H * 8);
  L.epart_v = take_other(V * 8);
  L.bm = take(W * 4);
  L.wcnt = take(W * 4);
  L.wp = take(W * 4);
  L.wi = take(W * 4);
  L.incpos = take(6 * H * 4);
  L.roff = take((6 * H + 1) * 4);
  L.coff = take((6 * H + 1) * 4);
  L.erow = take(6 * H * 8);
  L.brow = take((size_t)lim.max_blocks * 4);  // the row of every BSR block
  L.irow = take(6 * H * 4);
  L.csort = take(36 * H * 4);
  L.cval = take(36 * H * 4);
  L.colrun = take(36 * H * 4);
  // block totals of the word scan (two per 1024 words) and of the column scan (one per 256 rows)
  L.part = take(std::max<size_t>(2 * (W / 1024 + 2), 6 * H / 256 + 2) * 4);
  L.scan_tmp_bytes = scan_bytes;
  L.scan_tmp = take_other(scan_bytes);
  L.bvh_keys = take_other(T * 4);
  L.bvh_qend = take_other(T * 4);
  L.bvh_vals = take_other(T * 4);
  L.bvh_vals2 = take_other(T * 4);
  L.bvh_hist = take_other((size_t)kMaxBuckets * 4);
  L.bvh_offset = take_other(((size_t)kMaxBuckets + 1) * 4);
  L.bvh_boxes = take_other((2 * T + 64) * 32);  // implicit tree: at most 2T nodes of 32 B
  L.bvh_leaves = take_other((T + 4) * 64);      // sorted leaf records, padded to a multiple of 4
  L.bvh_tbox = take_other(T * 6 * 8);
  L.bvh_centroid = take_other(T * 3 * 4);
  L.bvh_part = take_other(512 * 6 * 4);
  L.bvh_ext = take_other(512 * 8);
  // saved traversal states (32 B each) of the queries handed to the wave-cooperative kernel
  L.bvh_heavy_bytes = (size_t)std::min<int64_t>(2 * T, (int64_t)1 << 20) * 32;
  L.bvh_heavy = take_other(L.bvh_heavy_bytes);
  L.hash_grid = take_other(64);
  const size_t E = (size_t)kHashEntriesPerTri * T;
  L.hash_key = take_other(E * 8);
  L.hash_tri = take_other(E * 4);
  L.hash_rank = take_other(E * 4);
  L.hash_skey = take_other(E * 8);
  L.hash_stri = take_other(E * 4);
  L.touched = take(6 * H * 4);  // the vertex of each row
  L.inc2 = take(6 * H * sizeof(Incidence));
  L.pcg_vec = take_other(5 * 3 * (size_t)lim.max_verts * 8);
  L.pcg_flag = take_other(V * 4);  // active-row flags, their scan and the active-row list
  L.pcg_pos = take_other(V * 4);
  L.pcg_act = take_other(V * 4);
  L.pcg_part = take_other(5 * 256 * 4 * 8);
  L.pcg_state = take_other(64);
  L.total = o;
  return L;
}

static hipEvent_t pool_get(Ctx* c) {
  if (c->n_pool > 0) return c->event_pool[--c->n_pool];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static void pool_put(Ctx* c, hipEvent_t e) {
  if (!e) return;
  if (c->n_pool == c->cap_pool) {
    const int cap = c->cap_pool ? 2 * c->cap_pool : 64;
    auto* np = static_cast<hipEvent_t*>(realloc(c->event_pool, cap * sizeof(hipEvent_t)));
    if (!np) {
      (void)hipEventDestroy(e);
      return;
    }
    c->event_pool = np;
    c->cap_pool = cap;
  }
  c->event_pool[c->n_pool++] = e;
}

void stage_begin(Ctx* c, int stage, hipStream_t s) {
  if (!(c->timing_mask & (1u << stage))) return;
  if (c->n_timers == c->cap_timers) {
    const int cap = c->cap_timers ? 2 * c->cap_timers : 64;
    auto* nt = static_cast<TimerRec*>(realloc(c->timers, cap * sizeof(TimerRec)));
    if (!nt) return;
    c->timers = nt;
    c->cap_timers = cap;
  }
  TimerRec& r = c->timers[c->n_timers];
  r.stage = stage;
  r.start = pool_get(c);
  r.stop = nullptr;
  if (!r.start || hipEventRecord(r.start, s) != hipSuccess) {
    pool_put(c, r.start);
    return;
  }
  ++c->n_timers;
}

void stage_end(Ctx* c, int stage, hipStream_t s) {
  if (!(c->timing_mask & (1u << stage)) || c->n_timers == 0) return;
  TimerRec& r = c->timers[c->n_timers - 1];
  if (r.stage != stage || r.stop) return;
  r.stop = pool_get(c);
  if (r.stop && hipEventRecord(r.stop, s) != hipSuccess) {
    pool_put(c, r.stop);
    r.stop = nullptr;
  }
}

}  // namespace ttie

using namespace ttie;

struct ttie_ctx : public Ctx {};

namespace {

thread_local std::string g_err;

ttie_status fail(ttie_status st, const char* msg) {
  g_err = msg;
  return st;
}

ttie_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return TTIE_ERR_HIP;
}

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = prev == dev || hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (ok && prev >= 0) (void)hipSetDevice(prev);
  }
};

bool limits_ok(const ttie_limits* l) {
  return l && l->max_verts >= 0 && l->max_tris >= 0 && l->max_pairs >= 0 && l->max_hits >= 0 &&
         l->max_blocks >= 0 && l->max_verts < (1ll << 30) && l->max_tris < (1ll << 31) &&
         l->max_pairs < (1ll << 32) && l->max_hits < (1ll << 26) && 36 * l->max_hits < (1ll << 31);
}

ttie_status check_mesh(ttie_ctx* c, const ttie_mesh* m) {
  if (!m) return fail(TTIE_ERR_INVALID_ARGUMENT, "mesh is NULL");
  if (m->n_verts < 0 || m->n_tris < 0) return fail(TTIE_ERR_INVALID_ARGUMENT, "negative mesh size");
  if ((m->n_verts > 0 && !m->x) || (m->n_tris > 0 && !m->tris))
    return fail(TTIE_ERR_INVALID_ARGUMENT, "mesh array is NULL");
  if (m->n_verts > c->lim.max_verts) return fail(TTIE_ERR_CAPACITY, "n_verts exceeds the workspace limit");
  if (m->n_tris > c->lim.max_tris) return fail(TTIE_ERR_CAPACITY, "n_tris exceeds the workspace limit");
  return TTIE_OK;
}

ttie_status need_ws(ttie_ctx* c) {
  if (!c) return fail(TTIE_ERR_INVALID_ARGUMENT, "context is NULL");
  if (!c->have_ws) return fail(TTIE_ERR_INVALID_ARGUMENT, "no workspace set (ttie_set_workspace)");
  return TTIE_OK;
}

}  // namespace

extern "C" {

const char* ttie_version(void) { return "ttie 0.1.0 (gfx950)"; }

const char* ttie_last_error(void) { return g_err.c_str(); }

ttie_status ttie_create(int device, ttie_ctx** out) {
  if (!out) return fail(TTIE_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(TTIE_ERR_NO_DEVICE, "no HIP device");
  if (device < 0 || device >= n) return fail(TTIE_ERR_INVALID_ARGUMENT, "device index out of range");
  {
    DeviceGuard g(device);
    if (!g.ok) return fail(TTIE_ERR_HIP, "cannot select device");
    const hipError_t e = scratch_lookup(device);
    if (e != hipSuccess) return hip_fail(e, "ttie_create: address of the static scratch");
  }
  auto* c = new ttie_ctx();
  std::memset(static_cast<Ctx*>(c), 0, sizeof(Ctx));
  c->device = device;
  *out = c;
  g_err.clear();
  return TTIE_OK;
}

ttie_status ttie_destroy(ttie_ctx* ctx) {
  if (!ctx) return fail(TTIE_ERR_INVALID_ARGUMENT, "context is NULL");
  for (int k = 0; k < ctx->n_timers; ++k) {
    if (ctx->timers[k].start) (void)hipEventDestroy(ctx->timers[k].start);
    if (ctx->timers[k].stop) (void)hipEventDestroy(ctx->timers[k].stop);
  }
  for (int k = 0; k < ctx->n_pool; ++k) (void)hipEventDestroy(ctx->event_pool[k]);
  free(ctx->timers);
  free(ctx->event_pool);
  delete ctx;
  return TTIE_OK;
}

ttie_status ttie_workspace_size(ttie_ctx* ctx, const ttie_limits* limits, size_t* bytes_host) {
  if (!ctx || !bytes_host) return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL argument");
  if (!limits_ok(limits)) return fail(TTIE_ERR_INVALID_ARGUMENT, "limits out of range");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(TTIE_ERR_HIP, "cannot select device");
  const size_t scan = scan_temp_bytes(scan_len(*limits));
  *bytes_host = layout_with(*limits, scan).total;
  return TTIE_OK;
}

ttie_status ttie_set_workspace(ttie_ctx* ctx, const ttie_limits* limits, void* dptr, size_t bytes, void* stream) {
  if (!ctx || !dptr) return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL argument");
  if (!limits_ok(limits)) return fail(TTIE_ERR_INVALID_ARGUMENT, "limits out of range");
  if (((uintptr_t)dptr) & 255) return fail(TTIE_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(TTIE_ERR_HIP, "cannot select device");
  const size_t scan = scan_temp_bytes(scan_len(*limits));
  Layout L = layout_with(*limits, scan);
  if (bytes < L.total) return fail(TTIE_ERR_CAPACITY, "workspace smaller than ttie_workspace_size");
  ctx->lim = *limits;
  ctx->ws = static_cast<char*>(dptr);
  ctx->ws_bytes = bytes;
  ctx->L = L;
  ctx->have_ws = 1;
  ctx->last_valid = 0;
  hipStream_t s = (hipStream_t)stream;
  // the counters and the per-vertex incidence counts start (and are kept) at zero
  hipError_t e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.counters), sizeof(Counters) / 4, s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.cnt), 32 * (limits->max_verts / 32 + 2), s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.wcnt), limits->max_verts / 32 + 2, s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.bm), limits->max_verts / 32 + 2, s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.cur), limits->max_verts + 1, s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.ncol), limits->max_verts + 1, s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.bvh_hist), kMaxBuckets, s);
  // the scan's counters and tile words (each scan leaves them zero again)
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.scan_tmp), (int64_t)(L.scan_tmp_bytes / 4), s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, L.epart_v), 2 * (limits->max_verts + 1), s);
  if (e != hipSuccess) return hip_fail(e, "ttie_set_workspace");
  return TTIE_OK;
}

ttie_status ttie_get_status(ttie_ctx* ctx, void* stream, ttie_status* status_host) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (!status_host) return fail(TTIE_ERR_INVALID_ARGUMENT, "status_host is NULL");
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  int32_t v = 0;
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(&v, ctx->ws + ctx->L.counters, sizeof(v), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(ctx, ctx->L.counters), 1, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "ttie_get_status");
  *status_host = (ttie_status)v;
  return TTIE_OK;
}

static ttie_status broadphase_impl(ttie_ctx* ctx, const ttie_mesh* mesh, int method, int n_prob, const int64_t* tri_off,
                                   const double* x_end, int32_t* pairs, int64_t capacity, int64_t* n_pairs,
                                   void* stream, const char* who) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (ttie_status st = check_mesh(ctx, mesh)) return st;
  const int base_method = method & ~TTIE_BROAD_VERTEX_ADJACENT;
  if (base_method != TTIE_BROAD_BRUTE && base_method != TTIE_BROAD_LBVH && base_method != TTIE_BROAD_HASH)
    return fail(TTIE_ERR_INVALID_ARGUMENT, "bad method");
  if (!n_pairs || (capacity > 0 && !pairs) || capacity < 0)
    return fail(TTIE_ERR_INVALID_ARGUMENT, "bad pair output");
  if (capacity > ctx->lim.max_pairs) return fail(TTIE_ERR_CAPACITY, "capacity exceeds limits.max_pairs");
  if (((uintptr_t)pairs) & 7) return fail(TTIE_ERR_INVALID_ARGUMENT, "pairs must be 8-byte aligned");
  if (((uintptr_t)n_pairs) & 7) return fail(TTIE_ERR_INVALID_ARGUMENT, "n_pairs must be 8-byte aligned");
  if (base_method == TTIE_BROAD_BRUTE && mesh->n_tris * (mesh->n_tris - 1) / 2 >= (1ll << 32))
    return fail(TTIE_ERR_UNSUPPORTED, "brute force beyond 2^32 pairs");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_broadphase(ctx, mesh, method, x_end, n_prob, tri_off, pairs, capacity, n_pairs,
                                   (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, who);
  return TTIE_OK;
}

ttie_status ttie_broadphase(ttie_ctx* ctx, const ttie_mesh* mesh, int method, const double* x_end, int32_t* pairs,
                            int64_t capacity, int64_t* n_pairs, void* stream) {
  return broadphase_impl(ctx, mesh, method, 1, nullptr, x_end, pairs, capacity, n_pairs, stream, "ttie_broadphase");
}

ttie_status ttie_batch_broadphase(ttie_ctx* ctx, const ttie_mesh* mesh, int n_problems, const int64_t* tri_off,
                                  const double* x_end, int32_t* pairs, int64_t capacity, int64_t* n_pairs,
                                  void* stream) {
  if (n_problems < 1 || n_problems > TTIE_MAX_PROBLEMS)
    return fail(TTIE_ERR_INVALID_ARGUMENT, "n_problems outside [1, TTIE_MAX_PROBLEMS]");
  if (!tri_off) return fail(TTIE_ERR_INVALID_ARGUMENT, "tri_off is NULL");
  return broadphase_impl(ctx, mesh, TTIE_BROAD_LBVH, n_problems, tri_off, x_end, pairs, capacity, n_pairs, stream,
                         "ttie_batch_broadphase");
}

static ttie_status check_eval_args(const ttie_mesh* mesh, const int32_t* pairs, const int64_t* n_pairs,
                                   int64_t pair_capacity, const ttie_options* opts, double* energy, void* grad,
                                   int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity) {
  if (!opts) return fail(TTIE_ERR_INVALID_ARGUMENT, "options are NULL");
  if (opts->precision != TTIE_FP64 && opts->precision != TTIE_MIXED) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad precision");
  if (opts->psd_mode < 0 || opts->psd_mode > 3) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad psd_mode");
  if (opts->interval != TTIE_INTERVAL_EQ1 && opts->interval != TTIE_INTERVAL_APPENDIX_HALF)
    return fail(TTIE_ERR_INVALID_ARGUMENT, "bad interval");
  if (opts->flags & ~TTIE_EVAL_VERTEX_ADJACENT) return fail(TTIE_ERR_INVALID_ARGUMENT, "unknown option flags");
  if ((!pairs && pair_capacity > 0) || !n_pairs || !energy || (!grad && mesh->n_verts > 0))
    return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL required argument");
  if (((uintptr_t)pairs) & 7) return fail(TTIE_ERR_INVALID_ARGUMENT, "pairs must be 8-byte aligned");
  if (pair_capacity < 0) return fail(TTIE_ERR_CAPACITY, "negative pair_capacity");
  const bool bsr = row_ptr || col_idx || vals;
  if (bsr && (!row_ptr || !col_idx || !vals)) return fail(TTIE_ERR_INVALID_ARGUMENT, "partial BSR output");
  if (bsr && block_capacity < 0) return fail(TTIE_ERR_INVALID_ARGUMENT, "negative block_capacity");
  return TTIE_OK;
}

static ttie_status eval_entry(ttie_ctx* ctx, const ttie_mesh* mesh, const int32_t* pairs, const int64_t* n_pairs,
                              int64_t pair_capacity, const ttie_options* opts, double* energy, void* grad, uint8_t* flags,
                              double* pair_T, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity,
                              int64_t* n_blocks, int64_t* n_hits, int n_prob, const int64_t* vert_off,
                              double* energies, void* stream, const char* who) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (ttie_status st = check_mesh(ctx, mesh)) return st;
  if (ttie_status st = check_eval_args(mesh, pairs, n_pairs, pair_capacity, opts, energy, grad, row_ptr, col_idx, vals,
                                       block_capacity))
    return st;
  if (pair_capacity > ctx->lim.max_pairs) return fail(TTIE_ERR_CAPACITY, "pair_capacity outside [0, limits.max_pairs]");
  if (row_ptr && block_capacity > ctx->lim.max_blocks)
    return fail(TTIE_ERR_CAPACITY, "block_capacity exceeds limits.max_blocks");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_eval(ctx, mesh, pairs, n_pairs, pair_capacity, opts, energy, grad, flags, pair_T, row_ptr,
                             col_idx, vals, row_ptr ? block_capacity : 0, n_blocks, n_hits, n_prob, vert_off, energies,
                             nullptr, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, who);
  ctx->last_precision = opts->precision;
  ctx->last_psd = opts->psd_mode;
  ctx->last_interval = opts->interval;
  ctx->last_nverts = mesh->n_verts;
  ctx->last_valid = 1;
  return TTIE_OK;
}



ttie_status ttie_eval(ttie_ctx* ctx, const ttie_mesh* mesh, const int32_t* pairs, const int64_t* n_pairs,
                      int64_t pair_capacity, const ttie_options* opts, double* energy, void* grad, uint8_t* flags, double* pair_T,
                      int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity, int64_t* n_blocks,
                      int64_t* n_hits, void* stream) {
  return eval_entry(ctx, mesh, pairs, n_pairs, pair_capacity, opts, energy, grad, flags, pair_T, row_ptr, col_idx, vals,
                    block_capacity, n_blocks, n_hits, 0, nullptr, nullptr, stream, "ttie_eval");
}

ttie_status ttie_eval_static(ttie_ctx* ctx, const ttie_mesh* mesh, const int32_t* pairs, const int64_t* n_pairs,
                             int64_t pair_capacity, int64_t max_hits, const ttie_options* opts, double* energy,
                             void* grad, uint8_t* flags, double* pair_T, int32_t* row_ptr, int32_t* col_idx, void* vals,
                             int64_t block_capacity, int64_t* n_blocks, int64_t* n_hits, int32_t* status,
                             void* stream) {
  if (!ctx) return fail(TTIE_ERR_INVALID_ARGUMENT, "context is NULL");
  if (!mesh) return fail(TTIE_ERR_INVALID_ARGUMENT, "mesh is NULL");
  if (mesh->n_verts < 0 || mesh->n_tris < 0) return fail(TTIE_ERR_INVALID_ARGUMENT, "negative mesh size");
  if ((mesh->n_verts > 0 && !mesh->x) || (mesh->n_tris > 0 && !mesh->tris))
    return fail(TTIE_ERR_INVALID_ARGUMENT, "mesh array is NULL");
  if (ttie_status st = check_eval_args(mesh, pairs, n_pairs, pair_capacity, opts, energy, grad, row_ptr, col_idx, vals,
                                       block_capacity))
    return st;
  if (max_hits < 0) return fail(TTIE_ERR_INVALID_ARGUMENT, "negative max_hits");
  // the evaluation's regions only, laid out for this call's sizes
  ttie_limits lim{mesh->n_verts, 0, pair_capacity, max_hits, row_ptr ? block_capacity : 0};
  if (!limits_ok(&lim)) return fail(TTIE_ERR_INVALID_ARGUMENT, "sizes out of range");
  const Layout L = layout_with(lim, 0, true);
  if (L.total > (size_t)TTIE_STATIC_SCRATCH_BYTES)
    return fail(TTIE_ERR_CAPACITY, "the sizes need more than the TTIE_STATIC_SCRATCH_BYTES of static scratch");
  void* base = scratch_of(ctx->device);
  if (!base) return fail(TTIE_ERR_HIP, "static scratch not available on this device");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(TTIE_ERR_HIP, "cannot select device");
  // a private view of the context on the static array: no stage timers (they create events)
  Ctx t = *static_cast<Ctx*>(ctx);
  t.timing_mask = 0;
  t.timers = nullptr;
  t.n_timers = t.cap_timers = 0;
  t.event_pool = nullptr;
  t.n_pool = t.cap_pool = 0;
  t.lim = lim;
  t.ws = static_cast<char*>(base);
  t.ws_bytes = (size_t)TTIE_STATIC_SCRATCH_BYTES;
  t.L = L;
  t.have_ws = 1;
  hipStream_t s = (hipStream_t)stream;
  // the array keeps the last call's contents, laid out for that call's sizes: the counters and
  // the counts the evaluation expects at zero are cleared (fill kernels, so a capture holds no
  // memset nodes)
  hipError_t e = launch_fill_zero_i32(wsp<int32_t>(&t, L.counters), sizeof(Counters) / 4, s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(&t, L.cnt), 32 * (lim.max_verts / 32 + 2), s);
  if (e == hipSuccess) e = launch_fill_zero_i32(wsp<int32_t>(&t, L.wcnt), lim.max_verts / 32 + 2, s);
  if (e == hipSuccess)
    e = launch_eval(&t, mesh, pairs, n_pairs, pair_capacity, opts, energy, grad, flags, pair_T, row_ptr, col_idx, vals,
                    row_ptr ? block_capacity : 0, n_blocks, n_hits, 0, nullptr, nullptr, status, s);
  if (e != hipSuccess) return hip_fail(e, "ttie_eval_static");
  return TTIE_OK;
}

ttie_status ttie_batch_eval(ttie_ctx* ctx, const ttie_mesh* mesh, int n_problems, const int64_t* vert_off,
                            const int32_t* pairs, const int64_t* n_pairs, int64_t pair_capacity,
                            const ttie_options* opts, double* energies, double* energy, void* grad, uint8_t* flags,
                            double* pair_T, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity,
                            int64_t* n_blocks, int64_t* n_hits, void* stream) {
  if (n_problems < 1 || n_problems > TTIE_MAX_PROBLEMS)
    return fail(TTIE_ERR_INVALID_ARGUMENT, "n_problems outside [1, TTIE_MAX_PROBLEMS]");
  if (!vert_off || !energies) return fail(TTIE_ERR_INVALID_ARGUMENT, "vert_off or energies is NULL");
  return eval_entry(ctx, mesh, pairs, n_pairs, pair_capacity, opts, energy, grad, flags, pair_T, row_ptr, col_idx, vals,
                    block_capacity, n_blocks, n_hits, n_problems, vert_off, energies, stream, "ttie_batch_eval");
}

ttie_status ttie_get_hits(ttie_ctx* ctx, int64_t capacity, int32_t* ij, double* tc, double* T, double* a, double* b,
                          double* g, double* M, int64_t* count_host, void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (!ctx->last_valid) return fail(TTIE_ERR_INVALID_ARGUMENT, "no evaluation yet");
  if (!count_host || capacity < 0) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad argument");
  DeviceGuard guard(ctx->device);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  Counters ctr;
  if (e == hipSuccess) e = hipMemcpy(&ctr, ctx->ws + ctx->L.counters, sizeof(ctr), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "ttie_get_hits");
  const int64_t H = ctr.last_hits;
  *count_host = H;
  if (H > capacity) return fail(TTIE_ERR_CAPACITY, "more hits than capacity");
  std::vector<HitGeom> hg(H);
  const bool fp64 = ctx->last_precision == TTIE_FP64;
  const size_t rs = fp64 ? sizeof(AsmRec<double>) : sizeof(AsmRec<float>);
  std::vector<char> rec(H * rs);
  if (H > 0) {
    e = hipMemcpy(hg.data(), ctx->ws + ctx->L.hits, H * sizeof(HitGeom), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(rec.data(), ctx->ws + ctx->L.recs, H * rs, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "ttie_get_hits");
  }
  std::vector<int64_t> order(H);
  for (int64_t k = 0; k < H; ++k) order[k] = k;
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return hg[x].key < hg[y].key; });
  for (int64_t q = 0; q < H; ++q) {
    const int64_t k = order[q];
    const HitGeom& h = hg[k];
    if (ij) {
      ij[2 * q] = (int32_t)(h.key >> 32);
      ij[2 * q + 1] = (int32_t)(h.key & 0xffffffff);
    }
    if (tc) {
      tc[2 * q] = h.t0;
      tc[2 * q + 1] = h.t1;
    }
    for (int z = 0; z < 18; ++z) {
      double av, bv, gv, mv = 0.0;
      if (fp64) {
        const auto* r = reinterpret_cast<const AsmRec<double>*>(rec.data() + k * rs);
        av = r->a[z];
        bv = r->b[z];
        gv = r->g[z];
        if (z < 3) mv = r->M[z];
        if (T && z == 0) T[q] = r->T;
      } else {
        const auto* r = reinterpret_cast<const AsmRec<float>*>(rec.data() + k * rs);
        av = r->a[z];
        bv = r->b[z];
        gv = r->g[z];
        if (z < 3) mv = r->M[z];
        if (T && z == 0) T[q] = r->T;
      }
      if (a) a[18 * q + z] = av;
      if (b) b[18 * q + z] = bv;
      if (g) g[18 * q + z] = gv;
      if (M && z < 3) M[3 * q + z] = mv;
    }
  }
  return TTIE_OK;
}

ttie_status ttie_bsr_symbolic(ttie_ctx* ctx, int32_t* row_ptr, int32_t* col_idx, int64_t capacity, int64_t* n_blocks,
                              void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (!ctx->last_valid) return fail(TTIE_ERR_INVALID_ARGUMENT, "no evaluation yet");
  if (!row_ptr || !n_blocks || capacity < 0 || (capacity > 0 && !col_idx))
    return fail(TTIE_ERR_INVALID_ARGUMENT, "bad output arrays");
  if (((uintptr_t)n_blocks) & 7) return fail(TTIE_ERR_INVALID_ARGUMENT, "n_blocks must be 8-byte aligned");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_bsr_symbolic(ctx, row_ptr, col_idx, capacity, n_blocks, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_bsr_symbolic");
  return TTIE_OK;
}

ttie_status ttie_bsr_numeric(ttie_ctx* ctx, const int32_t* row_ptr, const int32_t* col_idx, void* vals, void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (!ctx->last_valid) return fail(TTIE_ERR_INVALID_ARGUMENT, "no evaluation yet");
  if (!row_ptr || !col_idx || !vals) return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL array");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_bsr_numeric(ctx, row_ptr, col_idx, vals, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_bsr_numeric");
  return TTIE_OK;
}

ttie_status ttie_hvp(ttie_ctx* ctx, const ttie_mesh* mesh, const void* v, void* Hv, int mode, void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (ttie_status st = check_mesh(ctx, mesh)) return st;
  if (!ctx->last_valid) return fail(TTIE_ERR_INVALID_ARGUMENT, "no evaluation yet");
  if (mesh->n_verts != ctx->last_nverts) return fail(TTIE_ERR_INVALID_ARGUMENT, "mesh differs from the evaluation");
  if (mode != TTIE_HVP_EXACT && mode != TTIE_HVP_PSD) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad mode");
  if ((!v || !Hv) && mesh->n_verts > 0) return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL vector");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_hvp(ctx, mesh, v, Hv, mode, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_hvp");
  return TTIE_OK;
}

ttie_status ttie_bsr_mv(ttie_ctx* ctx, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                        const void* vals, const void* x, void* y, int precision, void* stream) {
  if (!ctx) return fail(TTIE_ERR_INVALID_ARGUMENT, "context is NULL");
  if (n_rows < 0 || (n_rows > 0 && (!row_ptr || !x || !y)))
    return fail(TTIE_ERR_INVALID_ARGUMENT, "bad argument");
  if (precision != TTIE_FP64 && precision != TTIE_MIXED) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad precision");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_bsr_mv(n_rows, row_ptr, col_idx, vals, x, y, precision, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_bsr_mv");
  return TTIE_OK;
}

ttie_status ttie_pcg(ttie_ctx* ctx, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                     const void* b, double scale, void* x, double mu_rel, int max_iter, double tol, int precision,
                     double* info, void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (n_rows < 0 || n_rows > ctx->lim.max_verts) return fail(TTIE_ERR_CAPACITY, "n_rows outside [0, max_verts]");
  if (n_rows > 0 && (!row_ptr || !col_idx || !vals || !b || !x)) return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL array");
  if (precision != TTIE_FP64 && precision != TTIE_MIXED) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad precision");
  if (max_iter < 0 || !(tol >= 0.0) || !(mu_rel >= 0.0)) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad parameters");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_pcg(ctx, n_rows, row_ptr, col_idx, vals, b, scale, x, mu_rel, max_iter, tol, precision, info,
                            (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_pcg");
  return TTIE_OK;
}

ttie_status ttie_pcg_mf(ttie_ctx* ctx, int64_t n_rows, const void* b, double scale, void* x, double mu_rel, int max_iter,
                        double tol, double* info, void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (!ctx->last_valid) return fail(TTIE_ERR_INVALID_ARGUMENT, "no evaluation to take the Hessian from");
  if (n_rows != ctx->last_nverts) return fail(TTIE_ERR_INVALID_ARGUMENT, "n_rows differs from the last evaluation");
  if (n_rows > 0 && (!b || !x)) return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL array");
  if (max_iter < 0 || !(tol >= 0.0) || !(mu_rel >= 0.0)) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad parameters");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_pcg_mf(ctx, n_rows, b, scale, x, mu_rel, max_iter, tol, info, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_pcg_mf");
  return TTIE_OK;
}

ttie_status ttie_springs_pattern(ttie_ctx* ctx, const ttie_mesh* mesh, int32_t* row_ptr, int32_t* col_idx,
                                 int64_t block_capacity, int64_t* n_blocks, void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (ttie_status st = check_mesh(ctx, mesh)) return st;
  if (!row_ptr || !n_blocks || (block_capacity > 0 && !col_idx) || block_capacity < 0)
    return fail(TTIE_ERR_INVALID_ARGUMENT, "bad output arrays");
  if (mesh->n_verts + 1 >= (1ll << 31)) return fail(TTIE_ERR_UNSUPPORTED, "too many vertices for int32 offsets");
  if (6 * mesh->n_tris + 2 * mesh->n_verts >= (1ll << 31))
    return fail(TTIE_ERR_UNSUPPORTED, "too many edges for int32 offsets");
  DeviceGuard g(ctx->device);
  ctx->last_valid = 0;  // the incidence buffers are reused
  hipError_t e = launch_springs_pattern(ctx, mesh, row_ptr, col_idx, block_capacity, n_blocks, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_springs_pattern");
  return TTIE_OK;
}

ttie_status ttie_qs_eval(ttie_ctx* ctx, int64_t n_verts, const int32_t* row_ptr, const int32_t* col_idx,
                         const double* x, const double* rest, const double* x_prev, double k, double m, double w,
                         const double* e_ttie, const double* g_ttie, double* phi, double* grad, double* vals,
                         void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (n_verts < 0 || n_verts > ctx->lim.max_verts) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad n_verts");
  if (!row_ptr || !phi || (n_verts > 0 && (!col_idx || !x || !rest || !x_prev)))
    return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL array");
  if (!(k >= 0.0) || !(m >= 0.0) || !(w >= 0.0) || !std::isfinite(k) || !std::isfinite(m) || !std::isfinite(w))
    return fail(TTIE_ERR_INVALID_ARGUMENT, "k, m and w must be finite and >= 0");
  if ((e_ttie == nullptr) != (g_ttie == nullptr)) return fail(TTIE_ERR_INVALID_ARGUMENT, "give both E and its gradient");
  if (w > 0.0 && !e_ttie) return fail(TTIE_ERR_INVALID_ARGUMENT, "w > 0 needs E and its gradient");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_qs_eval(ctx, n_verts, row_ptr, col_idx, x, rest, x_prev, k, m, w, e_ttie, g_ttie, phi, grad,
                                vals, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_qs_eval");
  return TTIE_OK;
}

ttie_status ttie_pcg_coupled(ttie_ctx* ctx, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                             const double* vals, double w, const double* b, double scale, double* x, double mu,
                             int max_iter, double tol, double* info, void* stream) {
  if (ttie_status st = need_ws(ctx)) return st;
  if (!ctx->last_valid) return fail(TTIE_ERR_INVALID_ARGUMENT, "no evaluation to take the Hessian from");
  if (ctx->last_precision != TTIE_FP64) return fail(TTIE_ERR_UNSUPPORTED, "the last evaluation must be TTIE_FP64");
  if (n_rows != ctx->last_nverts) return fail(TTIE_ERR_INVALID_ARGUMENT, "n_rows differs from the last evaluation");
  if (n_rows > 0 && (!b || !x || !row_ptr || !col_idx || !vals)) return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL array");
  if (max_iter < 0 || !(tol >= 0.0) || !(mu >= 0.0) || !(w >= 0.0)) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad parameters");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_pcg_coupled(ctx, n_rows, row_ptr, col_idx, vals, w, b, scale, x, mu, max_iter, tol, info,
                                    (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_pcg_coupled");
  return TTIE_OK;
}

ttie_status ttie_axpy(ttie_ctx* ctx, int64_t n_verts, double alpha, const double* x, const void* d, double* out,
                      int precision, void* stream) {
  if (!ctx) return fail(TTIE_ERR_INVALID_ARGUMENT, "context is NULL");
  if (n_verts < 0 || (n_verts > 0 && (!x || !d || !out))) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad argument");
  if (precision != TTIE_FP64 && precision != TTIE_MIXED) return fail(TTIE_ERR_INVALID_ARGUMENT, "bad precision");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_axpy(n_verts, alpha, x, d, out, precision, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ttie_axpy");
  return TTIE_OK;
}

ttie_status ttie_set_param(ttie_ctx* ctx, int param, int64_t value) {
  if (!ctx) return fail(TTIE_ERR_INVALID_ARGUMENT, "context is NULL");
  if (param < 0 || param >= TTIE_PARAM_COUNT) return fail(TTIE_ERR_INVALID_ARGUMENT, "unknown parameter");
  static const int64_t lo[TTIE_PARAM_COUNT] = {64, 64, 16, 16, 64};
  static const int64_t hi[TTIE_PARAM_COUNT] = {65536, 65536, 1 << 20, 1 << 20, 1 << 20};
  if (value != 0 && (value < lo[param] || value > hi[param])) return fail(TTIE_ERR_INVALID_ARGUMENT, "value out of range");
  if (param == TTIE_PARAM_SCREEN_TILE && value % 64 != 0)
    return fail(TTIE_ERR_INVALID_ARGUMENT, "screening tile not a multiple of 64");
  ctx->param[param] = value;
  return TTIE_OK;
}

ttie_status ttie_get_param(ttie_ctx* ctx, int param, int64_t* value_host) {
  if (!ctx || !value_host) return fail(TTIE_ERR_INVALID_ARGUMENT, "NULL argument");
  if (param < 0 || param >= TTIE_PARAM_COUNT) return fail(TTIE_ERR_INVALID_ARGUMENT, "unknown parameter");
  *value_host = ctx_param(ctx, param);
  return TTIE_OK;
}

ttie_status ttie_set_timing(ttie_ctx* ctx, uint32_t stage_mask) {
  if (!ctx) return fail(TTIE_ERR_INVALID_ARGUMENT, "context is NULL");
  ctx->timing_mask = stage_mask & ((1u << TTIE_STAGE_COUNT) - 1u);
  return TTIE_OK;
}

ttie_status ttie_read_timers(ttie_ctx* ctx, int n_stages, int64_t* launches, double* total_ms) {
  if (!ctx || n_stages < 0 || (n_stages > 0 && (!launches || !total_ms)))
    return fail(TTIE_ERR_INVALID_ARGUMENT, "bad argument");
  DeviceGuard g(ctx->device);
  for (int k = 0; k < n_stages; ++k) {
    launches[k] = 0;
    total_ms[k] = 0.0;
  }
  ttie_status st = TTIE_OK;
  for (int k = 0; k < ctx->n_timers; ++k) {
    TimerRec& r = ctx->timers[k];
    if (r.stop && r.stage < n_stages) {
      float ms = 0.f;
      if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
        launches[r.stage] += 1;
        total_ms[r.stage] += ms;
      } else {
        st = fail(TTIE_ERR_HIP, "event timing failed");
      }
    }
    pool_put(ctx, r.start);
    pool_put(ctx, r.stop);
  }
  ctx->n_timers = 0;
  return st;
}

}  // extern "C"
