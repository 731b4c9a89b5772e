// Library-internal declarations: the context, the workspace carve-up and the launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/ttie.h"
#include "pair.h"

namespace ttie {

constexpr int kMortonBucketBits = 22;  // at most 2^22 buckets in the broad-phase counting sort
constexpr int kMaxProblems = TTIE_MAX_PROBLEMS;
constexpr int kHashEntriesPerTri = 8;  // spatial-hash entries reserved per triangle

// Per-hit assembly record in the evaluation's precision S.
template <class S>
struct AsmRec {
  int32_t vid[6];
  int32_t pad;
  int64_t key;
  double T;
  S a[18], b[18], g[18];
  S M[3];
};

// One vertex incidence of a hit: which hit, which of its six slots, and the hit's pair key
// (the per-row summation order).
struct Incidence {
  int64_t key;
  int32_t hit;
  int32_t slot;
};

// Device counters and scalars at the head of the workspace.
struct Counters {
  int32_t status;          // latched TTIE status (first error wins)
  uint32_t n_hits;         // intersecting pairs found by the last screening
  uint32_t last_touched;   // vertices touched by the hits of the last completed evaluation (its rows)
  uint32_t n_defer;        // candidates whose signs need the exact fallback
  uint32_t tile_next;      // next tile of the screening's tile queue (0 between calls)
  uint32_t last_hits;      // hits of the last completed evaluation (for hvp / get_hits)
  uint64_t n_entries;      // (cell, triangle) entries of the spatial-hash broad phase
  uint32_t n_heavy;        // broad-phase work items handed to a wave-cooperative kernel
  uint32_t pad_;
};

// Counters of the one-launch scan (tiles taken, tiles done); both are zero between scans.
struct ScanState {
  uint32_t next_tile;
  uint32_t done;
};

// Number of distinct vertex ids of triangle a that also belong to triangle b.
__device__ __forceinline__ int shared_vertices(const int32_t* a, const int32_t* b) {
  int n = 0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const bool in = (a[x] == b[0]) | (a[x] == b[1]) | (a[x] == b[2]);
    const bool dup = (x > 0 && a[x] == a[0]) | (x > 1 && a[x] == a[1]);
    n += in & !dup;
  }
  return n;
}

// Pairs sharing a vertex are adjacent (Sec. 1) and carry no energy; with the vertex-adjacent
// option only pairs sharing two or more vertices are, and a pair sharing exactly one vertex is
// evaluated like any other.  The option is a kernel argument, so the branch is uniform and the
// default keeps the nine plain comparisons.
__device__ __forceinline__ bool is_adjacent(const int32_t* a, const int32_t* b, bool vertex_adjacent) {
  if (!vertex_adjacent) {
    bool any = false;
#pragma unroll
    for (int x = 0; x < 3; ++x) any |= (a[x] == b[0]) | (a[x] == b[1]) | (a[x] == b[2]);
    return any;
  }
  return shared_vertices(a, b) >= 2;
}

// Blocks are dealt to the XCDs round-robin; renumbering them so that each XCD runs a
// contiguous range of logical blocks keeps each XCD's L2 on one region of the data (nblocks a
// multiple of 8).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks) {
  const int64_t per = nblocks / 8;
  return (b % 8) * per + b / 8;
}

// A thread-strided loop over n items that keeps each XCD on one contiguous eighth of them
// (blocks are dealt to the XCDs round-robin, so block b runs on XCD b mod 8): the thread's
// first item, the end of its XCD's range and the stride.  With a grid that is not a multiple of
// 8 it is the plain grid-strided loop.
struct XcdItems {
  int64_t first, end, step;
};
// (blocks [0, G) of the grid take part: G = gridDim.x unless given)
__device__ __forceinline__ XcdItems xcd_items(int64_t n, int64_t G = -1) {
  if (G < 0) G = gridDim.x;
  const int64_t B = blockDim.x;
  if (G % 8 != 0) return {(int64_t)blockIdx.x * B + threadIdx.x, n, G * B};
  const int64_t per = (n + 7) / 8, beg = min(n, (int64_t)(blockIdx.x % 8) * per);
  return {beg + (int64_t)(blockIdx.x / 8) * B + threadIdx.x, min(n, beg + per), (G / 8) * B};
}

// wave-aggregated append to a counter-indexed list: one atomic per wave; every lane of the wave
// must call it
__device__ __forceinline__ uint32_t wave_slot(bool want, uint32_t* counter) {
  const uint64_t mask = __ballot(want);
  if (!mask) return 0xffffffffu;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  return want ? base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull)) : 0xffffffffu;
}

struct Layout {
  size_t counters, hits, defer, recs, cnt, cur, off, ncol, inc, colbuf, cstage, hvbuf, epart_v, scan_tmp,
      scan_tmp_bytes;
  // rows of the touched vertices: bitmap, per-word counts and prefixes, incidence places,
  // row offsets (incidences, BSR blocks) and row energies
  size_t bm, wcnt, wp, wi, incpos, roff, coff, erow, part, full, nfull, brow;
  // per incidence place: its row; per column candidate place (ranked): the packed (hit, row
  // slot, column slot), the vertex; per distinct column: the start of its candidate run
  size_t irow, csort, cval, colrun;
  // the first stage's exact plane sides of each candidate passed to the full screening
  size_t fsig;
  size_t bvh_heavy, bvh_heavy_bytes, bvh_ext, hash_grid, hash_key, hash_tri, hash_rank, hash_skey, hash_stri, bvh_keys, bvh_qend, bvh_vals, bvh_vals2, bvh_hist, bvh_offset, bvh_boxes, bvh_leaves,
      bvh_tbox, bvh_centroid, bvh_part, touched, inc2, pcg_vec, pcg_part, pcg_state, pcg_flag, pcg_pos, pcg_act;
  size_t total;
};

struct TimerRec {
  int stage;
  hipEvent_t start, stop;
};

struct Ctx {
  int device;
  uint32_t timing_mask;
  TimerRec* timers;        // pending event pairs (library-owned host array)
  int n_timers, cap_timers;
  hipEvent_t* event_pool;  // reusable events
  int n_pool, cap_pool;
  ttie_limits lim;
  char* ws;
  size_t ws_bytes;
  Layout L;
  int have_ws;
  // the last evaluation (for hvp / get_hits)
  int last_precision;
  int last_psd;
  int last_interval;
  int64_t last_nverts;
  int last_valid;
  int64_t param[TTIE_PARAM_COUNT];  // launch parameters, 0 = default
};

// a launch parameter of the context (its default when unset)
inline int64_t ctx_param(const Ctx* c, int k) {
  static const int64_t kDefault[TTIE_PARAM_COUNT] = {4096, 2048, 128, 64, 0};
  return c->param[k] ? c->param[k] : kDefault[k];
}

template <class T>
inline T* wsp(Ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

// Stage timers: begin/end record an event pair around the kernels of `stage` when enabled.
void stage_begin(Ctx* c, int stage, hipStream_t s);
void stage_end(Ctx* c, int stage, hipStream_t s);

// launchers (return hipSuccess or the first error)
hipError_t launch_fill_zero_i32(int32_t* p, int64_t n, hipStream_t s);
// n_prob problems own the triangle ranges [tri_off[p], tri_off[p + 1]) (device array; NULL:
// one problem); no pair joins two problems
hipError_t launch_broadphase(Ctx* c, const ttie_mesh* m, int method, const double* x_end, int n_prob,
                             const int64_t* tri_off, int32_t* pairs, int64_t capacity, int64_t* n_pairs, hipStream_t s);
hipError_t launch_pcg(Ctx* c, int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                      const void* b, double scale, void* x, double mu_rel, int max_iter, double tol, int precision,
                      double* info, hipStream_t s);
hipError_t launch_pcg_coupled(Ctx* c, int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                              double w, const double* b, double scale, double* x, double mu, int max_iter, double tol,
                              double* info, hipStream_t s);
hipError_t launch_springs_pattern(Ctx* c, const ttie_mesh* m, int32_t* row_ptr, int32_t* col_idx, int64_t cap,
                                  int64_t* n_blocks, hipStream_t s);
hipError_t launch_qs_eval(Ctx* c, int64_t nv, const int32_t* row_ptr, const int32_t* col_idx, const double* x,
                          const double* rest, const double* x_prev, double ks, double m, double w,
                          const double* e_ttie, const double* g_ttie, double* phi, double* grad, double* vals,
                          hipStream_t s);
hipError_t launch_pcg_mf(Ctx* c, int64_t n, const void* b, double scale, void* x, double mu_rel, int max_iter,
                         double tol, double* info, hipStream_t s);
hipError_t launch_axpy(int64_t n_verts, double alpha, const double* x, const void* d, double* out, int precision,
                       hipStream_t s);
hipError_t launch_eval(Ctx* c, const ttie_mesh* m, const int32_t* pairs, const int64_t* n_pairs,
                       int64_t pair_capacity, const ttie_options* o, double* energy, void* grad, uint8_t* flags, double* pair_T,
                       int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity, int64_t* n_blocks,
                       int64_t* n_hits, int n_prob, const int64_t* vert_off, double* energies, int32_t* status_out,
                       hipStream_t s);
hipError_t launch_hvp(Ctx* c, const ttie_mesh* m, const void* v, void* Hv, int mode, hipStream_t s);
// BSR pattern and values of the last evaluation's PSD Hessian, as two calls
hipError_t launch_bsr_symbolic(Ctx* c, int32_t* row_ptr, int32_t* col_idx, int64_t capacity, int64_t* n_blocks,
                               hipStream_t s);
hipError_t launch_bsr_numeric(Ctx* c, const int32_t* row_ptr, const int32_t* col_idx, void* vals, hipStream_t s);
hipError_t launch_bsr_mv(int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                         const void* x, void* y, int precision, hipStream_t s);
hipError_t launch_init_counters(Ctx* c, hipStream_t s);
size_t scan_temp_bytes(int64_t n);
// exclusive scan of n int32 in one launch (csrc/scan.hip); scan_temp_bytes sizes its state
hipError_t launch_scan_i32(Ctx* c, const int32_t* in, int32_t* out, int64_t n, hipStream_t s);

}  // namespace ttie
