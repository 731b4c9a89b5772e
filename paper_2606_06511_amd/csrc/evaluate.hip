// Evaluation kernels: screening of the candidate pairs, per-hit derivatives, and the
// deterministic (no floating-point atomics) assembly of energy, gradient and BSR Hessian.
//
// Pipeline on one stream, no host synchronization:
//   k_screen         one lane per candidate: adjacency, FP64-filtered plane sides and flag,
//                    FP64 interval ends; hits and filter-uncertain candidates are appended
//                    with one atomic per wave (ballot + mbcnt)
//   k_screen_exact   the uncertain candidates again, with the exact fallback
//   k_derivs<S>      one lane per hit: a = dt_c^0, b = dt_c^1, T, g (Eq. 3), 2x2 Hessian core;
//                    counts the hit's six vertices and lists the vertices touched first
//   scan             exclusive scan of the per-vertex incidence counts
//   k_fill           scatter (pair key, hit, slot) incidences into per-vertex lists
//   k_rows_sort<S>   one wave per touched vertex: rank-sort its incidences by pair key (the
//                    summation order) and list its distinct neighbour vertices (BSR columns)
//   scan             BSR row pointers from the column counts
//   k_rows_asm<S>    one wave per touched vertex, a lane per column: blocks J_k^T M J_l summed
//                    in pair-key order; the gradient row and the row's energy share
//   k_rows_final<S>  every vertex: zero gradient rows, energy summed in vertex order (fixed
//                    tree per block), coordinate checks, per-vertex counters cleared
//   k_eval_finish    block partials summed in block order; scalar outputs; counters reset
#include <algorithm>


#include "internal.h"

namespace ttie {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ void latch(int32_t* status, int code) { atomicCAS(status, 0, code); }

__global__ void k_fill_zero_i32(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

__device__ __forceinline__ bool load_tri(const double* x, int64_t nv, const int32_t* tris, int64_t t, int32_t vid[3],
                                         Tri64& T) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    vid[k] = tris[3 * t + k];
    ok = ok && vid[k] >= 0 && vid[k] < nv;
  }
  if (!ok) return false;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) T.p[k][c] = x[3 * (int64_t)vid[k] + c];
  return true;
}


// Screens candidate p (p < 0: inactive lane).  Every lane of the wave must call it.
template <bool kExact>
__device__ __forceinline__ void screen_one(int64_t p, const double* __restrict__ x, int64_t nv,
                                           const int32_t* __restrict__ tris, int64_t nt,
                                           const int32_t* __restrict__ pairs, double half, bool va,
                                           HitGeom* __restrict__ hits, uint32_t max_hits, int32_t* __restrict__ defer,
                                           int64_t max_defer, Counters* ctr, uint8_t* __restrict__ flags,
                                           double* __restrict__ pair_T, int& status) {
  int kind = PAIR_NONE;
  Screen sc;
  sc.t0 = sc.t1 = 0.0;
  sc.desc = 0;
  int32_t i = 0, j = 0;
  if (p >= 0) {
    i = pairs[2 * p];
    j = pairs[2 * p + 1];
    int32_t vi[3], vj[3];
    Tri64 A, B;
    if (i < 0 || j < 0 || i >= nt || j >= nt || i == j || !load_tri(x, nv, tris, i, vi, A) ||
        !load_tri(x, nv, tris, j, vj, B)) {
      status = STATUS_INDEX;
    } else {
      if (is_adjacent(vi, vj, va)) {
        kind = PAIR_ADJACENT;
      } else {
        sc = screen_pair<kExact>(A, B, half, status);
        kind = sc.kind;
      }
    }
    if (kind != PAIR_DEFER) {
      if (flags) flags[p] = (uint8_t)kind;
      if (pair_T) {
        const double pr = sc.t0 * sc.t1;
        pair_T[p] = kind == PAIR_HIT ? pr * pr : 0.0;
      }
    }
  }
  if (!kExact) {
    const uint32_t ds = wave_slot(kind == PAIR_DEFER, &ctr->n_defer);
    if (kind == PAIR_DEFER) {
      if ((int64_t)ds < max_defer) defer[ds] = (int32_t)p;
      else status = STATUS_CAPACITY;
    }
  }
  const bool is_hit = kind == PAIR_HIT;
  const uint32_t slot = wave_slot(is_hit, &ctr->n_hits);
  if (is_hit) {
    if (slot < max_hits) {
      HitGeom g;
      g.key = ((int64_t)i << 32) | (int64_t)(uint32_t)j;
      g.pair = (int32_t)p;
      g.desc = sc.desc;
      g.t0 = sc.t0;
      g.t1 = sc.t1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        g.da[k] = sc.da[k];
        g.db[k] = sc.db[k];
      }
      hits[slot] = g;
    } else {
      status = STATUS_CAPACITY;
    }
  }
}

// ---- the fast pass: FP64 filters only, uncertain pairs deferred --------------------------
// The screening of Sec. 1 is a cascade whose stages let fewer and fewer pairs through: on the
// noisy spheres about 35% of the candidates have a vertex of T_a on each side of T_b's plane,
// about 19% also the converse, and 0.2% intersect.  One lane per candidate all the way down
// would make every wave execute every stage (some lane nearly always goes on).  Instead each
// wave runs a stage on 64 candidates at once and queues the survivors in LDS; the next stage
// runs when 64 are queued.  The last stage is the full screening of screen_one, so every
// decision and value is exactly the one-pass result.
constexpr int kQueue = 128;  // queue slots per wave and stage (at most 63 waiting + 64 arriving)

enum { STEP_SETTLED = 0, STEP_DEFER = 1, STEP_NEXT = 2, STEP_FULL = 3 };

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Appends the lanes that want it to a wave's LDS queue; n is wave-uniform.
__device__ __forceinline__ void queue_push(uint32_t* q, int& n, bool want, int64_t p) {
  const uint64_t mask = __ballot(want);
  if (want) q[n + __popcll(mask & ((1ull << __lane_id()) - 1ull))] = (uint32_t)p;
  n += __popcll(mask);
  wave_sync_lds();
}

__device__ __forceinline__ void defer_append(bool want, int64_t p, int32_t* defer, int64_t max_defer, Counters* ctr,
                                             int& status) {
  const uint32_t ds = wave_slot(want, &ctr->n_defer);
  if (want) {
    if ((int64_t)ds < max_defer) defer[ds] = (int32_t)p;
    else status = STATUS_CAPACITY;
  }
}

__device__ __forceinline__ void settle(int64_t p, int kind, uint8_t* flags, double* pair_T) {
  if (flags) flags[p] = (uint8_t)kind;
  if (pair_T) pair_T[p] = 0.0;
}

__device__ __forceinline__ bool load_pair(int64_t p, const double* x, int64_t nv, const int32_t* tris, int64_t nt,
                                          const int32_t* pairs, int32_t vi[3], int32_t vj[3], Tri64& A, Tri64& B) {
  const int32_t i = pairs[2 * p], j = pairs[2 * p + 1];
  if (i < 0 || j < 0 || i >= nt || j >= nt || i == j) return false;
  return load_tri(x, nv, tris, i, vi, A) && load_tri(x, nv, tris, j, vj, B);
}

// Stage 1 (every candidate): indices, adjacency, T_a's sides against T_b's plane.
__device__ __forceinline__ int screen_stage1(int64_t p, const double* x, int64_t nv, const int32_t* tris, int64_t nt,
                                             const int32_t* pairs, bool va, uint8_t* flags, double* pair_T,
                                             int& status) {
  int32_t vi[3], vj[3];
  Tri64 A, B;
  if (!load_pair(p, x, nv, tris, nt, pairs, vi, vj, A, B)) {
    status = STATUS_INDEX;
    settle(p, PAIR_NONE, flags, pair_T);
    return STEP_SETTLED;
  }
  if (is_adjacent(vi, vj, va)) {
    settle(p, PAIR_ADJACENT, flags, pair_T);
    return STEP_SETTLED;
  }
  int sa[3];
  double da[3];
  if (!plane_sides<false>(B, A, sa, da, status)) return STEP_DEFER;
  if ((sa[0] | sa[1] | sa[2]) == 0) return STEP_FULL;  // T_a in T_b's plane: the coplanar test
  if (!make_cut(sa[0], sa[1], sa[2]).straddle) {
    settle(p, PAIR_NONE, flags, pair_T);
    return STEP_SETTLED;
  }
  return STEP_NEXT;
}

// Stage 2 (T_a straddles T_b's plane): T_b's sides against T_a's plane.
__device__ __forceinline__ int screen_stage2(int64_t p, const double* x, int64_t nv, const int32_t* tris, int64_t nt,
                                             const int32_t* pairs, uint8_t* flags, double* pair_T, int& status) {
  int32_t vi[3], vj[3];
  Tri64 A, B;
  load_pair(p, x, nv, tris, nt, pairs, vi, vj, A, B);  // checked in stage 1
  int sb[3];
  double db[3];
  if (!plane_sides<false>(A, B, sb, db, status)) return STEP_DEFER;
  if (!make_cut(sb[0], sb[1], sb[2]).straddle) {
    settle(p, PAIR_NONE, flags, pair_T);
    return STEP_SETTLED;
  }
  return STEP_NEXT;
}

__global__ void __launch_bounds__(kBlock) k_screen(const double* __restrict__ x, int64_t nv,
                                                   const int32_t* __restrict__ tris, int64_t nt,
                                                   const int32_t* __restrict__ pairs, const int64_t* n_pairs_dev,
                                                   int64_t max_pairs, double half, int va, HitGeom* __restrict__ hits,
                                                   uint32_t max_hits, int32_t* __restrict__ defer, Counters* ctr,
                                                   uint8_t* __restrict__ flags, double* __restrict__ pair_T) {
  __shared__ uint32_t q1s[kWaves][kQueue], q2s[kWaves][kQueue];
  const int wave = threadIdx.x / 64, lane = __lane_id();
  uint32_t* q1 = q1s[wave];
  uint32_t* q2 = q2s[wave];
  const int64_t np = min(*n_pairs_dev, max_pairs);
  // each wave screens one contiguous chunk of the list; blocks are renumbered so that each XCD
  // runs a contiguous range of chunks (its L2 then sees one region of the mesh)
  const int64_t G = gridDim.x;
  const int64_t lb = (G % 8 == 0) ? xcd_block(blockIdx.x, G) : (int64_t)blockIdx.x;
  const int64_t nw = G * kWaves;
  const int64_t chunk = ((np + nw - 1) / nw + 63) / 64 * 64;
  const int64_t beg = (lb * kWaves + wave) * chunk, end = min(np, beg + chunk);
  int n1 = 0, n2 = 0, status = 0;
  int64_t base = beg;
  // One stage per round, chosen wave-uniformly: the last stage as soon as 64 candidates wait for
  // it, then the middle one, then a new batch; at the end of the chunk the queues drain.  Each
  // stage runs from one place in the code, so only one of them is live in registers at a time.
  // Stage 1 runs only with both queues below 64 and stage 2 only with the last one below 64, so
  // no queue ever holds more than 127.
  while (true) {
    const bool more = base < end;
    int st = STEP_SETTLED;
    int64_t p = -1;
    if (n2 >= 64 || (!more && n1 == 0 && n2 > 0)) {
      const int take = min(n2, 64);
      p = lane < take ? (int64_t)q2[n2 - take + lane] : -1;
      wave_sync_lds();
      n2 -= take;
      screen_one<false>(p, x, nv, tris, nt, pairs, half, va != 0, hits, max_hits, defer, max_pairs, ctr, flags,
                        pair_T, status);
      continue;
    }
    if (n1 >= 64 || (!more && n1 > 0)) {
      const int take = min(n1, 64);
      p = lane < take ? (int64_t)q1[n1 - take + lane] : -1;
      wave_sync_lds();
      n1 -= take;
      if (p >= 0) st = screen_stage2(p, x, nv, tris, nt, pairs, flags, pair_T, status);
      defer_append(st == STEP_DEFER, p, defer, max_pairs, ctr, status);
      queue_push(q2, n2, st == STEP_NEXT, p);
      continue;
    }
    if (!more) break;
    p = base + lane < end ? base + lane : -1;
    base += 64;
    if (p >= 0) st = screen_stage1(p, x, nv, tris, nt, pairs, va != 0, flags, pair_T, status);
    defer_append(st == STEP_DEFER, p, defer, max_pairs, ctr, status);
    queue_push(q2, n2, st == STEP_FULL, p);
    queue_push(q1, n1, st == STEP_NEXT, p);
  }
  if (status) latch(&ctr->status, status);
}

// exact pass over the deferred candidates
__global__ void __launch_bounds__(kBlock) k_screen_exact(const double* __restrict__ x, int64_t nv,
                                                         const int32_t* __restrict__ tris, int64_t nt,
                                                         const int32_t* __restrict__ pairs, int64_t max_pairs,
                                                         double half, int va, HitGeom* __restrict__ hits,
                                                         uint32_t max_hits,
                                                         const int32_t* __restrict__ defer, Counters* ctr,
                                                         uint8_t* __restrict__ flags, double* __restrict__ pair_T) {
  const int64_t nd = min((int64_t)ctr->n_defer, max_pairs);
  int status = 0;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nd; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = base + threadIdx.x;
    screen_one<true>(q < nd ? (int64_t)defer[q] : -1, x, nv, tris, nt, pairs, half, va != 0, hits, max_hits, nullptr,
                     0, ctr, flags, pair_T, status);
  }
  if (status) latch(&ctr->status, status);
}

// Pair-local coordinates of a hit in scalar S: relative to u0 (formed in float64) and multiplied
// by 2^-e, e the exponent of the largest of them (returned), so that the largest lies in [1, 2).
// Scaling by a power of two is exact and changes no relative rounding; it only keeps a tiny or
// huge pair's products inside float32's range.
template <class S>
__device__ __forceinline__ int local_coords(const double* x, const int32_t vid[6], V3<S> X[6]) {
  const double o0 = x[3 * (int64_t)vid[0]], o1 = x[3 * (int64_t)vid[0] + 1], o2 = x[3 * (int64_t)vid[0] + 2];
  double d[6][3];
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double* p = x + 3 * (int64_t)vid[k];
    d[k][0] = p[0] - o0;
    d[k][1] = p[1] - o1;
    d[k][2] = p[2] - o2;
    m = fmax(m, fmax(fabs(d[k][0]), fmax(fabs(d[k][1]), fabs(d[k][2]))));
  }
  const int e = m > 0.0 ? ilogb(m) : 0;
#pragma unroll
  for (int k = 0; k < 6; ++k)
    X[k] = V3<S>{Sc<S>::c(ldexp(d[k][0], -e)), Sc<S>::c(ldexp(d[k][1], -e)), Sc<S>::c(ldexp(d[k][2], -e))};
  return e;
}

__device__ __forceinline__ void hit_vids(const int32_t* tris, int64_t key, int32_t vid[6]) {
  const int64_t i = key >> 32, j = key & 0xffffffffll;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    vid[k] = tris[3 * i + k];
    vid[3 + k] = tris[3 * j + k];
  }
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_derivs(const double* __restrict__ x, const int32_t* __restrict__ tris,
                                                   const HitGeom* __restrict__ hits, Counters* ctr, uint32_t max_hits,
                                                   int psd_mode, double half, AsmRec<S>* __restrict__ recs,
                                                   int32_t* __restrict__ cnt, int32_t* __restrict__ touched) {
  const uint32_t H = min(ctr->n_hits, max_hits);
  for (uint32_t base = blockIdx.x * blockDim.x; base < H; base += gridDim.x * blockDim.x) {
    const uint32_t h = base + threadIdx.x;
    const bool active = h < H;
    int32_t vid[6] = {0, 0, 0, 0, 0, 0};
    if (active) {
      const HitGeom g = hits[h];
      AsmRec<S> r;
      hit_vids(tris, g.key, r.vid);
      r.pad = 0;
      r.key = g.key;
      V3<S> X[6];
      const int e = local_coords<S>(x, r.vid, X);
      interval_grads<S>(X, g.da, g.db, e, g.desc, half, r.a, r.b);
      const double t0 = g.t0, t1 = g.t1;
      const double pr = t0 * t1;
      r.T = pr * pr;
      // Eq. 3: dT = 2 t0 t1^2 a + 2 t1 t0^2 b
      const S ca = Sc<S>::c(2.0 * pr * t1), cb = Sc<S>::c(2.0 * pr * t0);
      double aa = 0, bb = 0, ab = 0;
#pragma unroll
      for (int k = 0; k < 18; ++k) {
        r.g[k] = ca * r.a[k] + cb * r.b[k];
        aa += (double)r.a[k] * (double)r.a[k];
        bb += (double)r.b[k] * (double)r.b[k];
        ab += (double)r.a[k] * (double)r.b[k];
      }
      double M[3];
      hessian_core(psd_mode, t0, t1, aa, bb, ab, M);
      r.M[0] = Sc<S>::c(M[0]);
      r.M[1] = Sc<S>::c(M[1]);
      r.M[2] = Sc<S>::c(M[2]);
      recs[h] = r;
#pragma unroll
      for (int k = 0; k < 6; ++k) vid[k] = r.vid[k];
    }
    // count the six incidences (all six atomics in flight at once); a vertex whose count
    // leaves 0 joins the touched list, the wave reserving its slots with one atomic
    int32_t old[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) old[k] = active ? atomicAdd(&cnt[vid[k]], 1) : 1;
    uint64_t fm[6];
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      fm[k] = __ballot(old[k] == 0);
      total += (uint32_t)__popcll(fm[k]);
    }
    if (total) {
      uint32_t wbase = 0;
      if (__lane_id() == 0) wbase = atomicAdd(&ctr->n_touched, total);
      wbase = __builtin_amdgcn_readfirstlane(wbase);
      const uint64_t below = (1ull << __lane_id()) - 1ull;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if (old[k] == 0) touched[wbase + (uint32_t)__popcll(fm[k] & below)] = vid[k];
        wbase += (uint32_t)__popcll(fm[k]);
      }
    }
  }
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_fill(const AsmRec<S>* __restrict__ recs, const Counters* ctr,
                                                 uint32_t max_hits, const int32_t* __restrict__ off,
                                                 int32_t* __restrict__ cur, Incidence* __restrict__ inc) {
  const uint32_t H = min(ctr->n_hits, max_hits);
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < 6 * H; t += gridDim.x * blockDim.x) {
    const uint32_t h = t / 6, k = t % 6;
    const int32_t v = recs[h].vid[k];
    const int32_t pos = off[v] + atomicAdd(&cur[v], 1);
    inc[pos] = Incidence{recs[h].key, (int32_t)h, (int32_t)k};
  }
}

constexpr int kCandCap = 256;  // column candidates staged in LDS per wave
constexpr int kRowStage = 16;  // incidences (and their hit records) a wave stages in LDS per row

// The distinct columns of one row, in increasing vertex order, written to out: the six vertex
// ids of every incident hit go to cand with a first-occurrence flag each, and a kept candidate
// goes to the number of kept candidates with a smaller id.  Returns the count (every lane).
template <class S>
__device__ __forceinline__ int32_t row_columns(int32_t* cand, uint8_t* first, int32_t m, bool staged,
                                               const Incidence* sinc, const Incidence* __restrict__ rinc,
                                               const AsmRec<S>* __restrict__ recs, int32_t* __restrict__ out,
                                               int lane) {
  if (staged) {
    for (int32_t c = lane; c < m; c += 64) cand[c] = recs[sinc[c / 6].hit].vid[c % 6];
  } else {
    for (int32_t c = lane; c < m; c += 64) cand[c] = recs[rinc[c / 6].hit].vid[c % 6];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int32_t c = lane; c < m; c += 64) {
    const int32_t val = cand[c];
    // no early exit: the loads are independent, so they pipeline instead of each waiting for
    // the previous compare
    uint32_t dup = 0;
    for (int32_t j = 0; j < c; ++j) dup |= (uint32_t)(cand[j] == val);
    first[c] = dup ? 0 : 1;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  int32_t kept = 0;
  for (int32_t c = lane; c < m; c += 64) {
    if (!first[c]) continue;
    const int32_t val = cand[c];
    int32_t pos = 0;
    for (int32_t j = 0; j < m; ++j) pos += (int32_t)(first[j] != 0 && cand[j] < val);
    out[pos] = val;
    ++kept;
  }
  for (int w = 32; w > 0; w >>= 1) kept += __shfl_xor(kept, w);
  return kept;
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_rows_sort(const int32_t* __restrict__ touched, const Counters* ctr,
                                                      const int32_t* __restrict__ off,
                                                      const Incidence* __restrict__ inc,
                                                      Incidence* __restrict__ inc2, const AsmRec<S>* __restrict__ recs,
                                                      int32_t* __restrict__ colbuf, int32_t* __restrict__ cstage,
                                                      int64_t cstage_len, int32_t* __restrict__ ncol, int want_bsr) {
  __shared__ int32_t lcand[kWaves][kCandCap];
  __shared__ uint8_t lflag[kWaves][kCandCap];
  __shared__ Incidence sinc[kWaves][64];
  const int wave = threadIdx.x / 64, lane = __lane_id();
  const uint32_t U = ctr->n_touched;
  for (uint32_t u = blockIdx.x * kWaves + wave; u < U; u += gridDim.x * kWaves) {
    const int32_t v = touched[u];
    const int32_t b = off[v], n = off[v + 1] - b;
    // rank sort of the row's incidences by (pair key, slot, position): deterministic even when
    // a hit holds the vertex twice (a pair sharing one vertex), and a permutation even if a
    // caller repeats a pair.  Rows of up to 64 (wave-uniform test) rank from LDS.
    if (n <= 64) {
      Incidence me{};
      if (lane < n) sinc[wave][lane] = me = inc[b + lane];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (lane < n) {
        int32_t rank = 0;
        for (int32_t j = 0; j < n; ++j) {
          const Incidence o = sinc[wave][j];
          rank += (o.key < me.key) |
                  ((o.key == me.key) & ((o.slot < me.slot) | ((o.slot == me.slot) & (j < lane))));
        }
        inc2[b + rank] = me;
      }
    } else {
      for (int32_t i = lane; i < n; i += 64) {
        const Incidence me = inc[b + i];
        int32_t rank = 0;
        for (int32_t j = 0; j < n; ++j) {
          const Incidence o = inc[b + j];
          rank += o.key < me.key || (o.key == me.key && (o.slot < me.slot || (o.slot == me.slot && j < i)));
        }
        inc2[b + rank] = me;
      }
    }
    if (want_bsr) {
      // candidate columns: the six vertices of every incident hit, staged in LDS (or, for very
      // large rows, in the workspace) with a first-occurrence flag each.  The two cases are
      // separate calls so that the LDS one reads LDS directly (a pointer that may point to
      // either memory would compile to slower generic loads).
      const int32_t m = 6 * n;
      int32_t kept;
      if (m <= kCandCap)
        kept = row_columns(lcand[wave], lflag[wave], m, n <= 64, sinc[wave], inc + b, recs, colbuf + 6 * (int64_t)b,
                           lane);
      else
        kept = row_columns(cstage + 6 * (int64_t)b, reinterpret_cast<uint8_t*>(cstage + cstage_len) + 6 * (int64_t)b,
                           m, false, sinc[wave], inc + b, recs, colbuf + 6 * (int64_t)b, lane);
      if (lane == 0) ncol[v] = kept;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the LDS staging is reused by the wave's next row
  }
}

template <class S>
__device__ __forceinline__ void block_jmj(const AsmRec<S>& r, int s, int l, S B[9]) {
  // J_s^T M J_l = M00 a_s a_l^T + M01 (a_s b_l^T + b_s a_l^T) + M11 b_s b_l^T
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const S as = r.a[3 * s + i], bs = r.b[3 * s + i], al = r.a[3 * l + j], bl = r.b[3 * l + j];
      B[3 * i + j] = B[3 * i + j] + (r.M[0] * as * al + r.M[1] * (as * bl + bs * al) + r.M[2] * bs * bl);
    }
}

// One touched row per wave: the gradient row and the energy of the hits this vertex owns
// (each hit counted at its first vertex), summed in pair-key order, then the row's BSR blocks,
// one lane per column.  The row's incidences and hit records pass through LDS in chunks of
// kRowStage (one memory round trip per chunk instead of a chain of dependent loads per
// incidence); the sums run over the incidences in order, chunk after chunk.
template <class S>
__global__ void __launch_bounds__(kBlock) k_rows_asm(const int32_t* __restrict__ touched, const Counters* ctr,
                                                     const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc2,
                                                     const AsmRec<S>* __restrict__ recs,
                                                     const int32_t* __restrict__ colbuf,
                                                     const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx,
                                                     S* __restrict__ vals, int64_t block_cap, S* __restrict__ grad,
                                                     double* __restrict__ epart, int32_t* status_word) {
  __shared__ AsmRec<S> srec[kWaves][kRowStage];
  __shared__ Incidence sinc[kWaves][kRowStage];
  constexpr int kWords = (int)(sizeof(AsmRec<S>) / 8);
  static_assert(sizeof(AsmRec<S>) % 8 == 0, "records are copied as 8-byte words");
  const int wave = threadIdx.x / 64, lane = __lane_id();
  AsmRec<S>* R = srec[wave];
  Incidence* I = sinc[wave];
  // stages incidences [k0, k0 + cnt) of the row starting at b (every lane of the wave calls it)
  auto stage = [&](int32_t b, int32_t k0, int32_t cnt) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the previous chunk is no longer read
    if (lane < cnt) I[lane] = inc2[b + k0 + lane];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < cnt * kWords; j += 64) {
      const int r = j / kWords, w = j % kWords;
      reinterpret_cast<uint2*>(&R[r])[w] = reinterpret_cast<const uint2*>(&recs[I[r].hit])[w];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  const uint32_t U = ctr->n_touched;
  int status = 0;
  for (uint32_t u = blockIdx.x * kWaves + wave; u < U; u += gridDim.x * kWaves) {
    const int32_t v = touched[u];
    const int32_t b = off[v], n = off[v + 1] - b;
    // gradient row (lanes 0-2) and energy (lane 3)
    S acc = Sc<S>::c(0.0);
    double erow = 0.0;
    for (int32_t k0 = 0; k0 < n; k0 += kRowStage) {
      const int32_t cnt = min(n - k0, kRowStage);
      stage(b, k0, cnt);
      if (lane < 4)
        for (int32_t k = 0; k < cnt; ++k) {
          if (lane < 3) acc = acc + R[k].g[3 * I[k].slot + lane];
          else if (I[k].slot == 0) erow += R[k].T;
        }
    }
    if (lane < 3) grad[3 * (int64_t)v + lane] = acc;
    else if (lane == 3) epart[v] = erow;
    if (!row_ptr) continue;
    // BSR blocks: lane q owns column q (rows with more than 64 columns take several rounds)
    const int32_t rp = row_ptr[v], nc = row_ptr[v + 1] - rp;
    for (int32_t q0 = 0; q0 < nc; q0 += 64) {
      const int32_t q = q0 + lane;
      const int32_t col = q < nc ? colbuf[6 * (int64_t)b + q] : -1;
      S B[9];
#pragma unroll
      for (int z = 0; z < 9; ++z) B[z] = Sc<S>::c(0.0);
      for (int32_t k0 = 0; k0 < n; k0 += kRowStage) {
        const int32_t cnt = min(n - k0, kRowStage);
        if (n > kRowStage || q0 > 0) stage(b, k0, cnt);  // a one-chunk row is still in LDS
        for (int32_t k = 0; k < cnt; ++k) {
          // the hit's slots holding this lane's column, in slot order: the lanes hold distinct
          // columns, so one pass of block_jmj serves every lane that matches a slot of the hit
          // (instead of one pass per slot, most with a single lane active)
          uint32_t match = 0;
#pragma unroll
          for (int l = 0; l < 6; ++l) match |= (uint32_t)(R[k].vid[l] == col) << l;
          while (match) {
            block_jmj(R[k], I[k].slot, __builtin_ctz(match), B);
            match &= match - 1;
          }
        }
      }
      if (q < nc) {
        const int64_t pos = (int64_t)rp + q;
        if (pos < block_cap) {
          col_idx[pos] = col;
#pragma unroll
          for (int z = 0; z < 9; ++z) vals[9 * pos + z] = B[z];
        } else {
          status = STATUS_CAPACITY;
        }
      }
    }
  }
  if (status) latch(status_word, status);
}

// Energy of each problem of a batch: block p sums the per-vertex energies of its vertex range
// in a fixed order (thread-strided, then a tree).  Runs before k_rows_final clears them.
__global__ void __launch_bounds__(kBlock) k_problem_energy(int64_t nv, int n_prob, const int64_t* __restrict__ vert_off,
                                                           const double* __restrict__ epart, double* __restrict__ energies,
                                                           Counters* ctr) {
  __shared__ double red[kBlock];
  const int p = blockIdx.x;
  int64_t b = vert_off[p], e = vert_off[p + 1];
  if (threadIdx.x == 0 && (b > e || b < 0 || e > nv || (p == 0 && b != 0) || (p == n_prob - 1 && e != nv)))
    latch(&ctr->status, STATUS_INVALID);
  b = max((int64_t)0, min(b, nv));
  e = max(b, min(e, nv));
  double acc = 0.0;
  for (int64_t v = b + threadIdx.x; v < e; v += kBlock) acc += epart[v];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) energies[p] = red[0];
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_rows_final(int64_t nv, const double* __restrict__ x,
                                                       int32_t* __restrict__ cnt, int32_t* __restrict__ cur,
                                                       int32_t* __restrict__ ncol, double* __restrict__ epart,
                                                       S* __restrict__ grad, double* __restrict__ blockpart,
                                                       Counters* ctr) {
  __shared__ double red[kBlock];
  double esum = 0.0;
  int code = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    if (cnt[v] > 0) {
      esum += epart[v];
      cnt[v] = 0;
      cur[v] = 0;
      ncol[v] = 0;
      epart[v] = 0.0;
    } else {
      grad[3 * v] = Sc<S>::c(0.0);
      grad[3 * v + 1] = Sc<S>::c(0.0);
      grad[3 * v + 2] = Sc<S>::c(0.0);
    }
    // every coordinate: finite, and 0 or of magnitude in [2^-200, 2^200] (the domain on which
    // the exact predicates are exact)
    for (int c = 0; c < 3; ++c) {
      const double q = fabs(x[3 * v + c]);
      if (!(q <= 1.7976931348623157e308)) code = STATUS_NONFINITE;
      else if (q != 0.0 && (q < 6.223015277861142e-61 || q > 1.6069380442589903e60) && !code)
        code = STATUS_UNSUPPORTED;
    }
  }
  if (code) latch(&ctr->status, code);
  red[threadIdx.x] = esum;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) blockpart[blockIdx.x] = red[0];
}

// Sums the block partials in block order, writes the scalar outputs, hands the hit list to
// hvp / get_hits and resets the counters for the next evaluation (one wave).
__global__ void __launch_bounds__(kBlock) k_eval_finish(int nblocks, const double* __restrict__ blockpart, Counters* ctr,
                                                        uint32_t max_hits, const int32_t* __restrict__ row_ptr,
                                                        int64_t nv, int64_t block_cap, double* energy,
                                                        int64_t* n_blocks, int64_t* n_hits) {
  // fixed-order sum: thread t adds partials t, t + 256, ..., then a tree
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += kBlock) acc += blockpart[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double E = red[0];
  *energy = E;
  const uint32_t H = ctr->n_hits;
  if (n_hits) *n_hits = (int64_t)H;
  if (H > max_hits) latch(&ctr->status, STATUS_CAPACITY);
  if (row_ptr) {
    const int64_t nb = row_ptr[nv];
    if (n_blocks) *n_blocks = nb;
    if (nb > block_cap) latch(&ctr->status, STATUS_CAPACITY);
  }
  ctr->last_hits = min(H, max_hits);
  ctr->last_touched = ctr->n_touched;
  ctr->n_hits = 0;
  ctr->n_defer = 0;
  ctr->n_touched = 0;
}

// ------------------------------------------------------------------------------------------
// The BSR Hessian of the last evaluation as two calls: the pattern (symbolic) and the values
// on a caller's pattern (numeric), from the hit records and the sorted incidence lists the
// evaluation leaves in the workspace.
// ------------------------------------------------------------------------------------------
// Symbolic, first pass: the distinct columns of every touched row (as in k_rows_sort) and
// their count.
template <class S>
__global__ void __launch_bounds__(kBlock) k_sym_cols(const int32_t* __restrict__ touched, const Counters* ctr,
                                                     const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc2,
                                                     const AsmRec<S>* __restrict__ recs, int32_t* __restrict__ colbuf,
                                                     int32_t* __restrict__ cstage, int64_t cstage_len,
                                                     int32_t* __restrict__ ncol) {
  __shared__ int32_t lcand[kWaves][kCandCap];
  __shared__ uint8_t lflag[kWaves][kCandCap];
  __shared__ Incidence sinc[kWaves][64];
  const int wave = threadIdx.x / 64, lane = __lane_id();
  const uint32_t U = ctr->last_touched;
  for (uint32_t u = blockIdx.x * kWaves + wave; u < U; u += gridDim.x * kWaves) {
    const int32_t v = touched[u];
    const int32_t b = off[v], n = off[v + 1] - b;
    const int32_t m = 6 * n;
    int32_t kept;
    if (m <= kCandCap)
      kept = row_columns(lcand[wave], lflag[wave], m, false, sinc[wave], inc2 + b, recs, colbuf + 6 * (int64_t)b,
                         lane);
    else
      kept = row_columns(cstage + 6 * (int64_t)b, reinterpret_cast<uint8_t*>(cstage + cstage_len) + 6 * (int64_t)b,
                         m, false, sinc[wave], inc2 + b, recs, colbuf + 6 * (int64_t)b, lane);
    if (lane == 0) ncol[v] = kept;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Symbolic, second pass (after the row pointers): column indices of every touched row, the
// column counts cleared for the next call, the block count.
__global__ void __launch_bounds__(kBlock) k_sym_write(const int32_t* __restrict__ touched, Counters* ctr,
                                                      const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ colbuf,
                                                      const int32_t* __restrict__ row_ptr, int64_t nv,
                                                      int32_t* __restrict__ col_idx, int64_t cap,
                                                      int32_t* __restrict__ ncol, int64_t* n_blocks) {
  const int wave = threadIdx.x / 64, lane = __lane_id();
  const uint32_t U = ctr->last_touched;
  int status = 0;
  for (uint32_t u = blockIdx.x * kWaves + wave; u < U; u += gridDim.x * kWaves) {
    const int32_t v = touched[u];
    const int32_t b = off[v], rp = row_ptr[v], nc = row_ptr[v + 1] - rp;
    for (int32_t q = lane; q < nc; q += 64) {
      if ((int64_t)rp + q < cap) col_idx[rp + q] = colbuf[6 * (int64_t)b + q];
      else status = STATUS_CAPACITY;
    }
    if (lane == 0) ncol[v] = 0;
  }
  if (status) latch(&ctr->status, status);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t nb = row_ptr[nv];
    *n_blocks = nb;
    if (nb > cap) latch(&ctr->status, STATUS_CAPACITY);
  }
}

template <class S>
__global__ void k_zero_blocks(const int32_t* __restrict__ row_ptr, int64_t nv, S* __restrict__ vals) {
  const int64_t n = 9 * (int64_t)row_ptr[nv];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    vals[i] = S(0);
}

// Numeric: the blocks J_k^T M J_l of every touched row, summed in pair-key order (the order of
// the one-call assembly, so the values are the same bit for bit) into the caller's columns.  A
// hit vertex missing from its row's columns latches TTIE_ERR_INVALID_ARGUMENT.
template <class S>
__global__ void __launch_bounds__(kBlock) k_num_rows(const int32_t* __restrict__ touched, Counters* ctr,
                                                     const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc2,
                                                     const AsmRec<S>* __restrict__ recs,
                                                     const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx, S* __restrict__ vals) {
  const int wave = threadIdx.x / 64, lane = __lane_id();
  const uint32_t U = ctr->last_touched;
  int status = 0;
  for (uint32_t u = blockIdx.x * kWaves + wave; u < U; u += gridDim.x * kWaves) {
    const int32_t v = touched[u];
    const int32_t b = off[v], n = off[v + 1] - b;
    const int32_t rp = row_ptr[v], nc = row_ptr[v + 1] - rp;
    // coverage: every vertex of every incident hit is a column of the row (binary search)
    for (int32_t t = lane; t < 6 * n; t += 64) {
      const int32_t want = recs[inc2[b + t / 6].hit].vid[t % 6];
      int32_t lo = 0, hi = nc;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col_idx[rp + mid] < want) lo = mid + 1;
        else hi = mid;
      }
      if (lo >= nc || col_idx[rp + lo] != want) status = STATUS_INVALID;
    }
    for (int32_t q0 = 0; q0 < nc; q0 += 64) {
      const int32_t q = q0 + lane;
      const int32_t col = q < nc ? col_idx[rp + q] : -1;
      S B[9];
#pragma unroll
      for (int z = 0; z < 9; ++z) B[z] = Sc<S>::c(0.0);
      for (int32_t k = 0; k < n; ++k) {
        const Incidence in = inc2[b + k];
        const AsmRec<S>& r = recs[in.hit];
        uint32_t match = 0;
#pragma unroll
        for (int l = 0; l < 6; ++l) match |= (uint32_t)(r.vid[l] == col) << l;
        while (match) {
          block_jmj(r, in.slot, __builtin_ctz(match), B);
          match &= match - 1;
        }
      }
      if (q < nc) {
#pragma unroll
        for (int z = 0; z < 9; ++z) vals[9 * ((int64_t)rp + q) + z] = B[z];
      }
    }
  }
  if (status) latch(&ctr->status, status);
}

// ------------------------------------------------------------------------------------------
// Hessian-vector products
// ------------------------------------------------------------------------------------------
template <class S>
__global__ void __launch_bounds__(kBlock) k_hvp_exact(const double* __restrict__ x, const S* __restrict__ v,
                                                      const HitGeom* __restrict__ hits, const AsmRec<S>* __restrict__ recs,
                                                      const Counters* ctr, uint32_t max_hits, double half,
                                                      S* __restrict__ hv) {
  using DS = Dual<S>;
  const uint32_t H = ctr->last_hits;
  for (uint32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < H; h += gridDim.x * blockDim.x) {
    const HitGeom g = hits[h];
    const AsmRec<S>& r = recs[h];
    V3<S> Xv[6];
    const int e = local_coords<S>(x, r.vid, Xv);
    V3<DS> X[6];
    S vv[18];
    // the coordinates are scaled by 2^-e, so their tangents along v are too; the tangents of a
    // and b (degree 0) then come out in the original units
    const S sv = Sc<S>::c(ldexp(1.0, -e));
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
      for (int c = 0; c < 3; ++c) vv[3 * k + c] = v[3 * (int64_t)r.vid[k] + c];
      X[k] = V3<DS>{DS{Xv[k].x, sv * vv[3 * k]}, DS{Xv[k].y, sv * vv[3 * k + 1]}, DS{Xv[k].z, sv * vv[3 * k + 2]}};
    }
    DS a[18], b[18];
    interval_grads<DS>(X, g.da, g.db, e, g.desc, half, a, b);
    // first-order tangents of t_c^0, t_c^1 along v
    S t0d = S(0), t1d = S(0);
#pragma unroll
    for (int k = 0; k < 18; ++k) {
      t0d = t0d + a[k].v * vv[k];
      t1d = t1d + b[k].v * vv[k];
    }
    const DS t0{Sc<S>::c(g.t0), t0d}, t1{Sc<S>::c(g.t1), t1d};
    const DS two{Sc<S>::c(2.0), S(0)};
    const DS ca = two * t0 * t1 * t1, cb = two * t1 * t0 * t0;
#pragma unroll
    for (int k = 0; k < 18; ++k) hv[18 * (int64_t)h + k] = (ca * a[k] + cb * b[k]).d;
  }
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_hvp_psd(const S* __restrict__ v, const AsmRec<S>* __restrict__ recs,
                                                    const Counters* ctr, uint32_t max_hits, S* __restrict__ hv) {
  const uint32_t H = ctr->last_hits;
  for (uint32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < H; h += gridDim.x * blockDim.x) {
    const AsmRec<S>& r = recs[h];
    S av = S(0), bv = S(0);
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const S vk = v[3 * (int64_t)r.vid[k] + c];
        av = av + r.a[3 * k + c] * vk;
        bv = bv + r.b[3 * k + c] * vk;
      }
    const S ca = r.M[0] * av + r.M[1] * bv, cb = r.M[1] * av + r.M[2] * bv;
#pragma unroll
    for (int k = 0; k < 18; ++k) hv[18 * (int64_t)h + k] = ca * r.a[k] + cb * r.b[k];
  }
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_hvp_rows(int64_t nv, const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc, const S* __restrict__ hv,
                                                     S* __restrict__ out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    S acc[3] = {S(0), S(0), S(0)};
    for (int32_t k = off[v]; k < off[v + 1]; ++k) {
      const Incidence in = inc[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = acc[c] + hv[18 * (int64_t)in.hit + 3 * in.slot + c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) out[3 * v + c] = acc[c];
  }
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_bsr_mv(int64_t n_rows, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, const S* __restrict__ vals,
                                                   const S* __restrict__ xin, S* __restrict__ y) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rows; r += (int64_t)gridDim.x * blockDim.x) {
    S acc[3] = {S(0), S(0), S(0)};
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      const int64_t c = col_idx[k];
      const S x0 = xin[3 * c], x1 = xin[3 * c + 1], x2 = xin[3 * c + 2];
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] = acc[i] + vals[9 * (int64_t)k + 3 * i] * x0 +
                                           vals[9 * (int64_t)k + 3 * i + 1] * x1 + vals[9 * (int64_t)k + 3 * i + 2] * x2;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) y[3 * r + i] = acc[i];
  }
}

// ------------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------------
static unsigned grid_for(int64_t n, unsigned cap = 4096) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_fill_zero_i32(int32_t* p, int64_t n, hipStream_t s) {
  k_fill_zero_i32<<<grid_for(n), kBlock, 0, s>>>(p, n);
  return hipGetLastError();
}

static hipError_t scan_i32(Ctx* c, const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  return launch_scan_i32(c, in, out, n, s);
}

template <class S>
static hipError_t eval_impl(Ctx* c, const ttie_mesh* m, const int32_t* pairs, const int64_t* n_pairs,
                            int64_t pair_cap, const ttie_options* o, double* energy, S* grad, uint8_t* flags,
                            double* pair_T, int32_t* row_ptr, int32_t* col_idx, S* vals, int64_t block_cap,
                            int64_t* n_blocks, int64_t* n_hits, int n_prob, const int64_t* vert_off, double* energies,
                            hipStream_t s) {
  const Layout& L = c->L;
  Counters* ctr = wsp<Counters>(c, L.counters);
  HitGeom* hits = wsp<HitGeom>(c, L.hits);
  AsmRec<S>* recs = wsp<AsmRec<S>>(c, L.recs);
  int32_t* cnt = wsp<int32_t>(c, L.cnt);
  int32_t* cur = wsp<int32_t>(c, L.cur);
  int32_t* off = wsp<int32_t>(c, L.off);
  int32_t* ncol = wsp<int32_t>(c, L.ncol);
  Incidence* inc = wsp<Incidence>(c, L.inc);
  Incidence* inc2 = wsp<Incidence>(c, L.inc2);
  int32_t* colbuf = wsp<int32_t>(c, L.colbuf);
  int32_t* cstage = wsp<int32_t>(c, L.cstage);
  int32_t* touched = wsp<int32_t>(c, L.touched);
  double* epart = wsp<double>(c, L.epart_v);
  double* blockpart = wsp<double>(c, L.epart);
  int32_t* defer = wsp<int32_t>(c, L.defer);
  const uint32_t max_hits = (uint32_t)c->lim.max_hits;
  const double half = o->interval == TTIE_INTERVAL_APPENDIX_HALF ? 0.5 : 1.0;
  const int va = (o->flags & TTIE_EVAL_VERTEX_ADJACENT) ? 1 : 0;
  const int64_t nv = m->n_verts;
  const bool bsr = row_ptr != nullptr;

  stage_begin(c, TTIE_STAGE_SCREEN, s);
  k_screen<<<grid_for(pair_cap, (unsigned)ctx_param(c, TTIE_PARAM_SCREEN_BLOCKS)), kBlock, 0, s>>>(m->x, nv, m->tris, m->n_tris, pairs, n_pairs, pair_cap, half,
                                                       va, hits, max_hits, defer, ctr, flags, pair_T);
  stage_end(c, TTIE_STAGE_SCREEN, s);
  stage_begin(c, TTIE_STAGE_SCREEN_EXACT, s);
  k_screen_exact<<<grid_for(pair_cap, 256), kBlock, 0, s>>>(m->x, nv, m->tris, m->n_tris, pairs, pair_cap, half, va,
                                                            hits, max_hits, defer, ctr, flags, pair_T);
  stage_end(c, TTIE_STAGE_SCREEN_EXACT, s);
  stage_begin(c, TTIE_STAGE_DERIVS, s);
  k_derivs<S><<<grid_for(c->lim.max_hits, 1024), kBlock, 0, s>>>(m->x, m->tris, hits, ctr, max_hits, o->psd_mode,
                                                                 half, recs, cnt, touched);
  stage_end(c, TTIE_STAGE_DERIVS, s);
  stage_begin(c, TTIE_STAGE_ASSEMBLY, s);
  hipError_t err = scan_i32(c, cnt, off, nv + 1, s);
  if (err != hipSuccess) return err;
  k_fill<S><<<grid_for(6 * c->lim.max_hits, 1024), kBlock, 0, s>>>(recs, ctr, max_hits, off, cur, inc);
  const unsigned grows = (unsigned)std::min<int64_t>(ctx_param(c, TTIE_PARAM_ROW_BLOCKS),
                                                     (6 * c->lim.max_hits + kWaves - 1) / kWaves + 1);
  k_rows_sort<S><<<grows, kBlock, 0, s>>>(touched, ctr, off, inc, inc2, recs, colbuf, cstage, 36 * c->lim.max_hits,
                                          ncol, bsr ? 1 : 0);
  if (bsr) {
    err = scan_i32(c, ncol, row_ptr, nv + 1, s);
    if (err != hipSuccess) return err;
  }
  k_rows_asm<S><<<grows, kBlock, 0, s>>>(touched, ctr, off, inc2, recs, colbuf, bsr ? row_ptr : nullptr, col_idx,
                                         vals, block_cap, grad, epart, &ctr->status);
  if (energies) k_problem_energy<<<n_prob, kBlock, 0, s>>>(nv, n_prob, vert_off, epart, energies, ctr);
  k_rows_final<S><<<kRowBlocks, kBlock, 0, s>>>(nv, m->x, cnt, cur, ncol, epart, grad, blockpart, ctr);
  k_eval_finish<<<1, kBlock, 0, s>>>(kRowBlocks, blockpart, ctr, max_hits, bsr ? row_ptr : nullptr, nv, block_cap, energy,
                                 n_blocks, n_hits);
  stage_end(c, TTIE_STAGE_ASSEMBLY, s);
  return hipGetLastError();
}

hipError_t launch_eval(Ctx* c, const ttie_mesh* m, const int32_t* pairs, const int64_t* n_pairs,
                       int64_t pair_capacity, const ttie_options* o, double* energy, void* grad, uint8_t* flags, double* pair_T,
                       int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity, int64_t* n_blocks,
                       int64_t* n_hits, int n_prob, const int64_t* vert_off, double* energies, hipStream_t s) {
  if (o->precision == TTIE_FP64)
    return eval_impl<double>(c, m, pairs, n_pairs, pair_capacity, o, energy, (double*)grad, flags, pair_T, row_ptr, col_idx,
                             (double*)vals, block_capacity, n_blocks, n_hits, n_prob, vert_off, energies, s);
  return eval_impl<float>(c, m, pairs, n_pairs, pair_capacity, o, energy, (float*)grad, flags, pair_T, row_ptr, col_idx,
                          (float*)vals, block_capacity, n_blocks, n_hits, n_prob, vert_off, energies, s);
}

template <class S>
static hipError_t bsr_symbolic_impl(Ctx* c, int32_t* row_ptr, int32_t* col_idx, int64_t cap, int64_t* n_blocks,
                                    hipStream_t s) {
  const Layout& L = c->L;
  Counters* ctr = wsp<Counters>(c, L.counters);
  const int64_t nv = c->last_nverts;
  const unsigned grows = (unsigned)std::min<int64_t>(ctx_param(c, TTIE_PARAM_ROW_BLOCKS),
                                                     (6 * c->lim.max_hits + kWaves - 1) / kWaves + 1);
  stage_begin(c, TTIE_STAGE_ASSEMBLY, s);
  k_sym_cols<S><<<grows, kBlock, 0, s>>>(wsp<int32_t>(c, L.touched), ctr, wsp<int32_t>(c, L.off),
                                         wsp<Incidence>(c, L.inc2), wsp<AsmRec<S>>(c, L.recs),
                                         wsp<int32_t>(c, L.colbuf), wsp<int32_t>(c, L.cstage),
                                         36 * c->lim.max_hits, wsp<int32_t>(c, L.ncol));
  hipError_t err = scan_i32(c, wsp<int32_t>(c, L.ncol), row_ptr, nv + 1, s);
  if (err != hipSuccess) return err;
  k_sym_write<<<grows, kBlock, 0, s>>>(wsp<int32_t>(c, L.touched), ctr, wsp<int32_t>(c, L.off),
                                       wsp<int32_t>(c, L.colbuf), row_ptr, nv, col_idx, cap, wsp<int32_t>(c, L.ncol),
                                       n_blocks);
  stage_end(c, TTIE_STAGE_ASSEMBLY, s);
  return hipGetLastError();
}

template <class S>
static hipError_t bsr_numeric_impl(Ctx* c, const int32_t* row_ptr, const int32_t* col_idx, S* vals, hipStream_t s) {
  const Layout& L = c->L;
  Counters* ctr = wsp<Counters>(c, L.counters);
  const int64_t nv = c->last_nverts;
  const unsigned grows = (unsigned)std::min<int64_t>(ctx_param(c, TTIE_PARAM_ROW_BLOCKS),
                                                     (6 * c->lim.max_hits + kWaves - 1) / kWaves + 1);
  stage_begin(c, TTIE_STAGE_ASSEMBLY, s);
  k_zero_blocks<S><<<grid_for(9 * c->lim.max_blocks, 2048), kBlock, 0, s>>>(row_ptr, nv, vals);
  k_num_rows<S><<<grows, kBlock, 0, s>>>(wsp<int32_t>(c, L.touched), ctr, wsp<int32_t>(c, L.off),
                                         wsp<Incidence>(c, L.inc2), wsp<AsmRec<S>>(c, L.recs), row_ptr, col_idx,
                                         vals);
  stage_end(c, TTIE_STAGE_ASSEMBLY, s);
  return hipGetLastError();
}

hipError_t launch_bsr_symbolic(Ctx* c, int32_t* row_ptr, int32_t* col_idx, int64_t capacity, int64_t* n_blocks,
                               hipStream_t s) {
  if (c->last_precision == TTIE_FP64) return bsr_symbolic_impl<double>(c, row_ptr, col_idx, capacity, n_blocks, s);
  return bsr_symbolic_impl<float>(c, row_ptr, col_idx, capacity, n_blocks, s);
}

hipError_t launch_bsr_numeric(Ctx* c, const int32_t* row_ptr, const int32_t* col_idx, void* vals, hipStream_t s) {
  if (c->last_precision == TTIE_FP64) return bsr_numeric_impl<double>(c, row_ptr, col_idx, (double*)vals, s);
  return bsr_numeric_impl<float>(c, row_ptr, col_idx, (float*)vals, s);
}

template <class S>
static hipError_t hvp_impl(Ctx* c, const ttie_mesh* m, const S* v, S* Hv, int mode, hipStream_t s) {
  const Layout& L = c->L;
  Counters* ctr = wsp<Counters>(c, L.counters);
  const uint32_t max_hits = (uint32_t)c->lim.max_hits;
  S* hvbuf = wsp<S>(c, L.hvbuf);
  const unsigned gh = grid_for(c->lim.max_hits, 1024);
  const double half = c->last_interval == TTIE_INTERVAL_APPENDIX_HALF ? 0.5 : 1.0;
  stage_begin(c, TTIE_STAGE_HVP, s);
  if (mode == TTIE_HVP_EXACT)
    k_hvp_exact<S><<<gh, kBlock, 0, s>>>(m->x, v, wsp<HitGeom>(c, L.hits), wsp<AsmRec<S>>(c, L.recs), ctr, max_hits,
                                         half, hvbuf);
  else
    k_hvp_psd<S><<<gh, kBlock, 0, s>>>(v, wsp<AsmRec<S>>(c, L.recs), ctr, max_hits, hvbuf);
  k_hvp_rows<S><<<grid_for(m->n_verts, 2048), kBlock, 0, s>>>(m->n_verts, wsp<int32_t>(c, L.off),
                                                               wsp<Incidence>(c, L.inc2), hvbuf, Hv);
  stage_end(c, TTIE_STAGE_HVP, s);
  return hipGetLastError();
}

hipError_t launch_hvp(Ctx* c, const ttie_mesh* m, const void* v, void* Hv, int mode, hipStream_t s) {
  if (c->last_precision == TTIE_FP64) return hvp_impl<double>(c, m, (const double*)v, (double*)Hv, mode, s);
  return hvp_impl<float>(c, m, (const float*)v, (float*)Hv, mode, s);
}

hipError_t launch_bsr_mv(int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                         const void* x, void* y, int precision, hipStream_t s) {
  if (precision == TTIE_FP64)
    k_bsr_mv<double><<<grid_for(n_rows, 4096), kBlock, 0, s>>>(n_rows, row_ptr, col_idx, (const double*)vals,
                                                               (const double*)x, (double*)y);
  else
    k_bsr_mv<float><<<grid_for(n_rows, 4096), kBlock, 0, s>>>(n_rows, row_ptr, col_idx, (const float*)vals,
                                                              (const float*)x, (float*)y);
  return hipGetLastError();
}

}  // namespace ttie
