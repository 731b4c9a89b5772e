// Evaluation kernels: screening of the candidate pairs, per-hit derivatives, and the
// deterministic (no floating-point atomics) assembly of energy, gradient and BSR Hessian.
//
// Pipeline on one stream, no host synchronization:
//   k_screen         one lane per candidate: adjacency and the FP64-filtered plane sides of both
//                    triangles; candidates that straddle both ways, and filter-uncertain ones, are
//                    appended to lists with one atomic per wave (ballot + mbcnt); checks the
//                    coordinate domain and clears the bitmap of touched vertices
//   k_screen_flag    the exact flag of the straddling candidates from their plane sides and four
//                    orientations; non-hits settled, the rest compacted in the wave's list
//   k_screen_full    the full screening of what is left (hits, in-plane pairs): segment ends,
//                    line frame, exact flag, FP64 interval ends; hits appended
//   k_screen_exact   the uncertain candidates again, with the exact fallback
//   k_derivs<S>      one lane per hit: a = dt_c^0, b = dt_c^1, T, g (Eq. 3), 2x2 Hessian core;
//                    counts the hit's six incidences and marks its vertices in the bitmap
//   k_rank           one block: per bitmap word, the touched vertices and the incidences below it
//   k_fill           scatter (pair key, hit, slot) incidences into per-vertex lists; name the rows
//   k_rank_inc<S>    one thread per incidence: its place in its row in pair-key order (the
//                    summation order); its hit's vertices as the row's column candidates
//   k_rank_cand, k_row_cols  one thread per candidate: ranked by vertex, then the distinct
//                    vertices numbered (the row's BSR columns) with their candidate runs
//   k_col_part, k_col_scan  BSR offsets of the rows from their column counts; column indices
//   k_assemble<S>    one thread per gradient entry (with the row's energy; the row's count
//                    cleared) and per BSR block J_k^T M J_l, each summed over its row's
//                    incidences in pair-key order; in the same launch, one thread per vertex
//                    for the dense outputs (BSR row pointers, zero gradient rows of untouched
//                    vertices, word counts cleared)
//   k_finish         energy summed in row order, scalar outputs, counters reset
// Everything from k_derivs to k_assemble's sums scales with the hits, not with the mesh.
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
// code: 0, or the exact plane sides of a pair that straddles both ways as the first stage found
// them (bit 12 set; bits 2k..2k+1 hold sa[k] + 1 and bits 6+2k..7+2k sb[k] + 1).
__device__ __forceinline__ uint32_t side_code(const int (&sa)[3], const int (&sb)[3]) {
  uint32_t c = 1u << 12;
#pragma unroll
  for (int k = 0; k < 3; ++k) c |= (uint32_t)(sa[k] + 1) << (2 * k) | (uint32_t)(sb[k] + 1) << (6 + 2 * k);
  return c;
}

template <bool kExact>
__device__ __forceinline__ void screen_one(int64_t p, uint32_t code, const double* __restrict__ x, int64_t nv,
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
        if (code) {
          int sa[3], sb[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            sa[k] = (int)((code >> (2 * k)) & 3u) - 1;
            sb[k] = (int)((code >> (6 + 2 * k)) & 3u) - 1;
          }
          sc = screen_pair_sides<kExact>(A, B, sa, sb, half, status);
        } else {
          sc = screen_pair<kExact>(A, B, half, status);
        }
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
// about 19% also the converse, and 0.2% intersect.  k_screen decides both plane tests for every
// candidate, one lane each, on the six vertices it loads; it is small, so many waves fit on a
// SIMD to hide the latency of those gathers.  The survivors (both triangles straddle the other's
// plane, or T_a lies in T_b's plane) are written to a list, and k_screen_full runs the full
// screening of screen_one on them, so its long tail of work is not paid by every wave for one
// or two lanes.  Every decision and value is exactly the one-pass result.
enum { STEP_SETTLED = 0, STEP_DEFER = 1, STEP_FULL = 3 };

__device__ __forceinline__ void append(bool want, int64_t p, int32_t* list, int64_t cap, uint32_t* counter,
                                       int& status) {
  const uint32_t ds = wave_slot(want, counter);
  if (want) {
    if ((int64_t)ds < cap) list[ds] = (int32_t)p;
    else status = STATUS_CAPACITY;
  }
}

__device__ __forceinline__ void settle(int64_t p, int kind, uint8_t* flags, double* pair_T) {
  if (flags) flags[p] = (uint8_t)kind;
  if (pair_T) pair_T[p] = 0.0;
}

__device__ __forceinline__ bool load_pair(int64_t p, const double* x, int64_t nv, const int32_t* tris, int64_t nt,
                                          const int32_t* pairs, int32_t vi[3], int32_t vj[3], Tri64& A, Tri64& B) {
  const int2 ij = reinterpret_cast<const int2*>(pairs)[p];
  if (ij.x < 0 || ij.y < 0 || ij.x >= nt || ij.y >= nt || ij.x == ij.y) return false;
  return load_tri(x, nv, tris, ij.x, vi, A) && load_tri(x, nv, tris, ij.y, vj, B);
}

// Status of one coordinate: finite, and 0 or of magnitude in [2^-200, 2^200] (the domain on
// which the exact predicates are exact and overflow-free), decided on the bit pattern.
__device__ __forceinline__ int coord_status(double q) {
  constexpr uint64_t kInf = 0x7ff0000000000000ull, kLo = 823ull << 52, kHi = 1223ull << 52;  // 2^-200, 2^200
  const uint64_t a = (uint64_t)__double_as_longlong(q) & 0x7fffffffffffffffull;
  if (a >= kInf) return STATUS_NONFINITE;
  return (a != 0 && (a < kLo || a > kHi)) ? STATUS_UNSUPPORTED : 0;
}

// Stage 1 (every candidate): indices, adjacency, T_a's sides against T_b's plane, then T_b's
// sides against T_a's plane.
__device__ __forceinline__ int screen_stage1(int64_t p, const double* x, int64_t nv, const int32_t* tris, int64_t nt,
                                             const int32_t* pairs, bool va, uint8_t* flags, double* pair_T,
                                             uint32_t& code, int& status) {
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
  int sa[3], sb[3];
  double d[3];
  if (!plane_sides<false>(B, A, sa, d, status)) return STEP_DEFER;
  if ((sa[0] | sa[1] | sa[2]) == 0) return STEP_FULL;  // T_a in T_b's plane: the coplanar test
  if (!make_cut(sa[0], sa[1], sa[2]).straddle) {
    settle(p, PAIR_NONE, flags, pair_T);
    return STEP_SETTLED;
  }
  if (!plane_sides<false>(A, B, sb, d, status)) return STEP_DEFER;
  if (!make_cut(sb[0], sb[1], sb[2]).straddle) {
    settle(p, PAIR_NONE, flags, pair_T);
    return STEP_SETTLED;
  }
  code = side_code(sa, sb);
  return STEP_FULL;
}

// The candidate list is split into one contiguous chunk per wave (a multiple of 64 long, the
// same split in both screening kernels).  Blocks are renumbered so that each XCD screens a
// contiguous range of the list (its L2 then sees one region of the mesh).
__device__ __forceinline__ void wave_chunk(int64_t np, int64_t& beg, int64_t& end, int64_t& wid) {
  const int64_t G = gridDim.x;
  const int64_t lb = (G % 8 == 0) ? xcd_block(blockIdx.x, G) : (int64_t)blockIdx.x;
  const int64_t nw = G * kWaves;
  const int64_t chunk = ((np + nw - 1) / nw + 63) / 64 * 64;
  wid = lb * kWaves + threadIdx.x / 64;
  beg = min(np, wid * chunk);
  end = min(np, beg + chunk);
}

// First stage over the candidate list, one lane per candidate.  A wave writes the candidates it
// passes to the full screening, with their plane sides, into its own chunk's index range of
// `full` and `fsig` (no atomics) and their number to nfull[wave].  Also clears the touched-vertex bitmap of the previous
// evaluation (read by the calls after it) before k_derivs marks this one's, and checks every
// coordinate against the exact predicates' domain (a violation is reported, never acted on: out
// of it the exact arithmetic only loses exactness, it stays within its arrays).
__global__ void __launch_bounds__(kBlock) k_screen(const double* __restrict__ x, int64_t nv,
                                                   const int32_t* __restrict__ tris, int64_t nt,
                                                   const int32_t* __restrict__ pairs, const int64_t* n_pairs_dev,
                                                   int64_t max_pairs, int va, int32_t* __restrict__ defer,
                                                   int32_t* __restrict__ full, uint16_t* __restrict__ fsig,
                                                   int32_t* __restrict__ nfull, Counters* ctr,
                                                   uint8_t* __restrict__ flags,
                                                   double* __restrict__ pair_T, uint32_t* __restrict__ bm, int64_t nbm,
                                                   int64_t tile) {
  int status = 0;
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, gs = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = gt; w < nbm; w += gs) bm[w] = 0u;
  for (int64_t c = gt; c < 3 * nv; c += gs)
    if (const int cs = coord_status(x[c])) status = status == STATUS_NONFINITE ? status : cs;
  const int64_t np = min(*n_pairs_dev, max_pairs);
  const int lane = __lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  // one unit of the list: its candidates in batches of 64, the passed ones to its range of full
  const auto unit = [&](int64_t beg, int64_t end, int64_t u) {
    int32_t nf = 0;
    for (int64_t base = beg; base < end; base += 64) {
      const int64_t p = base + lane;
      int st = STEP_SETTLED;
      uint32_t code = 0;
      if (p < end) st = screen_stage1(p, x, nv, tris, nt, pairs, va != 0, flags, pair_T, code, status);
      append(st == STEP_DEFER, p, defer, max_pairs, &ctr->n_defer, status);
      const uint64_t fm = __ballot(st == STEP_FULL);
      if (st == STEP_FULL) {
        const int64_t at = beg + nf + __popcll(fm & below);
        full[at] = (int32_t)p;
        fsig[at] = (uint16_t)code;
      }
      nf += __popcll(fm);
    }
    if (lane == 0) nfull[u] = nf;
  };
  if (tile == 0) {
    int64_t beg, end, wid;
    wave_chunk(np, beg, end, wid);
    unit(beg, end, wid);
  } else {
    // the tile queue: the next tile from the device counter until the list is done
    for (;;) {
      uint32_t t = 0;
      if (lane == 0) t = atomicAdd(&ctr->tile_next, 1u);
      t = __shfl(t, 0);
      const int64_t beg = (int64_t)t * tile;
      if (beg >= np) break;
      unit(beg, min(np, beg + tile), (int64_t)t);
    }
  }
  if (status) latch(&ctr->status, status);
}

// The exact flag of the candidates the first stage passed on with their plane sides, one lane
// each, on the four orientations only (a small kernel: more waves hide the gathers).  Pairs that
// do not intersect are settled, the ones whose signs need the exact path go to the deferred
// list, and the rest -- hits, pairs with a triangle in the other's plane and pairs with a
// vertex exactly on the other plane -- stay in the wave's list (compacted in place: a batch's
// writes land below the entries still to be read) for k_screen_full.
__global__ void __launch_bounds__(kBlock) k_screen_flag(const double* __restrict__ x, int64_t nv,
                                                        const int32_t* __restrict__ tris,
                                                        const int32_t* __restrict__ pairs,
                                                        const int64_t* n_pairs_dev, int64_t max_pairs,
                                                        int32_t* __restrict__ defer, int32_t* __restrict__ full,
                                                        uint16_t* __restrict__ fsig, int32_t* __restrict__ nfull,
                                                        Counters* ctr, uint8_t* __restrict__ flags,
                                                        double* __restrict__ pair_T, int64_t tile) {
  const int64_t np = min(*n_pairs_dev, max_pairs);
  int64_t beg, end, wid;
  wave_chunk(np, beg, end, wid);
  const int lane = __lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  int status = 0;
  // the wave's units: its chunk, or with the tile queue every nw-th tile from its own id
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  const int64_t units = tile ? (np + tile - 1) / tile : wid + 1;
  for (int64_t u = wid; u < units; u += nw) {
  if (tile) beg = u * tile;
  const int32_t nf = nfull[u];
  int32_t kept = 0;
  for (int32_t k0 = 0; k0 < nf; k0 += 64) {
    const int32_t k = k0 + lane;
    int32_t p = -1;
    uint32_t code = 0;
    int verdict = 1;  // 0 settled, 1 kept, 2 deferred
    if (k < nf) {
      p = full[beg + k];
      code = fsig[beg + k];
      int sa[3], sb[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sa[c] = (int)((code >> (2 * c)) & 3u) - 1;
        sb[c] = (int)((code >> (6 + 2 * c)) & 3u) - 1;
      }
      // a vertex exactly on the other plane (rare), or a pair without sides (a triangle in
      // the other's plane), is left to k_screen_full's general path
      if (code && sa[0] && sa[1] && sa[2] && sb[0] && sb[1] && sb[2]) {
        const LoneCut la = lone_cut(sa[0], sa[1], sa[2]), lb = lone_cut(sb[0], sb[1], sb[2]);
        const int2 ij = reinterpret_cast<const int2*>(pairs)[p];
        const int64_t ta = 3 * (int64_t)ij.x, tb = 3 * (int64_t)ij.y;
        const int32_t ia[3] = {tris[ta], tris[ta + 1], tris[ta + 2]};  // one load per row
        const int32_t ib[3] = {tris[tb], tris[tb + 1], tris[tb + 2]};
        // the six vertices in cut order, loaded straight from their ids
        const int64_t vp = pick(ia[0], ia[1], ia[2], la.k), vq0 = pick(ia[0], ia[1], ia[2], la.q0),
                      vq1 = pick(ia[0], ia[1], ia[2], la.q1);
        const int64_t vr = pick(ib[0], ib[1], ib[2], lb.k), vs0 = pick(ib[0], ib[1], ib[2], lb.q0),
                      vs1 = pick(ib[0], ib[1], ib[2], lb.q1);
        const auto ld = [x](int64_t v) { return V3<double>{x[3 * v], x[3 * v + 1], x[3 * v + 2]}; };
        const V3<double> P = ld(vp), R = ld(vr);
        const V3<double> Q[2] = {ld(vq0), ld(vq1)}, S[2] = {ld(vs0), ld(vs1)};
        const int sq[2] = {pick(sa[0], sa[1], sa[2], la.q0), pick(sa[0], sa[1], sa[2], la.q1)};
        const int ss[2] = {pick(sb[0], sb[1], sb[2], lb.q0), pick(sb[0], sb[1], sb[2], lb.q1)};
        const int xr = cuts_intersect_lone(P, Q, sq, R, S, ss);
        verdict = xr == 0 ? 0 : (xr == 2 ? 2 : 1);
        if (verdict == 0) settle(p, PAIR_NONE, flags, pair_T);
      }
    }
    append(verdict == 2, p, defer, max_pairs, &ctr->n_defer, status);
    const bool keep = k < nf && verdict == 1;
    const uint64_t km = __ballot(keep);
    if (keep) {
      const int64_t at = beg + kept + __popcll(km & below);
      full[at] = p;
      fsig[at] = (uint16_t)code;
    }
    kept += (int32_t)__popcll(km);
  }
  if (lane == 0) nfull[u] = kept;
  }
  if (status) latch(&ctr->status, status);
}

// The full screening (screen_one) of the candidates k_screen_flag kept: few per chunk (the hits,
// and pairs with a triangle in the other's plane), so each wave takes the lists of kMergeChunks
// consecutive chunks and screens them 64 at a time (a wave per chunk would pay its chain of
// dependent loads for one or two pairs).  A pair that straddles both ways comes with its exact
// plane sides, so the plane distances are computed again for a hit only.
constexpr int kMergeChunks = 16;
constexpr int64_t kMaxUnits = 65536 * kWaves;  // entries of nfull: chunks of a 65536-block grid, or tiles

__global__ void __launch_bounds__(kBlock) k_screen_full(const double* __restrict__ x, int64_t nv,
                                                        const int32_t* __restrict__ tris, int64_t nt,
                                                        const int32_t* __restrict__ pairs, const int64_t* n_pairs_dev,
                                                        int64_t max_pairs, int64_t n_chunks, int64_t tile, double half,
                                                        int va,
                                                        HitGeom* __restrict__ hits, uint32_t max_hits,
                                                        int32_t* __restrict__ defer, const int32_t* __restrict__ full,
                                                        const uint16_t* __restrict__ fsig,
                                                        const int32_t* __restrict__ nfull, Counters* ctr,
                                                        uint8_t* __restrict__ flags, double* __restrict__ pair_T) {
  const int64_t np = min(*n_pairs_dev, max_pairs);
  // the units' length and count: the tiles, or the chunks of the screening grid's n_chunks
  // waves (as wave_chunk computes them there)
  const int64_t chunk = tile ? tile : ((np + n_chunks - 1) / n_chunks + 63) / 64 * 64;
  if (tile) n_chunks = (np + tile - 1) / tile;
  const int lane = __lane_id();
  const int64_t c0 = ((int64_t)blockIdx.x * kWaves + threadIdx.x / 64) * kMergeChunks;
  int32_t cnt = 0;
  if (lane < kMergeChunks && c0 + lane < n_chunks) cnt = nfull[c0 + lane];
  // inclusive prefix of the chunk counts, then every lane holds all of them
  int32_t incl = cnt;
#pragma unroll
  for (int d = 1; d < kMergeChunks; d <<= 1) {
    const int32_t y = __shfl_up(incl, d);
    if (lane >= d) incl += y;
  }
  int32_t pre[kMergeChunks];
#pragma unroll
  for (int j = 0; j < kMergeChunks; ++j) pre[j] = __shfl(incl, j);
  const int32_t total = pre[kMergeChunks - 1];
  int status = 0;
  for (int32_t e0 = 0; e0 < total; e0 += 64) {
    const int32_t e = e0 + lane;
    int64_t p = -1;
    uint32_t code = 0;
    if (e < total) {
      // the chunk holding entry e, and e's place in its list
      int j = 0;
      int32_t below = 0;
#pragma unroll
      for (int k = 0; k < kMergeChunks - 1; ++k)
        if (e >= pre[k]) {
          j = k + 1;
          below = pre[k];
        }
      const int64_t at = min(np, (c0 + j) * chunk) + (e - below);
      p = full[at];
      code = fsig[at];
    }
    screen_one<false>(p, code, x, nv, tris, nt, pairs, half, va != 0, hits, max_hits, defer, max_pairs, ctr, flags,
                      pair_T, status);
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
    screen_one<true>(q < nd ? (int64_t)defer[q] : -1, 0u, x, nv, tris, nt, pairs, half, va != 0, hits, max_hits, nullptr,
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

// ---- rows of the touched vertices -------------------------------------------------------
// The assembly works on the vertices the hits touch, in increasing vertex order: the compact
// rows 0..R-1.  k_derivs marks each touched vertex in a bitmap (one bit per vertex) and counts
// its incidences (cnt, and per bitmap word wcnt).  One scan over the words (k_rank) then gives,
// for word w, the touched vertices below it (wp[w]) and their incidences (wi[w]), so that
//   row of touched vertex v             = wp[v/32] + popcount(word bits below v)
//   first incidence of vertex v's list  = wi[v/32] + sum of cnt over the vertices below v in its word
// Everything after the screening scales with the hits, not with N_v, except the final pass
// that writes the dense outputs (gradient rows, BSR row pointers, incidence offsets).
// The word scan (blocks of kRankBlockWords words) and the column scan (blocks of kColBlockRows
// rows) run in two launches each: the first writes each block's totals, the second adds the
// totals of the blocks below its own and scans inside the block.  (Counting into a few shared totals with atomics instead serialises on the
// contended addresses: measured 55 us for the 4M-triangle sphere's 27 K hits.)
constexpr int kRankThreads = 256;
constexpr int kRankWordsPerThread = 4;
constexpr int kRankBlockWords = kRankThreads * kRankWordsPerThread;

__device__ __forceinline__ uint32_t vrank(const uint32_t* __restrict__ bm, const uint32_t* __restrict__ wp, int64_t v) {
  const uint64_t w = (uint64_t)v >> 5;
  return wp[w] + (uint32_t)__popc(bm[w] & ((1u << (v & 31)) - 1u));
}

template <class S>
__global__ void __launch_bounds__(kBlock) k_derivs(const double* __restrict__ x, const int32_t* __restrict__ tris,
                                                   const HitGeom* __restrict__ hits, Counters* ctr, uint32_t max_hits,
                                                   int psd_mode, double half, AsmRec<S>* __restrict__ recs,
                                                   int32_t* __restrict__ cnt, uint32_t* __restrict__ wcnt,
                                                   uint32_t* __restrict__ bm, int32_t* __restrict__ incpos) {
  const uint32_t H = min(ctr->n_hits, max_hits);
  for (uint32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < H; h += gridDim.x * blockDim.x) {
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
    // the six incidences: each one's place in its vertex's list (all atomics in flight at
    // once), the per-word count, and the vertex's bit (set by its first incidence)
    int32_t vid[6], old[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) vid[k] = r.vid[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) old[k] = atomicAdd(&cnt[vid[k]], 1);
#pragma unroll
    for (int k = 0; k < 6; ++k) atomicAdd(&wcnt[(uint32_t)vid[k] >> 5], 1u);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (old[k] == 0) atomicOr(&bm[(uint32_t)vid[k] >> 5], 1u << (vid[k] & 31));
#pragma unroll
    for (int k = 0; k < 6; ++k) incpos[6 * (int64_t)h + k] = old[k];
  }
}

// Exclusive prefix sums of two per-thread values over a block of kRankThreads threads (in
// thread order); the totals come back in ta, tb.
__device__ __forceinline__ void block_scan2(uint32_t a, uint32_t b, uint32_t* sh, uint32_t& ea, uint32_t& eb,
                                            uint32_t& ta, uint32_t& tb) {
  const int lane = __lane_id(), wave = threadIdx.x / 64;
  uint32_t ia = a, ib = b;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t ya = __shfl_up(ia, d), yb = __shfl_up(ib, d);
    if (lane >= d) {
      ia += ya;
      ib += yb;
    }
  }
  if (lane == 63) {
    sh[wave] = ia;
    sh[32 + wave] = ib;
  }
  __syncthreads();
  uint32_t oa = 0, ob = 0;
  ta = 0;
  tb = 0;
#pragma unroll
  for (int k = 0; k < kRankThreads / 64; ++k) {
    const uint32_t sa = sh[k], sb = sh[32 + k];
    if (k < wave) {
      oa += sa;
      ob += sb;
    }
    ta += sa;
    tb += sb;
  }
  ea = oa + ia - a;
  eb = ob + ib - b;
}

// Sum over the block of two per-thread values (every thread gets both totals).
__device__ __forceinline__ void block_sum2(uint32_t a, uint32_t b, uint32_t* sh, uint32_t& ta, uint32_t& tb) {
  uint32_t ea, eb;
  block_scan2(a, b, sh, ea, eb, ta, tb);
}

// Loads four consecutive entries of two arrays (zero past n).
__device__ __forceinline__ void load4x2(const uint32_t* __restrict__ p, const uint32_t* __restrict__ q, int64_t i0,
                                        int64_t n, uint32_t a[4], uint32_t b[4]) {
  if (i0 + 4 <= n) {
    const uint4 x = *reinterpret_cast<const uint4*>(p + i0);
    const uint4 y = *reinterpret_cast<const uint4*>(q + i0);
    a[0] = x.x, a[1] = x.y, a[2] = x.z, a[3] = x.w;
    b[0] = y.x, b[1] = y.y, b[2] = y.z, b[3] = y.w;
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = i0 + k < n ? p[i0 + k] : 0u;
      b[k] = i0 + k < n ? q[i0 + k] : 0u;
    }
  }
}

// Per block of kRankBlockWords bitmap words: its touched vertices and incidences.
__global__ void __launch_bounds__(kRankThreads) k_rank_part(const uint32_t* __restrict__ bm,
                                                            const uint32_t* __restrict__ wcnt, int64_t nw,
                                                            uint32_t* __restrict__ part) {
  __shared__ uint32_t sh[64];
  uint32_t b[4], c[4];
  load4x2(bm, wcnt, (int64_t)blockIdx.x * kRankBlockWords + 4 * threadIdx.x, nw, b, c);
  uint32_t tb, tc;
  block_sum2(__popc(b[0]) + __popc(b[1]) + __popc(b[2]) + __popc(b[3]), c[0] + c[1] + c[2] + c[3], sh, tb, tc);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = tb;
    part[2 * blockIdx.x + 1] = tc;
  }
}

// wp[w] and wi[w] for every bitmap word (nw words, plus the totals R and the incidence count
// at index nw).  Block b scans words [b kRankBlockWords, (b + 1) kRankBlockWords), four per
// thread, from the totals of the blocks below it.
__global__ void __launch_bounds__(kRankThreads) k_rank(const uint32_t* __restrict__ bm,
                                                       const uint32_t* __restrict__ wcnt, int64_t nw,
                                                       const uint32_t* __restrict__ part, uint32_t* __restrict__ wp,
                                                       uint32_t* __restrict__ wi) {
  __shared__ uint32_t sh[64];
  uint32_t pr = 0, pi = 0;
  for (uint32_t q = threadIdx.x; q < blockIdx.x; q += kRankThreads) {
    pr += part[2 * q];
    pi += part[2 * q + 1];
  }
  uint32_t rows, incs;
  block_sum2(pr, pi, sh, rows, incs);
  __syncthreads();  // sh is reused
  const int64_t w0 = (int64_t)blockIdx.x * kRankBlockWords + 4 * threadIdx.x;
  uint32_t b[4], c[4];
  load4x2(bm, wcnt, w0, nw, b, c);
  uint32_t eb, ec, tb, tc;
  block_scan2(__popc(b[0]) + __popc(b[1]) + __popc(b[2]) + __popc(b[3]), c[0] + c[1] + c[2] + c[3], sh, eb, ec, tb,
              tc);
  uint32_t pb = rows + eb, pc = incs + ec;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (w0 + k < nw) {
      wp[w0 + k] = pb;
      wi[w0 + k] = pc;
    }
    pb += (uint32_t)__popc(b[k]);
    pc += c[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {  // the last block: the totals
    wp[nw] = rows + tb;
    wi[nw] = incs + tc;
  }
}

// First incidence of vertex v's list: the incidences of the words below v's and of the
// vertices below v in its word (one 128-byte line of cnt).
__device__ __forceinline__ uint32_t list_start(const int32_t* __restrict__ cnt, const uint32_t* __restrict__ wi,
                                               int32_t v) {
  const uint32_t w = (uint32_t)v >> 5, j = (uint32_t)v & 31u;
  const int4* line = reinterpret_cast<const int4*>(cnt + 32 * (int64_t)w);
  uint32_t below = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int4 y = line[q];
    below += (4 * q < (int)j ? (uint32_t)y.x : 0u) + (4 * q + 1 < (int)j ? (uint32_t)y.y : 0u) +
             (4 * q + 2 < (int)j ? (uint32_t)y.z : 0u) + (4 * q + 3 < (int)j ? (uint32_t)y.w : 0u);
  }
  return wi[w] + below;
}

// Scatters the incidences into per-vertex lists; an incidence that came first in its vertex
// names the vertex's row (rowv) and the row's first incidence (roff).
template <class S>
__global__ void __launch_bounds__(kBlock) k_fill(const AsmRec<S>* __restrict__ recs, const Counters* ctr,
                                                 uint32_t max_hits, const int32_t* __restrict__ incpos,
                                                 const int32_t* __restrict__ cnt, const uint32_t* __restrict__ bm,
                                                 const uint32_t* __restrict__ wp, const uint32_t* __restrict__ wi,
                                                 int64_t nw, Incidence* __restrict__ inc, int32_t* __restrict__ rowv,
                                                 int32_t* __restrict__ roff, int32_t* __restrict__ irow) {
  const uint32_t H = min(ctr->n_hits, max_hits);
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gt == 0) roff[wp[nw]] = (int32_t)wi[nw];
  for (int64_t t = gt; t < 6 * (int64_t)H; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t h = t / 6;
    const int k = (int)(t % 6);
    const int32_t v = recs[h].vid[k];
    const int32_t pos = incpos[t];
    const uint32_t start = list_start(cnt, wi, v);
    inc[start + pos] = Incidence{recs[h].key, (int32_t)h, k};
    const uint32_t r = vrank(bm, wp, v);
    irow[start + pos] = (int32_t)r;
    if (pos == 0) {
      rowv[r] = v;
      roff[r] = (int32_t)start;
    }
  }
}

constexpr int kColCap = 1024;  // column candidates of a row sorted in LDS

// Bitonic sort of s[0, p) (p a power of two, 64 <= p <= kColCap) by one wave in LDS.
__device__ __forceinline__ void wave_sort_lds(int32_t* s, int p, int lane) {
  for (int k = 2; k <= p; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < p; i += 64) {
        const int l = i ^ j;
        if (l > i) {
          const int32_t a = s[i], b = s[l];
          if ((a > b) == ((i & k) == 0)) {
            s[i] = b;
            s[l] = a;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
}

// Bitonic sort of one value per lane across the wave (ascending in lane order).
__device__ __forceinline__ int32_t wave_sort_reg(int32_t v, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int32_t o = __shfl_xor(v, j);
      const bool lower = (lane & j) == 0, up = (lane & k) == 0;
      v = (lower == up) ? min(v, o) : max(v, o);
    }
  return v;
}

// The distinct columns of one row in increasing vertex order, written to out: the six vertex
// ids of every incident hit, sorted, then the first of each run of equal ids kept.  Returns
// the count (every lane).  lds: kColCap ints of the wave's LDS; rows with more candidates
// rank every candidate against all the others in global memory (cand, flag: 6 n entries).
template <class S>
__device__ __forceinline__ int32_t row_columns(int32_t* lds, const Incidence* __restrict__ rinc, int32_t n,
                                               const AsmRec<S>* __restrict__ recs, int32_t* __restrict__ cand,
                                               uint8_t* __restrict__ flag, int32_t* __restrict__ out, int lane) {
  const int32_t m = 6 * n;
  const uint64_t below = (1ull << lane) - 1ull;
  if (m <= 64) {
    int32_t v = lane < m ? recs[rinc[lane / 6].hit].vid[lane % 6] : INT32_MAX;
    v = wave_sort_reg(v, lane);
    const int32_t prev = __shfl_up(v, 1);
    const bool keep = v != INT32_MAX && (lane == 0 || prev != v);
    const uint64_t km = __ballot(keep);
    if (keep) out[__popcll(km & below)] = v;
    return (int32_t)__popcll(km);
  }
  if (m <= kColCap) {
    int p = 128;
    while (p < m) p <<= 1;
    for (int32_t c = lane; c < p; c += 64) lds[c] = c < m ? recs[rinc[c / 6].hit].vid[c % 6] : INT32_MAX;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    wave_sort_lds(lds, p, lane);
    int32_t kept = 0;
    for (int32_t c0 = 0; c0 < m; c0 += 64) {
      const int32_t c = c0 + lane;
      const int32_t v = c < m ? lds[c] : INT32_MAX;
      const bool keep = v != INT32_MAX && (c == 0 || lds[c - 1] != v);
      const uint64_t km = __ballot(keep);
      if (keep) out[kept + __popcll(km & below)] = v;
      kept += (int32_t)__popcll(km);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the LDS is reused by the wave's next row
    return kept;
  }
  // very long rows: quadratic ranking in global memory (each candidate against all others)
  for (int32_t c = lane; c < m; c += 64) cand[c] = recs[rinc[c / 6].hit].vid[c % 6];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  for (int32_t c = lane; c < m; c += 64) {
    const int32_t val = cand[c];
    uint32_t dup = 0;
    for (int32_t j = 0; j < c; ++j) dup |= (uint32_t)(cand[j] == val);
    flag[c] = dup ? 0 : 1;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  int32_t kept = 0;
  for (int32_t c = lane; c < m; c += 64) {
    if (!flag[c]) continue;
    const int32_t val = cand[c];
    int32_t pos = 0;
    for (int32_t j = 0; j < m; ++j) pos += (int32_t)(flag[j] != 0 && cand[j] < val);
    out[pos] = val;
    ++kept;
  }
  for (int w = 32; w > 0; w >>= 1) kept += __shfl_xor(kept, w);
  return kept;
}

// The rows of the assembly, one thread per output, in three passes (a wave per row would run
// the row's chain of dependent loads once per row in turn):
//   k_rank_inc   one thread per incidence: its rank among the row's incidences by (pair key,
//                slot, position) -- the summation order, deterministic even when a hit holds the
//                vertex twice (a pair sharing one vertex) and a permutation even if a caller
//                repeats a pair -- and its place there, with its hit's six vertex ids as the
//                row's column candidates (in that order)
//   k_rank_cand  one thread per candidate: its rank among the row's candidates by (vertex,
//                candidate index), and whether it is the first of its vertex
//   k_row_cols   one thread per ranked first candidate: its number among the row's distinct
//                vertices -- the BSR columns in increasing order -- with the start of its run
//                of candidates (the incidences whose hit holds that column, in summation
//                order); the row's last candidate writes the row's column count
template <class S>
__global__ void __launch_bounds__(kBlock) k_rank_inc(const Counters* ctr, uint32_t max_hits,
                                                     const int32_t* __restrict__ irow,
                                                     const int32_t* __restrict__ roff,
                                                     const Incidence* __restrict__ inc,
                                                     const AsmRec<S>* __restrict__ recs,
                                                     Incidence* __restrict__ inc2, int32_t* __restrict__ cand) {
  const XcdItems it = xcd_items(6 * (int64_t)min(ctr->n_hits, max_hits));
  for (int64_t i = it.first; i < it.end; i += it.step) {
    const int32_t r = irow[i];
    const int32_t b = roff[r], n = roff[r + 1] - b;
    const Incidence me = inc[i];
    const int32_t self = (int32_t)(i - b);
    int32_t rank = 0;
#pragma unroll 4
    for (int32_t j = 0; j < n; ++j) {
      const Incidence o = inc[b + j];
      rank += (o.key < me.key) | ((o.key == me.key) & ((o.slot < me.slot) | ((o.slot == me.slot) & (j < self))));
    }
    inc2[b + rank] = me;
    const int32_t* vid = recs[me.hit].vid;
#pragma unroll
    for (int l = 0; l < 6; ++l) cand[6 * (int64_t)(b + rank) + l] = vid[l];
  }
}

__global__ void __launch_bounds__(kBlock) k_rank_cand(const Counters* ctr, uint32_t max_hits,
                                                      const int32_t* __restrict__ irow,
                                                      const int32_t* __restrict__ roff,
                                                      const Incidence* __restrict__ inc2,
                                                      const int32_t* __restrict__ cand, uint32_t* __restrict__ csort,
                                                      int32_t* __restrict__ cval, uint8_t* __restrict__ cflag) {
  const XcdItems it = xcd_items(36 * (int64_t)min(ctr->n_hits, max_hits));
  for (int64_t c = it.first; c < it.end; c += it.step) {
    const int64_t i = c / 6;
    const int32_t r = irow[i];
    const int32_t b = roff[r], m = 6 * (roff[r + 1] - b);
    const int64_t base = 6 * (int64_t)b;
    const int32_t self = (int32_t)(c - base);
    const int32_t v = cand[c];
    int32_t pos = 0;
    bool first = true;
#pragma unroll 4
    for (int32_t j = 0; j < m; ++j) {
      const int32_t w = cand[base + j];
      const bool dup = (w == v) & (j < self);
      pos += (int32_t)((w < v) | dup);
      first &= !dup;
    }
    const Incidence I = inc2[i];
    csort[base + pos] = ((uint32_t)I.hit << 6) | ((uint32_t)I.slot << 3) | (uint32_t)(c % 6);
    cval[base + pos] = v;
    cflag[base + pos] = first ? 1 : 0;
  }
}

__global__ void __launch_bounds__(kBlock) k_row_cols(const Counters* ctr, uint32_t max_hits,
                                                     const int32_t* __restrict__ irow,
                                                     const int32_t* __restrict__ roff,
                                                     const int32_t* __restrict__ cval,
                                                     const uint8_t* __restrict__ cflag, int32_t* __restrict__ colbuf,
                                                     int32_t* __restrict__ colrun, int32_t* __restrict__ ncol) {
  const XcdItems it = xcd_items(36 * (int64_t)min(ctr->n_hits, max_hits));
  for (int64_t e = it.first; e < it.end; e += it.step) {
    const int32_t r = irow[e / 6];
    const int32_t b = roff[r], m = 6 * (roff[r + 1] - b);
    const int64_t base = 6 * (int64_t)b;
    const int32_t pos = (int32_t)(e - base);
    const int32_t f = cflag[e];
    const bool last = pos == m - 1;
    if (!f && !last) continue;
    // the first-flags below pos (each byte 0 or 1): bytes up to a 4-byte boundary, then whole
    // words (the popcount of a word is its number of 1-bytes), then the last bytes
    int32_t d = 0;
    int64_t j = base;
    const int64_t stop = base + pos;
    for (; j < stop && (j & 3); ++j) d += cflag[j];
    const uint32_t* w = reinterpret_cast<const uint32_t*>(cflag + j);
    const int64_t nwd = (stop - j) >> 2;
#pragma unroll 4
    for (int64_t q = 0; q < nwd; ++q) d += __popc(w[q]);
    for (j += 4 * nwd; j < stop; ++j) d += cflag[j];
    if (f) {
      colbuf[base + d] = cval[e];
      colrun[base + d] = pos;
    }
    if (last) ncol[r] = d + f;
  }
}

// The column scan runs in blocks of kColBlockRows rows, one row per thread (a row's block
// indices or column indices are written by its thread, so more blocks write them side by side).
constexpr int kColBlockRows = kRankThreads;

// Per block of kColBlockRows rows: its BSR columns (R = wp[nw] rows in all).
__global__ void __launch_bounds__(kRankThreads) k_col_part(const uint32_t* __restrict__ wp, int64_t nw,
                                                           const int32_t* __restrict__ ncol, uint32_t* __restrict__ part) {
  __shared__ uint32_t sh[64];
  const uint32_t R = wp[nw];
  const int64_t r0 = (int64_t)blockIdx.x * kColBlockRows;
  if (r0 > R) return;
  const int64_t i = r0 + threadIdx.x;
  const uint32_t a = i < R ? (uint32_t)ncol[i] : 0u;
  uint32_t t, unused;
  block_sum2(a, 0u, sh, t, unused);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Exclusive scan of ncol[0, R) into coff[0, R] (R = wp[nw]): block b takes rows
// [b kColBlockRows, (b + 1) kColBlockRows), one per thread, from the totals of the blocks below
// it.  With brow, each block's row goes to brow; with col_idx, each row's column indices to
// col_idx.  The total coff[R] also goes to *n_blocks, and past cap latches TTIE_ERR_CAPACITY.
__global__ void __launch_bounds__(kRankThreads) k_col_scan(const uint32_t* __restrict__ wp, int64_t nw,
                                                           const int32_t* __restrict__ ncol,
                                                           const uint32_t* __restrict__ part, int32_t* __restrict__ coff,
                                                           const int32_t* __restrict__ roff,
                                                           const int32_t* __restrict__ colbuf,
                                                           int32_t* __restrict__ col_idx, int32_t* __restrict__ brow,
                                                           int64_t cap, int64_t* n_blocks, Counters* ctr) {
  __shared__ uint32_t sh[64];
  const uint32_t R = wp[nw];
  const int64_t r0 = (int64_t)blockIdx.x * kColBlockRows;
  if (r0 > R) return;
  uint32_t pr = 0;
  for (uint32_t q = threadIdx.x; q < blockIdx.x; q += kRankThreads) pr += part[q];
  uint32_t base, unused;
  block_sum2(pr, 0u, sh, base, unused);
  __syncthreads();  // sh is reused
  const int64_t i = r0 + threadIdx.x;
  const uint32_t v = i < R ? (uint32_t)ncol[i] : 0u;
  uint32_t e, e2, t, t2;
  block_scan2(v, 0u, sh, e, e2, t, t2);
  const uint32_t p = base + e;
  if (i < R) {
    coff[i] = (int32_t)p;
    // the row of each of its blocks (stores only), or the row's column indices
    if (brow)
      for (uint32_t q = 0; q < v && (int64_t)(p + q) < cap; ++q) brow[p + q] = (int32_t)i;
    if (col_idx) {
      const int32_t* cb = colbuf + 6 * (int64_t)roff[i];
      for (uint32_t q = 0; q < v && (int64_t)(p + q) < cap; ++q) col_idx[p + q] = cb[q];
    }
  }
  if (r0 + kColBlockRows > R && threadIdx.x == 0) {  // the block holding row R: the total
    const uint32_t total = base + t;
    coff[R] = (int32_t)total;
    if (n_blocks) *n_blocks = total;
    if ((int64_t)total > cap) latch(&ctr->status, STATUS_CAPACITY);
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

// The sums of the assembly, one thread per output: the 3 R gradient entries (with each row's
// energy: the hits the vertex owns, each counted at its first vertex), then -- when the BSR is
// wanted -- one per block.  A gradient sum runs over the row's incidences in pair-key order
// (inc2), a block's over its column's run of ranked candidates (the same order), kChunk at a
// time with the chunk's loads issued together.  Nothing depends on another thread, so all of
// them are in flight at once and the kernel costs about one chain of dependent loads.
// The blocks from `ablocks` on write the dense outputs meanwhile, one thread per vertex v in
// [0, nv] (a wave's stores are contiguous): the BSR row pointer row_ptr[v] = coff[row of v]
// and the zero gradient row of an untouched vertex; they also clear the per-word counts for
// the next evaluation (the row threads clear the per-vertex ones, which only rows hold).  These
// stores stream at HBM speed while the sums wait on their loads.
constexpr int kChunk = 4;

template <class S>
__global__ void __launch_bounds__(kBlock) k_assemble(const uint32_t* __restrict__ wp, int64_t nw,
                                                     const int32_t* __restrict__ rowv, const int32_t* __restrict__ roff,
                                                     const Incidence* __restrict__ inc2,
                                                     const AsmRec<S>* __restrict__ recs,
                                                     const int32_t* __restrict__ coff, const int32_t* __restrict__ brow,
                                                     const int32_t* __restrict__ colbuf,
                                                     const int32_t* __restrict__ colrun,
                                                     const uint32_t* __restrict__ csort, int32_t* __restrict__ col_idx,
                                                     S* __restrict__ vals, int64_t block_cap, S* __restrict__ grad,
                                                     double* __restrict__ erow, int32_t* __restrict__ cnt,
                                                     int64_t ablocks, int64_t nv, const uint32_t* __restrict__ bm,
                                                     uint32_t* __restrict__ wcnt, int32_t* __restrict__ row_ptr) {
  if ((int64_t)blockIdx.x >= ablocks) {
    const int64_t v = ((int64_t)blockIdx.x - ablocks) * blockDim.x + threadIdx.x;
    if (v > nv) return;
    const int64_t w = v >> 5;
    const uint32_t word = bm[w];
    const uint32_t j = (uint32_t)v & 31u;
    if (row_ptr) row_ptr[v] = coff[wp[w] + (uint32_t)__popc(word & ((1u << j) - 1u))];
    if (j == 0 && w < nw) wcnt[w] = 0u;
    if (v < nv && !((word >> j) & 1u)) {
#pragma unroll
      for (int k = 0; k < 3; ++k) grad[3 * v + k] = Sc<S>::c(0.0);
    }
    return;
  }
  const uint32_t R = wp[nw];
  const int64_t nb = coff ? min((int64_t)coff[R], block_cap) : 0;
  const int64_t ng = 3 * (int64_t)R;
  const XcdItems it = xcd_items(ng + nb, ablocks);
  for (int64_t t = it.first; t < it.end; t += it.step) {
    if (t < ng) {
      const int64_t r = t / 3;
      const int c = (int)(t % 3);
      const int32_t b = roff[r], n = roff[r + 1] - b;
      S acc = Sc<S>::c(0.0);
      double e = 0.0;
      for (int32_t k0 = 0; k0 < n; k0 += kChunk) {
        Incidence I[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
          if (k0 + k < n) I[k] = inc2[b + k0 + k];
        S gv[kChunk];
        double Tv[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
          if (k0 + k < n) {
            gv[k] = recs[I[k].hit].g[3 * I[k].slot + c];
            Tv[k] = recs[I[k].hit].T;
          }
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
          if (k0 + k < n) {
            acc = acc + gv[k];
            if (I[k].slot == 0) e += Tv[k];
          }
      }
      const int32_t v = rowv[r];
      grad[3 * (int64_t)v + c] = acc;
      if (c == 0) {
        erow[r] = e;
        cnt[v] = 0;  // the row's incidence count, zero again for the next evaluation
      }
    } else {
      const int64_t q = t - ng;
      const int32_t r = brow[q];
      const int32_t b = roff[r], n = roff[r + 1] - b;
      const int32_t c0 = coff[r], d = (int32_t)(q - c0), nc = coff[r + 1] - c0;
      const int64_t base = 6 * (int64_t)b;
      col_idx[q] = colbuf[base + d];
      // the column's run of ranked candidates: (hit, row slot, column slot) in summation order
      const int32_t e0 = colrun[base + d], e1 = d + 1 < nc ? colrun[base + d + 1] : 6 * n;
      S B[9];
#pragma unroll
      for (int z = 0; z < 9; ++z) B[z] = Sc<S>::c(0.0);
      for (int32_t e = e0; e < e1; e += kChunk) {
        uint32_t pk[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) pk[k] = e + k < e1 ? csort[base + e + k] : 0u;
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
          if (e + k < e1) block_jmj(recs[pk[k] >> 6], (int)((pk[k] >> 3) & 7u), (int)(pk[k] & 7u), B);
      }
#pragma unroll
      for (int z = 0; z < 9; ++z) vals[9 * q + z] = B[z];
    }
  }
}

// Sum of a[r] over r = r0 + threadIdx.x + k * kThreads < r1 (kThreads the block size), added in
// increasing r; sixteen loads are in flight at a time (the adds of zero past the end leave the sum unchanged, the terms
// being non-negative).
template <int kThreads = kBlock>
__device__ __forceinline__ double strided_sum(const double* __restrict__ a, uint32_t r0, uint32_t r1) {
  double acc = 0.0;
  for (uint32_t base = r0 + threadIdx.x; base < r1; base += 16 * kThreads) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t r = base + k * kThreads;
      v[k] = r < r1 ? a[r] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += v[k];
  }
  return acc;
}

// Energy of each problem of a batch: block p sums the energies of the rows of its vertex range
// in a fixed order (thread-strided, then a tree).
__global__ void __launch_bounds__(kBlock) k_problem_energy(int64_t nv, int n_prob, const int64_t* __restrict__ vert_off,
                                                           const uint32_t* __restrict__ bm,
                                                           const uint32_t* __restrict__ wp,
                                                           const double* __restrict__ erow, double* __restrict__ energies,
                                                           Counters* ctr) {
  __shared__ double red[kBlock];
  const int p = blockIdx.x;
  int64_t b = vert_off[p], e = vert_off[p + 1];
  if (threadIdx.x == 0 && (b > e || b < 0 || e > nv || (p == 0 && b != 0) || (p == n_prob - 1 && e != nv)))
    latch(&ctr->status, STATUS_INVALID);
  b = max((int64_t)0, min(b, nv));
  e = max(b, min(e, nv));
  const uint32_t r0 = vrank(bm, wp, b), r1 = vrank(bm, wp, e);
  const double acc = strided_sum(erow, r0, r1);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) energies[p] = red[0];
}

// The end of an evaluation, one block of kFinishThreads: the row energies summed in row order
// (thread-strided, then a tree), the scalar outputs, and the counters reset for the next call.
constexpr int kFinishThreads = 1024;
__global__ void __launch_bounds__(kFinishThreads) k_finish(int64_t nw, const uint32_t* __restrict__ wp,
                                                           const double* __restrict__ erow, Counters* ctr,
                                                           uint32_t max_hits, double* energy, int64_t* n_hits,
                                                           int32_t* status_out) {
  __shared__ double red[kFinishThreads];
  const uint32_t R = wp[nw];
  red[threadIdx.x] = strided_sum<kFinishThreads>(erow, 0, R);
  __syncthreads();
  for (int w = kFinishThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  *energy = red[0];
  const uint32_t H = ctr->n_hits;
  if (n_hits) *n_hits = (int64_t)H;
  if (H > max_hits) latch(&ctr->status, STATUS_CAPACITY);
  ctr->last_hits = min(H, max_hits);
  ctr->last_touched = R;
  ctr->n_hits = 0;
  ctr->n_defer = 0;
  ctr->tile_next = 0;
  // every other kernel of the evaluation has finished, so the latched status is final
  if (status_out) *status_out = __hip_atomic_load(&ctr->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------------------------------
// The BSR Hessian of the last evaluation as two calls: the pattern (symbolic) and the values
// on a caller's pattern (numeric), from the hit records and the sorted incidence lists the
// evaluation leaves in the workspace.
// ------------------------------------------------------------------------------------------
// Symbolic, first pass: the distinct columns of every touched row (by a wave per row) and
// their count.
template <class S>
__global__ void __launch_bounds__(kBlock) k_sym_cols(const Counters* ctr, const int32_t* __restrict__ roff,
                                                     const Incidence* __restrict__ inc2,
                                                     const AsmRec<S>* __restrict__ recs, int32_t* __restrict__ colbuf,
                                                     int32_t* __restrict__ cstage, int64_t cstage_len,
                                                     int32_t* __restrict__ ncol) {
  __shared__ int32_t lcol[kWaves][kColCap];
  const int wave = threadIdx.x / 64, lane = __lane_id();
  const uint32_t U = ctr->last_touched;
  for (uint32_t u = blockIdx.x * kWaves + wave; u < U; u += gridDim.x * kWaves) {
    const int32_t b = roff[u], n = roff[u + 1] - b;
    const int32_t kept = row_columns(lcol[wave], inc2 + b, n, recs, cstage + 6 * (int64_t)b,
                                     reinterpret_cast<uint8_t*>(cstage + cstage_len) + 6 * (int64_t)b,
                                     colbuf + 6 * (int64_t)b, lane);
    if (lane == 0) ncol[u] = kept;
  }
}

// Symbolic, last pass: the dense row pointers row_ptr[v] = coff[row of v], v in [0, nv].
__global__ void __launch_bounds__(kBlock) k_rowptr_fill(int64_t nv, const uint32_t* __restrict__ bm,
                                                        const uint32_t* __restrict__ wp,
                                                        const int32_t* __restrict__ coff, int32_t* __restrict__ row_ptr) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= nv; v += (int64_t)gridDim.x * blockDim.x)
    row_ptr[v] = coff[vrank(bm, wp, v)];
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
__global__ void __launch_bounds__(kBlock) k_num_rows(const int32_t* __restrict__ rowv, Counters* ctr,
                                                     const int32_t* __restrict__ roff,
                                                     const Incidence* __restrict__ inc2,
                                                     const AsmRec<S>* __restrict__ recs,
                                                     const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx, S* __restrict__ vals) {
  const int wave = threadIdx.x / 64, lane = __lane_id();
  const uint32_t U = ctr->last_touched;
  int status = 0;
  for (uint32_t u = blockIdx.x * kWaves + wave; u < U; u += gridDim.x * kWaves) {
    const int32_t v = rowv[u];
    const int32_t b = roff[u], n = roff[u + 1] - b;
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
__global__ void __launch_bounds__(kBlock) k_hvp_rows(int64_t nv, const uint32_t* __restrict__ bm,
                                                     const uint32_t* __restrict__ wp, const int32_t* __restrict__ roff,
                                                     const Incidence* __restrict__ inc, const S* __restrict__ hv,
                                                     S* __restrict__ out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    S acc[3] = {S(0), S(0), S(0)};
    // the vertex's incidences: its row's range of the summation-ordered list (none when the
    // last evaluation's hits do not touch it)
    const uint64_t w = (uint64_t)v >> 5;
    const uint32_t word = bm[w];
    int32_t k0 = 0, k1 = 0;
    if ((word >> (v & 31)) & 1u) {
      const uint32_t r = wp[w] + (uint32_t)__popc(word & ((1u << (v & 31)) - 1u));
      k0 = roff[r];
      k1 = roff[r + 1];
    }
    for (int32_t k = k0; k < k1; ++k) {
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

// rows of the touched vertices: the bitmap words (one more than needed, so that the row of v
// is defined for every v in [0, nv])
static int64_t bitmap_words(int64_t nv) { return nv / 32 + 1; }
static unsigned col_scan_blocks(const Ctx* c) {
  return (unsigned)((6 * c->lim.max_hits + 1 + kColBlockRows - 1) / kColBlockRows);
}

template <class S>
static hipError_t eval_impl(Ctx* c, const ttie_mesh* m, const int32_t* pairs, const int64_t* n_pairs,
                            int64_t pair_cap, const ttie_options* o, double* energy, S* grad, uint8_t* flags,
                            double* pair_T, int32_t* row_ptr, int32_t* col_idx, S* vals, int64_t block_cap,
                            int64_t* n_blocks, int64_t* n_hits, int n_prob, const int64_t* vert_off, double* energies,
                            int32_t* status_out, hipStream_t s) {
  const Layout& L = c->L;
  Counters* ctr = wsp<Counters>(c, L.counters);
  HitGeom* hits = wsp<HitGeom>(c, L.hits);
  AsmRec<S>* recs = wsp<AsmRec<S>>(c, L.recs);
  int32_t* cnt = wsp<int32_t>(c, L.cnt);
  uint32_t* wcnt = wsp<uint32_t>(c, L.wcnt);
  uint32_t* bm = wsp<uint32_t>(c, L.bm);
  uint32_t* wp = wsp<uint32_t>(c, L.wp);
  uint32_t* wi = wsp<uint32_t>(c, L.wi);
  int32_t* incpos = wsp<int32_t>(c, L.incpos);
  int32_t* rowv = wsp<int32_t>(c, L.touched);
  int32_t* roff = wsp<int32_t>(c, L.roff);
  int32_t* coff = wsp<int32_t>(c, L.coff);
  int32_t* ncol = wsp<int32_t>(c, L.ncol);
  Incidence* inc = wsp<Incidence>(c, L.inc);
  Incidence* inc2 = wsp<Incidence>(c, L.inc2);
  int32_t* colbuf = wsp<int32_t>(c, L.colbuf);
  int32_t* cstage = wsp<int32_t>(c, L.cstage);
  double* erow = wsp<double>(c, L.erow);
  uint32_t* part = wsp<uint32_t>(c, L.part);
  int32_t* defer = wsp<int32_t>(c, L.defer);
  int32_t* full = wsp<int32_t>(c, L.full);
  int32_t* nfull = wsp<int32_t>(c, L.nfull);
  int32_t* brow = wsp<int32_t>(c, L.brow);
  const uint32_t max_hits = (uint32_t)c->lim.max_hits;
  const double half = o->interval == TTIE_INTERVAL_APPENDIX_HALF ? 0.5 : 1.0;
  const int va = (o->flags & TTIE_EVAL_VERTEX_ADJACENT) ? 1 : 0;
  const int64_t nv = m->n_verts;
  const int64_t nw = bitmap_words(nv);
  const bool bsr = row_ptr != nullptr;

  stage_begin(c, TTIE_STAGE_SCREEN, s);
  // both screening kernels split the list the same way: the same grid
  const unsigned gscreen = grid_for(pair_cap, (unsigned)ctx_param(c, TTIE_PARAM_SCREEN_BLOCKS));
  uint16_t* fsig = wsp<uint16_t>(c, L.fsig);
  // the screening's units: one chunk per wave, or tiles from a queue (at most kMaxUnits of
  // them, the length of nfull)
  int64_t tile = ctx_param(c, TTIE_PARAM_SCREEN_TILE);
  if (tile) tile = std::max<int64_t>(tile, ((pair_cap + kMaxUnits - 1) / kMaxUnits + 63) / 64 * 64);
  k_screen<<<gscreen, kBlock, 0, s>>>(m->x, nv, m->tris, m->n_tris, pairs, n_pairs, pair_cap, va, defer, full, fsig,
                                      nfull, ctr, flags, pair_T, bm, nw, tile);
  k_screen_flag<<<gscreen, kBlock, 0, s>>>(m->x, nv, m->tris, pairs, n_pairs, pair_cap, defer, full, fsig, nfull, ctr,
                                           flags, pair_T, tile);
  const int64_t n_chunks = (int64_t)gscreen * kWaves;
  const int64_t max_units = tile ? (pair_cap + tile - 1) / tile : n_chunks;
  k_screen_full<<<(unsigned)std::max<int64_t>(1, (max_units + kWaves * kMergeChunks - 1) / (kWaves * kMergeChunks)),
                  kBlock, 0, s>>>(m->x, nv, m->tris, m->n_tris, pairs, n_pairs, pair_cap, n_chunks, tile, half, va,
                                  hits, max_hits, defer, full, fsig, nfull, ctr, flags, pair_T);
  stage_end(c, TTIE_STAGE_SCREEN, s);
  stage_begin(c, TTIE_STAGE_SCREEN_EXACT, s);
  k_screen_exact<<<grid_for(pair_cap, 256), kBlock, 0, s>>>(m->x, nv, m->tris, m->n_tris, pairs, pair_cap, half, va,
                                                            hits, max_hits, defer, ctr, flags, pair_T);
  stage_end(c, TTIE_STAGE_SCREEN_EXACT, s);
  stage_begin(c, TTIE_STAGE_DERIVS, s);
  // one wave per block, so the few waves of a small hit count spread over every CU
  k_derivs<S><<<(unsigned)std::min<int64_t>((c->lim.max_hits + 63) / 64, 4096), 64, 0, s>>>(
      m->x, m->tris, hits, ctr, max_hits, o->psd_mode, half, recs, cnt, wcnt, bm, incpos);
  stage_end(c, TTIE_STAGE_DERIVS, s);
  stage_begin(c, TTIE_STAGE_ASSEMBLY, s);
  const unsigned rank_blocks = (unsigned)((nw + kRankBlockWords - 1) / kRankBlockWords);
  k_rank_part<<<rank_blocks, kRankThreads, 0, s>>>(bm, wcnt, nw, part);
  k_rank<<<rank_blocks, kRankThreads, 0, s>>>(bm, wcnt, nw, part, wp, wi);
  int32_t* irow = wsp<int32_t>(c, L.irow);
  uint32_t* csort = wsp<uint32_t>(c, L.csort);
  int32_t* cval = wsp<int32_t>(c, L.cval);
  int32_t* colrun = wsp<int32_t>(c, L.colrun);
  uint8_t* cflag = reinterpret_cast<uint8_t*>(cstage + 36 * c->lim.max_hits);
  k_fill<S><<<grid_for(6 * c->lim.max_hits, 1024), kBlock, 0, s>>>(recs, ctr, max_hits, incpos, cnt, bm, wp, wi, nw,
                                                                   inc, rowv, roff, irow);
  k_rank_inc<S><<<grid_for(6 * c->lim.max_hits, 4096), kBlock, 0, s>>>(ctr, max_hits, irow, roff, inc, recs, inc2,
                                                                       cstage);
  if (bsr) {
    k_rank_cand<<<grid_for(36 * c->lim.max_hits, 4096), kBlock, 0, s>>>(ctr, max_hits, irow, roff, inc2, cstage, csort,
                                                                        cval, cflag);
    k_row_cols<<<grid_for(36 * c->lim.max_hits, 4096), kBlock, 0, s>>>(ctr, max_hits, irow, roff, cval, cflag, colbuf,
                                                                       colrun, ncol);
    k_col_part<<<col_scan_blocks(c), kRankThreads, 0, s>>>(wp, nw, ncol, part);
    k_col_scan<<<col_scan_blocks(c), kRankThreads, 0, s>>>(wp, nw, ncol, part, coff, roff, colbuf, nullptr, brow,
                                                           block_cap, n_blocks, ctr);
  }
  // the sums' blocks, then one block per kBlock vertices of the dense outputs
  const unsigned ablocks = grid_for(3 * 6 * c->lim.max_hits + (bsr ? block_cap : 0), 4096);
  k_assemble<S><<<ablocks + (unsigned)((nv + kBlock) / kBlock), kBlock, 0, s>>>(
      wp, nw, rowv, roff, inc2, recs, bsr ? coff : nullptr, brow, colbuf, colrun, csort, col_idx, vals, block_cap, grad,
      erow, cnt, ablocks, nv, bm, wcnt, bsr ? row_ptr : nullptr);
  if (energies) k_problem_energy<<<n_prob, kBlock, 0, s>>>(nv, n_prob, vert_off, bm, wp, erow, energies, ctr);
  k_finish<<<1, kFinishThreads, 0, s>>>(nw, wp, erow, ctr, max_hits, energy, n_hits, status_out);
  stage_end(c, TTIE_STAGE_ASSEMBLY, s);
  return hipGetLastError();
}

hipError_t launch_eval(Ctx* c, const ttie_mesh* m, const int32_t* pairs, const int64_t* n_pairs,
                       int64_t pair_capacity, const ttie_options* o, double* energy, void* grad, uint8_t* flags, double* pair_T,
                       int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity, int64_t* n_blocks,
                       int64_t* n_hits, int n_prob, const int64_t* vert_off, double* energies, int32_t* status_out,
                       hipStream_t s) {
  if (o->precision == TTIE_FP64)
    return eval_impl<double>(c, m, pairs, n_pairs, pair_capacity, o, energy, (double*)grad, flags, pair_T, row_ptr, col_idx,
                             (double*)vals, block_capacity, n_blocks, n_hits, n_prob, vert_off, energies, status_out, s);
  return eval_impl<float>(c, m, pairs, n_pairs, pair_capacity, o, energy, (float*)grad, flags, pair_T, row_ptr, col_idx,
                          (float*)vals, block_capacity, n_blocks, n_hits, n_prob, vert_off, energies, status_out, s);
}

template <class S>
static hipError_t bsr_symbolic_impl(Ctx* c, int32_t* row_ptr, int32_t* col_idx, int64_t cap, int64_t* n_blocks,
                                    hipStream_t s) {
  const Layout& L = c->L;
  Counters* ctr = wsp<Counters>(c, L.counters);
  const int64_t nv = c->last_nverts;
  const int64_t nw = bitmap_words(nv);
  const unsigned grows = (unsigned)std::min<int64_t>(ctx_param(c, TTIE_PARAM_ROW_BLOCKS),
                                                     (6 * c->lim.max_hits + kWaves - 1) / kWaves + 1);
  int32_t* coff = wsp<int32_t>(c, L.coff);
  stage_begin(c, TTIE_STAGE_ASSEMBLY, s);
  k_sym_cols<S><<<grows, kBlock, 0, s>>>(ctr, wsp<int32_t>(c, L.roff), wsp<Incidence>(c, L.inc2),
                                         wsp<AsmRec<S>>(c, L.recs), wsp<int32_t>(c, L.colbuf),
                                         wsp<int32_t>(c, L.cstage), 36 * c->lim.max_hits, wsp<int32_t>(c, L.ncol));
  k_col_part<<<col_scan_blocks(c), kRankThreads, 0, s>>>(wsp<uint32_t>(c, L.wp), nw, wsp<int32_t>(c, L.ncol),
                                                         wsp<uint32_t>(c, L.part));
  k_col_scan<<<col_scan_blocks(c), kRankThreads, 0, s>>>(wsp<uint32_t>(c, L.wp), nw, wsp<int32_t>(c, L.ncol),
                                                         wsp<uint32_t>(c, L.part), coff, wsp<int32_t>(c, L.roff),
                                                         wsp<int32_t>(c, L.colbuf), col_idx, nullptr, cap, n_blocks,
                                                         ctr);
  k_rowptr_fill<<<grid_for(nv + 1, 2048), kBlock, 0, s>>>(nv, wsp<uint32_t>(c, L.bm), wsp<uint32_t>(c, L.wp), coff,
                                                          row_ptr);
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
  k_num_rows<S><<<grows, kBlock, 0, s>>>(wsp<int32_t>(c, L.touched), ctr, wsp<int32_t>(c, L.roff),
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
  k_hvp_rows<S><<<grid_for(m->n_verts, 2048), kBlock, 0, s>>>(m->n_verts, wsp<uint32_t>(c, L.bm),
                                                               wsp<uint32_t>(c, L.wp), wsp<int32_t>(c, L.roff),
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
