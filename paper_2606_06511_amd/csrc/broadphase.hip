// Broad phase: candidate triangle pairs for the per-pair energy (Sec. 1.2 removes redundant
// pair tests with a spatial structure; this is a linear BVH over Morton-sorted triangles).
//
//   k_bp_init      reset the pair counter
//   k_tri_boxes    exact FP64 bounding box per triangle (optionally swept to a second position);
//                  per-block bounds of the box centres
//                  (order-preserving integer keys)
//   k_morton       reduce those bounds, then a 30-bit Morton code per box centre; counts of
//                  the top bits (about two triangles per bucket), each triangle taking its
//                  rank inside its bucket from the counting atomic
//   scan, scatter  counting sort of the triangles by bucket (order inside a bucket arbitrary)
//   k_levels       an implicit complete 4-ary tree over the sorted leaves: node (l, k) covers
//                  leaves [k 4^l, (k+1) 4^l); boxes are reduced level by level in LDS, four
//                  levels per launch from the leaves, five per launch above, so building needs
//                  no atomics and no fences.  The first launch also writes the sorted leaf
//                  records (FP64 box, vertex ids).  Each inner node also records a vertex
//                  all its triangles hold, if there is one.
//   k_traverse     two lanes per leaf s (its own 256-leaf subtree, staged in LDS, and the rest
//                  of the tree), depth first over the subtrees holding leaves after s,
//                  four child boxes per visit and a 64-bit mask stack, descending where the
//                  FP32 boxes (rounded outwards) overlap, so every unordered pair is reported
//                  once; a leaf is confirmed by the exact closed FP64 box test and the
//                  shared-vertex test; pairs are staged per wave in LDS (ballot + mbcnt) and
//                  flushed with one atomic per full buffer
//   k_traverse_heavy  the searches k_traverse deferred, a wave's lanes sharing one stack of
//                  nodes; a subtree whose triangles all hold a vertex of the query is skipped
//   k_brute        all i < j without a shared vertex (no box test)

#include "internal.h"

namespace ttie {

constexpr int kBpBlock = 256;
constexpr int kBoundsBlocks = 512;  // partial-bounds slots in the workspace

__device__ __forceinline__ uint32_t f2key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// zeroes the caller's pair count and the broad phase's counters (the LBVH and the hash do it in
// k_tri_boxes instead, saving a launch)
__global__ void k_bp_init(Counters* c, unsigned long long* npairs) {
  if (threadIdx.x == 0) {
    *npairs = 0;
    c->n_entries = 0;
    c->n_heavy = 0;
  }
}

__global__ void __launch_bounds__(kBpBlock) k_tri_boxes(const double* __restrict__ x, const double* __restrict__ x_end,
                                                        int64_t nv, const int32_t* __restrict__ tris, int64_t nt,
                                                        double* __restrict__ tbox, float* __restrict__ centre,
                                                        uint32_t* __restrict__ part, double* __restrict__ ext_part,
                                                        unsigned long long* npairs, Counters* ctr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *npairs = 0;
    ctr->n_entries = 0;
    ctr->n_heavy = 0;
  }
  __shared__ uint32_t smin[3][kBpBlock], smax[3][kBpBlock];
  __shared__ double sext[kBpBlock];
  uint32_t lmin[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, lmax[3] = {0u, 0u, 0u};
  double ext = 0.0;  // sum of the boxes' largest extents (the hash grid's cell size)
  bool bad = false;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    // the row, then all nine coordinates at once (a triangle with an index out of range is
    // reported and gets the empty box at the origin)
    const int32_t vr[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    const bool ok = vr[0] >= 0 && vr[0] < nv && vr[1] >= 0 && vr[1] < nv && vr[2] >= 0 && vr[2] < nv;
    if (ok) {
      double q[3][3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) q[k][c] = x[3 * (int64_t)vr[k] + c];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lo[c] = fmin(q[0][c], fmin(q[1][c], q[2][c]));
        hi[c] = fmax(q[0][c], fmax(q[1][c], q[2][c]));
      }
      if (x_end) {  // swept box: the triangle at both ends of the straight path
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) q[k][c] = x_end[3 * (int64_t)vr[k] + c];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lo[c] = fmin(lo[c], fmin(q[0][c], fmin(q[1][c], q[2][c])));
          hi[c] = fmax(hi[c], fmax(q[0][c], fmax(q[1][c], q[2][c])));
        }
      }
    } else {
      bad = true;
    }
    ext += fmax(hi[0] - lo[0], fmax(hi[1] - lo[1], hi[2] - lo[2]));
    for (int c = 0; c < 3; ++c) {
      tbox[6 * t + c] = lo[c];
      tbox[6 * t + 3 + c] = hi[c];
      const uint32_t kc = f2key((float)(0.5 * (lo[c] + hi[c])));
      centre[3 * t + c] = (float)(0.5 * (lo[c] + hi[c]));
      lmin[c] = min(lmin[c], kc);
      lmax[c] = max(lmax[c], kc);
    }
  }
  if (bad) atomicCAS(&ctr->status, 0, STATUS_INDEX);
  for (int c = 0; c < 3; ++c) {
    smin[c][threadIdx.x] = lmin[c];
    smax[c][threadIdx.x] = lmax[c];
  }
  sext[threadIdx.x] = ext;
  __syncthreads();
  for (int w = kBpBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      for (int c = 0; c < 3; ++c) {
        smin[c][threadIdx.x] = min(smin[c][threadIdx.x], smin[c][threadIdx.x + w]);
        smax[c][threadIdx.x] = max(smax[c][threadIdx.x], smax[c][threadIdx.x + w]);
      }
      sext[threadIdx.x] += sext[threadIdx.x + w];
    }
    __syncthreads();
  }
  // per-block partial bounds and extent sums; the next kernel reduces them (the kernel
  // boundary orders the two)
  if (threadIdx.x == 0) {
    for (int c = 0; c < 3; ++c) {
      part[6 * blockIdx.x + c] = smin[c][0];
      part[6 * blockIdx.x + 3 + c] = smax[c][0];
    }
    ext_part[blockIdx.x] = sext[0];
  }
}

// spread the low 10 bits of v to every third bit
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// the problem owning item t: the last p with off[p] <= t, clamped to [0, n_prob)
__device__ __forceinline__ int problem_of(const int64_t* __restrict__ off, int n_prob, int64_t t) {
  int lo = 0, hi = n_prob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Bucket of a triangle: its problem in the top bits, then the top mbits of its Morton code, so
// every problem's triangles form one contiguous range of the sorted order.
__global__ void __launch_bounds__(kBpBlock) k_morton(const float* __restrict__ centre, int64_t nt,
                                                     const uint32_t* __restrict__ part, int nparts,
                                                     const int64_t* __restrict__ tri_off, int n_prob, int mbits,
                                                     int32_t* __restrict__ hist, uint32_t* __restrict__ bucket,
                                                     int32_t* __restrict__ rank, Counters* ctr) {
  if (tri_off && blockIdx.x == 0) {
    // the problem ranges must tile [0, nt)
    bool bad = threadIdx.x == 0 && (tri_off[0] != 0 || tri_off[n_prob] != nt);
    for (int p = threadIdx.x; p < n_prob; p += kBpBlock) bad |= tri_off[p] > tri_off[p + 1];
    if (bad) atomicCAS(&ctr->status, 0, STATUS_INVALID);
  }
  // every block reduces the per-block bounds of k_tri_boxes (a few KB, cached): a strided
  // pass per thread, then a tree in LDS
  __shared__ uint32_t red[6][kBpBlock];
  __shared__ uint32_t sb[6];
  uint32_t v[6] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u};
  for (int b = threadIdx.x; b < nparts; b += kBpBlock)
    for (int c = 0; c < 6; ++c) v[c] = c < 3 ? min(v[c], part[6 * b + c]) : max(v[c], part[6 * b + c]);
  for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int w = kBpBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 6; ++c)
        red[c][threadIdx.x] = c < 3 ? min(red[c][threadIdx.x], red[c][threadIdx.x + w])
                                    : max(red[c][threadIdx.x], red[c][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 6) sb[threadIdx.x] = red[threadIdx.x][0];
  __syncthreads();
  float lo[3], inv[3];
  for (int c = 0; c < 3; ++c) {
    lo[c] = key2f(sb[c]);
    const float ext = key2f(sb[3 + c]) - lo[c];
    inv[c] = ext > 0.f ? 1023.f / ext : 0.f;
  }
  const int lane = __lane_id();
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nt; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = base + threadIdx.x;
    const bool active = t < nt;
    uint32_t bk = 0;
    if (active) {
      uint32_t q[3];
      for (int c = 0; c < 3; ++c) {
        const float f = (centre[3 * t + c] - lo[c]) * inv[c];
        q[c] = (uint32_t)fminf(fmaxf(f, 0.f), 1023.f);
      }
      const uint32_t code = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
      const uint32_t p = tri_off ? (uint32_t)problem_of(tri_off, n_prob, t) : 0u;
      bk = (p << mbits) | (code >> (30 - mbits));
      bucket[t] = bk;
    }
    // Neighbouring triangles share buckets: group the wave's lanes by bucket (ballots only),
    // then one lane per group reserves the group's ranks with a single atomic, all groups at
    // once.  The order inside a bucket is arbitrary.
    uint64_t todo = __ballot(active);
    uint64_t group = 0;
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const uint32_t b = __shfl(bk, leader);
      const uint64_t m = __ballot(active && bk == b) & todo;
      if ((m >> lane) & 1ull) group = m;
      todo &= ~m;
    }
    const int my_leader = active ? __ffsll((unsigned long long)group) - 1 : lane;
    int32_t gbase = 0;
    if (active && my_leader == lane) gbase = atomicAdd(&hist[bk], (int32_t)__popcll(group));
    gbase = __shfl(gbase, my_leader);
    if (active) rank[t] = gbase + (int32_t)__popcll(group & ((1ull << lane) - 1ull));
  }
}

// counting-sort scatter: triangle t goes to offset[bucket] + rank; then every bucket count is
// cleared for the next call
__global__ void __launch_bounds__(kBpBlock) k_scatter(int64_t nt, int64_t nbuckets, const uint32_t* __restrict__ bucket,
                                                      const int32_t* __restrict__ rank,
                                                      const int32_t* __restrict__ offset, int32_t* __restrict__ ids,
                                                      int32_t* __restrict__ hist) {
  const int64_t n = nt > nbuckets ? nt : nbuckets;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    if (t < nt) ids[offset[bucket[t]] + rank[t]] = (int32_t)t;
    if (t < nbuckets) hist[t] = 0;
  }
}

// Level geometry of the implicit 4-ary tree: m[l] = ceil(n / 4^l) nodes at level l, stored
// from off[l]; node (l, k) covers leaves [k 4^l, (k+1) 4^l) and its children are
// (l-1, 4k .. 4k+3), contiguous in memory; level L (m[L] = 1) is the root.
struct Levels {
  int L;
  int lt;  // levels lt..L are staged in LDS by the traversal (lt > L: none)
  int64_t m[24];
  int64_t off[24];
};

// FP32 node box, padded to two 16-byte halves.  The padding of lo holds, for an inner node, the
// bits of an int32: a vertex id that every triangle of the node's subtree holds, or kNoCommon
// (kEmpty for a node with no leaves, the identity of the merge).  A query that holds that
// vertex shares it with every leaf below, so none of them can be its candidate (Sec. 1: pairs
// with a shared vertex are adjacent), and k_traverse_heavy skips the subtree: the deferred
// searches are mostly those of fans of thin triangles around one vertex, whose boxes all
// overlap.  (k_traverse does not test it: the extra compares cost its every visit more than
// the few fan queries it meets save.)
struct Box32 {
  float lo[4];
  float hi[4];
};
constexpr int32_t kNoCommon = -1;
constexpr int32_t kEmpty = -2;

__device__ __forceinline__ int32_t box_common(const Box32& b) { return __float_as_int(b.lo[3]); }
__device__ __forceinline__ void set_common(Box32& b, int32_t v) { b.lo[3] = __int_as_float(v); }
__device__ __forceinline__ int32_t merge_common(int32_t a, int32_t b) {
  return a == kEmpty ? b : (b == kEmpty ? a : (a == b ? a : kNoCommon));
}
// Whether a query with vertex ids q skips the subtree of inner node b (never with the
// vertex-adjacent option, under which one shared vertex does not make a pair adjacent).
__device__ __forceinline__ bool skip_common(const Box32& b, const int32_t q[3], bool va) {
  const int32_t v = box_common(b);
  return !va & (v >= 0) & ((v == q[0]) | (v == q[1]) | (v == q[2]));
}

// sorted leaf record: the triangle's FP64 box, its vertex ids and its index
struct LeafRec {
  double lo[3], hi[3];
  int32_t v[3];
  int32_t tri;
};

__device__ __forceinline__ Box32 box_union(const Box32& a, const Box32& b) {
  Box32 r;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r.lo[c] = fminf(a.lo[c], b.lo[c]);
    r.hi[c] = fmaxf(a.hi[c], b.hi[c]);
  }
  set_common(r, merge_common(box_common(a), box_common(b)));
  r.hi[3] = 0.0f;
  return r;
}

// The shared vertex of up to four triangles (vertex ids, or kEmpty rows for absent leaves): the
// first vertex of the first present one that every present one holds.
__device__ __forceinline__ int32_t common_of_leaves(const int3& t0, const int3& t1, const int3& t2, const int3& t3) {
  const int3 f = t0.x != kEmpty ? t0 : (t1.x != kEmpty ? t1 : (t2.x != kEmpty ? t2 : t3));
  if (f.x == kEmpty) return kEmpty;
  const auto holds = [](const int3& t, int32_t v) { return t.x == kEmpty || t.x == v || t.y == v || t.z == v; };
  const int32_t cand[3] = {f.x, f.y, f.z};
#pragma unroll
  for (int u = 0; u < 3; ++u)
    if (holds(t0, cand[u]) && holds(t1, cand[u]) && holds(t2, cand[u]) && holds(t3, cand[u])) return cand[u];
  return kNoCommon;
}

// Reduces levels l0+1 .. l0+4 (256 threads) or l0+1 .. l0+5 (1024 threads) from the boxes of
// level l0 (l0 = 0: made from the sorted leaves, which are written too).  Block b owns level-l0
// nodes [kThreads b, kThreads (b + 1)).
// For a batch (tri_off != NULL) the leaf pass also writes qend[k]: the end of the sorted range of
// the problem owning leaf k (problem p + 1 starts at the offset of its first bucket).
template <int kThreads>
__global__ void __launch_bounds__(kThreads) k_levels(int l0, Levels lv, const double* __restrict__ tbox,
                                                     const int32_t* __restrict__ ids,
                                                     const int32_t* __restrict__ tris, Box32* __restrict__ boxes,
                                                     LeafRec* __restrict__ leaves, const int64_t* __restrict__ tri_off,
                                                     int n_prob, int mbits, const int32_t* __restrict__ offset,
                                                     int32_t* __restrict__ qend) {
  __shared__ Box32 sh[kThreads];
  __shared__ int3 sv[kThreads];  // the leaves' vertex ids (leaf pass only)
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  Box32 bx;
  for (int c = 0; c < 3; ++c) {
    bx.lo[c] = 3.0e38f;
    bx.hi[c] = -3.0e38f;
  }
  set_common(bx, kEmpty);
  bx.hi[3] = 0.0f;
  int3 tv = make_int3(kEmpty, kEmpty, kEmpty);
  if (k < lv.m[l0]) {
    if (l0 == 0) {
      const int32_t t = ids[k];
      LeafRec r;
      for (int c = 0; c < 3; ++c) {
        r.lo[c] = tbox[6 * (int64_t)t + c];
        r.hi[c] = tbox[6 * (int64_t)t + 3 + c];
        bx.lo[c] = __double2float_rd(r.lo[c]);
        bx.hi[c] = __double2float_ru(r.hi[c]);
        r.v[c] = tris[3 * (int64_t)t + c];
      }
      r.tri = t;
      // a leaf with a negative id (reported as an index error) shares nothing
      tv = (r.v[0] < 0 || r.v[1] < 0 || r.v[2] < 0) ? make_int3(kNoCommon, kNoCommon, kNoCommon)
                                                   : make_int3(r.v[0], r.v[1], r.v[2]);
      set_common(bx, kNoCommon);  // a leaf box's padding is not read
      leaves[k] = r;
      if (tri_off) {
        const int p = problem_of(tri_off, n_prob, t);
        qend[k] = p + 1 < n_prob ? offset[(int64_t)(p + 1) << mbits] : (int32_t)lv.m[0];
      }
      boxes[lv.off[0] + k] = bx;
    } else {
      bx = boxes[lv.off[l0] + k];
    }
  }
  sh[threadIdx.x] = bx;
  if (l0 == 0) sv[threadIdx.x] = tv;
  __syncthreads();
  constexpr int kLevels = kThreads == 256 ? 4 : 5;
  static_assert(kThreads == 1 << (2 * kLevels), "a block reduces kThreads nodes to one");
  for (int j = 1; j <= kLevels && l0 + j <= lv.L; ++j) {
    const int cnt = kThreads >> (2 * j);
    Box32 r;
    const bool act = threadIdx.x < cnt;
    if (act) {
      r = box_union(box_union(sh[4 * threadIdx.x], sh[4 * threadIdx.x + 1]),
                    box_union(sh[4 * threadIdx.x + 2], sh[4 * threadIdx.x + 3]));
      if (l0 == 0 && j == 1) {  // level 1: the vertex its (up to four) triangles share
        set_common(r, common_of_leaves(sv[4 * threadIdx.x], sv[4 * threadIdx.x + 1], sv[4 * threadIdx.x + 2],
                                       sv[4 * threadIdx.x + 3]));
      }
    }
    __syncthreads();
    if (act) {
      sh[threadIdx.x] = r;
      const int64_t node = (int64_t)blockIdx.x * cnt + threadIdx.x;
      if (node < lv.m[l0 + j]) boxes[lv.off[l0 + j] + node] = r;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ bool overlap32(const float q[6], const Box32& b) {
  return q[0] <= b.hi[0] && b.lo[0] <= q[3] && q[1] <= b.hi[1] && b.lo[1] <= q[4] && q[2] <= b.hi[2] &&
         b.lo[2] <= q[5];
}

// Per-wave LDS staging of emitted pairs.  Each step every lane of the wave offers at most one
// pair; positions come from a ballot and the lanes below (mbcnt), so the staging needs no
// atomics.  Only a flush -- when the wave's buffer is nearly full, and once at the end --
// reserves global space, with one atomic for the whole buffer.
constexpr int kEmitCap = 128;

// Where emitted pairs go: the pair array, its capacity, the caller's pair count (the
// reservation counter itself, zeroed at the start of the broad phase) and the status word.
struct PairSink {
  int32_t* pairs;
  int64_t cap;
  unsigned long long* count;
  int32_t* status;
};

// reserves n slots; past the capacity the count still grows and TTIE_ERR_CAPACITY is latched
__device__ __forceinline__ int64_t sink_reserve(const PairSink& o, uint32_t n) {
  const int64_t base = (int64_t)atomicAdd(o.count, (unsigned long long)n);
  if (base + n > o.cap) atomicCAS(o.status, 0, STATUS_CAPACITY);
  return base;
}

struct WaveEmitter {
  int2* buf;       // this wave's kEmitCap slots in LDS
  int count;       // wave-uniform fill level

  __device__ __forceinline__ void flush(const PairSink& o) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int lane = __lane_id();
    int64_t base = 0;
    if (lane == 0) base = sink_reserve(o, (uint32_t)count);
    base = __shfl(base, 0);
    for (int i = lane; i < count; i += 64) {
      const int64_t slot = base + i;
      if (slot < o.cap) reinterpret_cast<int2*>(o.pairs)[slot] = buf[i];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    count = 0;
  }

  __device__ __forceinline__ void push(bool want, int32_t a, int32_t b, const PairSink& o) {
    const uint64_t mask = __ballot(want);
    if (!mask) return;
    if (want) {
      const int lane = __lane_id();
      buf[count + __popcll(mask & ((1ull << lane) - 1ull))] = make_int2(min(a, b), max(a, b));
    }
    count += __popcll(mask);
    if (count > kEmitCap - 64) flush(o);
  }
};

// End of an emitting kernel: one atomic reserves the space of all the block's waves (every
// thread of the block must arrive here).
template <int kWaves>
__device__ __forceinline__ void block_flush(WaveEmitter& em, int* wcount, int64_t* bbase, const PairSink& o) {
  const int wave = threadIdx.x / 64;
  if (__lane_id() == 0) wcount[wave] = em.count;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kWaves; ++w) tot += wcount[w];
    *bbase = tot ? sink_reserve(o, tot) : 0;
  }
  __syncthreads();
  int64_t base = *bbase;
  for (int w = 0; w < wave; ++w) base += wcount[w];
  for (int i = __lane_id(); i < em.count; i += 64) {
    const int64_t slot = base + i;
    if (slot < o.cap) reinterpret_cast<int2*>(o.pairs)[slot] = em.buf[i];
  }
}

// Two lanes per leaf s, depth-first over the subtrees holding leaves after s.  A visited node
// tests its four children at once (one contiguous load); the pending children of every level
// on the current path are kept as 4-bit masks in one 64-bit word, so no stack is needed.
// Block b's 256 queries are exactly the leaves of the level-4 node b.  That subtree (leaf
// records, leaf boxes and the 84 boxes above them) is staged in LDS; waves 0-3 search it
// (the local part, LDS only) while waves 4-7 search everything after it from the root (the
// global part), so each query costs the larger of the two instead of their sum.
// The top levels of the tree (those that fit kTopCap boxes, never below level 4) are staged
// in LDS too, so the global part reads only the levels 3..0 of other blocks' subtrees.
constexpr int kSubLevels = 4;                       // 4^4 = 256 = kBpBlock leaves per block
constexpr int kSubInner = 64 + 16 + 4;              // boxes of levels 1..3 inside the subtree
constexpr int kTravThreads = 2 * kBpBlock;          // a local and a global lane per query
constexpr int kTravWaves = kTravThreads / 64;
constexpr int kTopCap = 864;                        // 27 KB of top-level boxes

// A lane that has visited `budget` nodes (a launch parameter, 128 by default) hands the rest
// of its search to k_traverse_heavy (a wave per query, or per batch of queries when many are
// deferred), by saving its depth-first state: the node it is about to visit and the pending
// siblings of every ancestor up to its starting level.  At the default budget few queries get
// there -- those whose boxes overlap hundreds of others, as in the fan of thin triangles around
// a pole; a low budget defers many short searches instead.
struct TravState {
  int32_t s;      // query leaf (sorted position)
  int32_t part;   // 1: global part (skips the query's own level-4 subtree)
  int32_t l, k;   // node about to be visited
  uint64_t pend;  // pending children per level, 4 bits each
  int32_t top;    // starting level
  int32_t last;   // end of the query's problem (leaves)
};

// LDS the traversal of one block works from
struct TravShared {
  int2 stage[kTravWaves][kEmitCap];
  int32_t lm[24], loff[24];  // the level table (node counts and offsets fit 32 bits)
  int wcount[kTravWaves];
  int64_t bbase;
  LeafRec sleaf[kBpBlock];
  Box32 sbox[kBpBlock + kSubInner];  // the block's subtree: level 0 at [0, 256), then 1, 2, 3
  Box32 stop[kTopCap];               // levels lt..L, in storage order
};

// The search of one part for the lane's query s.  kGlobal is wave-uniform (waves 0-3 search
// the block's own subtree, waves 4-7 the rest of the tree), so the sources are fixed: the local
// part reads only LDS, the global part reads the top levels from LDS and the lower levels and
// the leaves from global memory.  Tests are written without short-circuit branches and the
// climb takes the lowest pending bit, so the loop carries little divergence.
template <bool kGlobal>
__device__ __forceinline__ void traverse_part(TravShared& sh, int32_t n, int32_t blk, int32_t s, bool active, int lt,
                                              int32_t tbase, int L, const Box32* __restrict__ boxes,
                                              const LeafRec* __restrict__ leaves, const int32_t* __restrict__ qend,
                                              TravState* heavy, int64_t heavy_cap, int budget, bool va, WaveEmitter& em,
                                              const PairSink& sink, Counters* ctr, int& status) {
  const int qi = s - blk * kBpBlock;
  const bool small_tree = L <= kSubLevels;
  int l = kGlobal || small_tree ? L : kSubLevels;
  int32_t k = kGlobal || small_tree ? 0 : blk;
  const int top = l;   // the search ends when nothing is pending at or above this level
  uint64_t pend = 0;   // pending children of level j's current node at bits [4j, 4j + 4)
  float q[6] = {0, 0, 0, 0, 0, 0};
  LeafRec me{};
  int32_t last = n;    // leaves after s up to the end of the query's problem
  if (active) {
    if (qend) last = qend[s];
    me = sh.sleaf[qi];
    const Box32 b = sh.sbox[qi];
    for (int c = 0; c < 3; ++c) {
      q[c] = b.lo[c];
      q[3 + c] = b.hi[c];
    }
  }
  int visits = 0;
  bool may_defer = true;  // one attempt: with the list full the lane finishes its own search
  for (int32_t iter = 0; __ballot(active); ++iter) {
    if (iter > 2 * n + 64) {  // every node is visited at most once: only corruption gets here
      status = STATUS_CAPACITY;
      break;
    }
    // over budget: hand the remaining search to a wave of its own (when the list has room)
    const bool over = active && may_defer && visits >= budget;
    const uint32_t hs = wave_slot(over, &ctr->n_heavy);
    if (over) may_defer = false;
    if (over && (int64_t)hs < heavy_cap) {
      TravState t;
      t.s = s;
      t.part = kGlobal ? 1 : 0;
      t.l = l;
      t.k = k;
      t.pend = pend;
      t.top = top;
      t.last = last;
      heavy[hs] = t;
      active = false;
    }
    ++visits;
    // children of (l, k): (l - 1, 4k + i), only those holding leaves after s (and, in the
    // global part, never the block's own subtree) up to the problem's last leaf
    const int lc = l - 1;
    const int32_t c0 = 4 * k;
    uint32_t mask = 0;
    if (active) {
      int32_t first = lc > 0 ? (s >> (2 * lc)) : s + 1;
      if (kGlobal && lc == kSubLevels) first = blk + 1;
      const int32_t lastc = (last - 1) >> (2 * lc);
      const int32_t hi = min(lastc, sh.lm[lc] - 1);
      Box32 cb[4];
      if (!kGlobal) {
        const int lb = (lc == 0 ? 0 : (lc == 1 ? kBpBlock : (lc == 2 ? kBpBlock + 64 : kBpBlock + 80)));
        const int li = c0 - (blk << (2 * (kSubLevels - lc)));
#pragma unroll
        for (int i = 0; i < 4; ++i) cb[i] = sh.sbox[lb + li + i];
      } else if (lc >= lt) {
        const int ti = sh.loff[lc] - tbase + c0;
#pragma unroll
        for (int i = 0; i < 4; ++i) cb[i] = sh.stop[ti + i];
      } else {
        const Box32* g = boxes + sh.loff[lc] + c0;
#pragma unroll
        for (int i = 0; i < 4; ++i) cb[i] = g[i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int32_t c = c0 + i;
        const bool ov = (q[0] <= cb[i].hi[0]) & (cb[i].lo[0] <= q[3]) & (q[1] <= cb[i].hi[1]) &
                        (cb[i].lo[1] <= q[4]) & (q[2] <= cb[i].hi[2]) & (cb[i].lo[2] <= q[5]);
        mask |= (uint32_t)(ov & (c >= first) & (c <= hi)) << i;
      }
    }
    // leaves: exact FP64 box test and the shared-vertex test
    uint32_t want = 0;
    int32_t other[4] = {0, 0, 0, 0};
    if (active && lc == 0 && mask) {
      LeafRec o[4];
      if (!kGlobal) {
        const int li = c0 - blk * kBpBlock;
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = sh.sleaf[li + i];
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = leaves[c0 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        bool ex = (mask >> i) & 1u;
#pragma unroll
        for (int c = 0; c < 3; ++c) ex = ex & (me.lo[c] <= o[i].hi[c]) & (o[i].lo[c] <= me.hi[c]);
        want |= (uint32_t)(ex & !is_adjacent(me.v, o[i].v, va)) << i;
        other[i] = o[i].tri;
      }
    }
    if (__ballot(want != 0)) {
#pragma unroll
      for (int i = 0; i < 4; ++i) em.push((want >> i) & 1u, me.tri, other[i], sink);
    }
    if (active) {
      if (lc == 0) mask = 0;
      if (mask) {
        // descend into the first child; the others wait in this level's slot
        const int i = __builtin_ctz(mask);
        pend |= (uint64_t)(mask & ~(1u << i)) << (4 * lc);
        l = lc;
        k = c0 + i;
      } else {
        // resume at the lowest level at or above l with a pending child (slots above the
        // starting level are never set)
        const uint64_t rem = l < 16 ? pend >> (4 * l) : 0;
        if (rem == 0) {
          active = false;
        } else {
          const int b = __builtin_ctzll(rem);
          const int j = l + (b >> 2);
          pend &= ~(1ull << (4 * l + b));
          k = ((k >> (2 * (j - l))) & ~3) + (b & 3);
          l = j;
        }
      }
    }
  }
}

// kVA: pairs sharing exactly one vertex are candidates (a template argument, so the default
// keeps the plain shared-vertex test in its leaf loop)
template <bool kVA>
__global__ void __launch_bounds__(kTravThreads) k_traverse(int64_t n64, Levels lv, const Box32* __restrict__ boxes,
                                                           const LeafRec* __restrict__ leaves,
                                                           const int32_t* __restrict__ qend, TravState* heavy,
                                                           int64_t heavy_cap, int budget, int32_t* pairs,
                                                           int64_t cap,
                                                           unsigned long long* npairs, Counters* ctr) {
  __shared__ TravShared sh;
  const PairSink sink{pairs, cap, npairs, &ctr->status};
  const int32_t n = (int32_t)n64;
  const int32_t blk = (int32_t)xcd_block(blockIdx.x, gridDim.x);
  const int lt = lv.lt;
  const int32_t tbase = lt <= lv.L ? (int32_t)lv.off[lt] : 0;
  const int ntop = lt <= lv.L ? (int)(lv.off[lv.L] + 4 - tbase) : 0;  // through the padded root level
  for (int i = threadIdx.x; i < ntop; i += kTravThreads) sh.stop[i] = boxes[tbase + i];
  const int qi = threadIdx.x % kBpBlock;  // query within the block
  const bool global_part = __builtin_amdgcn_readfirstlane(threadIdx.x) >= kBpBlock;  // wave-uniform
  if (threadIdx.x < 24) {
    sh.lm[threadIdx.x] = (int32_t)lv.m[threadIdx.x];
    sh.loff[threadIdx.x] = (int32_t)lv.off[threadIdx.x];
  }
  // stage the block's subtree
  const int32_t s = blk * kBpBlock + qi;
  if (!global_part && s < n) {
    sh.sleaf[qi] = leaves[s];
    sh.sbox[qi] = boxes[s];
  }
  if (global_part) {
    const int t = qi;
    int l = 0, local = 0, base = kBpBlock;  // thread t < 84 loads inner box t
    if (t < 64) { l = 1; local = t; base = kBpBlock; }
    else if (t < 80) { l = 2; local = t - 64; base = kBpBlock + 64; }
    else if (t < 84) { l = 3; local = t - 80; base = kBpBlock + 80; }
    if (l > 0 && l <= lv.L) {
      const int64_t k = ((int64_t)blk << (2 * (kSubLevels - l))) + local;
      if (k < lv.m[l]) sh.sbox[base + local] = boxes[lv.off[l] + k];
    }
  }
  __syncthreads();

  WaveEmitter em{sh.stage[threadIdx.x / 64], 0};
  int status = 0;
  const bool small_tree = lv.L <= kSubLevels;
  if (global_part)
    traverse_part<true>(sh, n, blk, s, s < n && !small_tree, lt, tbase, lv.L, boxes, leaves, qend, heavy, heavy_cap,
                        budget, kVA, em, sink, ctr, status);
  else
    traverse_part<false>(sh, n, blk, s, s < n, lt, tbase, lv.L, boxes, leaves, qend, heavy, heavy_cap, budget, kVA,
                         em, sink, ctr, status);
  block_flush<kTravWaves>(em, sh.wcount, &sh.bbase, sink);
  if (status) atomicCAS(&ctr->status, 0, status);
}

// One wave per batch of saved queries (one query while the list is no longer than the grid,
// at most kHeavyQ), skipping every subtree whose triangles all hold one of the query's
// vertices: the remaining nodes of all of them form
// one stack in LDS, each entry tagged with its query's slot; every step each lane takes one
// node, tests its four children against that query's box, and pushes the overlapping inner
// children (or tests the leaves).  A query that overlaps hundreds of leaves needs tens of steps
// instead of hundreds of serial visits, and queries with a few visits left share the wave's
// lanes instead of holding a whole wave each.  Everything but the stack is read from global
// memory.
//
// Stack bound: a query saved at level l brings at most 1 + 3 (L - l) entries, and a step
// replaces at most 64 entries by at most 256 children one level down, so the stack holds at
// most Q (1 + 3 L) + 3 * 64 * L + 64 entries; the host picks Q so that this fits kHeavyStack.
constexpr int kHeavyStack = 4096;
constexpr int kHeavyQ = 32;

inline int heavy_batch(int L) {
  const int q = (kHeavyStack - 64 - 3 * 64 * L) / (1 + 3 * L);
  return q < 1 ? 1 : (q > kHeavyQ ? kHeavyQ : q);
}

__global__ void __launch_bounds__(64) k_traverse_heavy(Levels lv, const Box32* __restrict__ boxes,
                                                       const LeafRec* __restrict__ leaves,
                                                       const TravState* __restrict__ heavy, int64_t heavy_cap, int va,
                                                       int nq_max, int32_t* pairs, int64_t cap,
                                                       unsigned long long* npairs, Counters* ctr) {
  const PairSink sink{pairs, cap, npairs, &ctr->status};
  __shared__ int2 stack[kHeavyStack];  // (level | slot << 8, node)
  __shared__ int2 stage[kEmitCap];
  __shared__ int wcount[1];
  __shared__ int64_t bbase;
  __shared__ float sq[kHeavyQ][6];      // per slot: the query's FP32 box
  __shared__ LeafRec sme[kHeavyQ];      // its leaf record
  __shared__ int32_t ss[kHeavyQ], slast[kHeavyQ], spart[kHeavyQ];
  WaveEmitter em{stage, 0};
  const int lane = __lane_id();
  int status = 0;
  const int64_t nh = min((int64_t)ctr->n_heavy, heavy_cap);
  // one query per wave while the list is no longer than the grid, then batches just large
  // enough to cover it in one pass (at most nq_max)
  const int per = (int)min((int64_t)nq_max, max((int64_t)1, (nh + gridDim.x - 1) / gridDim.x));
  for (int64_t it0 = (int64_t)blockIdx.x * per; it0 < nh; it0 += (int64_t)gridDim.x * per) {
    const int nq = (int)min((int64_t)per, nh - it0);
    // lane j < nq loads query j and lists its remaining search: the node it was about to
    // visit and the pending siblings of its ancestors (slot j of pend: siblings at level j)
    TravState t{};
    int cnt = 0;
    if (lane < nq) {
      t = heavy[it0 + lane];
      const Box32 qb = boxes[lv.off[0] + t.s];
      for (int c = 0; c < 3; ++c) {
        sq[lane][c] = qb.lo[c];
        sq[lane][3 + c] = qb.hi[c];
      }
      sme[lane] = leaves[t.s];
      ss[lane] = t.s;
      slast[lane] = t.last;
      spart[lane] = t.part;
      cnt = 1;
      for (int j = t.l; j < t.top; ++j) cnt += __popc((uint32_t)(t.pend >> (4 * j)) & 15u);
    }
    int incl = cnt;
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d);
      if (lane >= d) incl += y;
    }
    int sp = __shfl(incl, 63);
    if (sp > kHeavyStack) {  // excluded by the host's choice of nq_max; never silent
      status = STATUS_CAPACITY;
      break;
    }
    if (lane < nq) {
      int pos = incl - cnt;
      stack[pos++] = make_int2(t.l | lane << 8, t.k);
      for (int j = t.l; j < t.top; ++j) {
        const uint32_t pm = (uint32_t)(t.pend >> (4 * j)) & 15u;
        const int32_t anc = t.k >> (2 * (j - t.l));
        for (int i = 0; i < 4; ++i)
          if (pm & (1u << i)) stack[pos++] = make_int2(j | lane << 8, (anc & ~3) + i);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    while (sp > 0) {
      const int take = sp < 64 ? sp : 64;
      int2 node = make_int2(0, 0);
      const bool act = lane < take;
      if (act) node = stack[sp - 1 - lane];
      sp -= take;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int slot = node.x >> 8;
      const int lc = (node.x & 255) - 1;
      const int64_t c0 = 4 * (int64_t)node.y;
      const int64_t s = ss[slot];
      uint32_t mask = 0;
      if (act) {
        float q[6];
        for (int c = 0; c < 6; ++c) q[c] = sq[slot][c];
        int64_t first = lc > 0 ? (s >> (2 * lc)) : s + 1;
        if (spart[slot] != 0 && lc == kSubLevels) first = s / kBpBlock + 1;
        const int64_t lastc = ((int64_t)slast[slot] - 1) >> (2 * lc);
        const int64_t mcount = lv.m[lc];
        const Box32* g = boxes + lv.off[lc] + c0;
        Box32 cb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) cb[i] = g[i];
        const int32_t* qv = sme[slot].v;
        const int32_t qv3[3] = {qv[0], qv[1], qv[2]};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t c = c0 + i;
          if (c < mcount && c >= first && c <= lastc && overlap32(q, cb[i]) &&
              !(lc > 0 && skip_common(cb[i], qv3, va != 0)))
            mask |= 1u << i;
        }
      }
      // leaves: exact tests and emission
      bool want[4] = {false, false, false, false};
      int32_t other[4] = {0, 0, 0, 0};
      int32_t mine = 0;
      if (act && lc == 0 && mask) {
        const LeafRec me = sme[slot];
        mine = me.tri;
        LeafRec o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = leaves[c0 + i];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          bool exact = (mask >> i) & 1u;
          for (int c = 0; c < 3; ++c) exact = exact && me.lo[c] <= o[i].hi[c] && o[i].lo[c] <= me.hi[c];
          want[i] = exact && !is_adjacent(me.v, o[i].v, va);
          other[i] = o[i].tri;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) em.push(want[i], mine, other[i], sink);
      // inner children: onto the stack (wave prefix sum of the counts), with the slot tag
      const int ccnt = act && lc > 0 ? __popc(mask) : 0;
      int cincl = ccnt;
      for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(cincl, d);
        if (lane >= d) cincl += y;
      }
      const int total = __shfl(cincl, 63);
      if (sp + total > kHeavyStack) {
        status = STATUS_CAPACITY;  // excluded by the bound above; never silent
        break;
      }
      int pos = sp + cincl - ccnt;
      for (int i = 0; i < 4; ++i)
        if (ccnt && (mask & (1u << i))) stack[pos++] = make_int2(lc | slot << 8, (int32_t)(c0 + i));
      sp += total;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    if (status) break;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the slot arrays are refilled by the next batch
  }
  block_flush<1>(em, wcount, &bbase, sink);
  if (status) atomicCAS(&ctr->status, 0, status);
}

__global__ void __launch_bounds__(kBpBlock) k_brute(const int32_t* __restrict__ tris, int64_t nt, int32_t* pairs,
                                                    int64_t cap, unsigned long long* npairs, int va, Counters* ctr) {
  const PairSink sink{pairs, cap, npairs, &ctr->status};
  __shared__ int2 stage[kBpBlock / 64][kEmitCap];
  WaveEmitter em{stage[threadIdx.x / 64], 0};
  for (int64_t i = blockIdx.y; i < nt; i += gridDim.y) {
    int32_t vi[3];
    for (int k = 0; k < 3; ++k) vi[k] = tris[3 * i + k];
    for (int64_t jb = (int64_t)blockIdx.x * blockDim.x; jb < nt; jb += (int64_t)gridDim.x * blockDim.x) {
      const int64_t j = jb + threadIdx.x;
      bool want = false;
      if (j > i && j < nt) {
        const int32_t vj[3] = {tris[3 * j], tris[3 * j + 1], tris[3 * j + 2]};
        want = !is_adjacent(vi, vj, va);
      }
      em.push(want, (int32_t)i, (int32_t)j, sink);
    }
  }
  if (em.count > 0) em.flush(sink);
}

// ---- spatial hashing (the broad phase of Sec. 1.2) -----------------------------------------
// A uniform grid of cell size h (twice the mean largest box extent) anchored at the lowest box
// centre.  Every triangle is entered in each cell its FP64 box covers; entries are counting-
// sorted by a hash of the cell (MurmurHash3's 64-bit finalizer), and a thread per entry tests
// the later entries of its bucket that name the same cell.  A pair is reported only from its
// reference cell -- the componentwise maximum of the two boxes' lowest cells, which both boxes
// cover exactly when they overlap -- so each overlapping pair is found once, and the result is
// the same canonical set as the LBVH's.
//
//   k_hash_cells    grid parameters (every block reduces the box partials the same way), cell
//                   ranges, entries reserved per wave with one atomic, bucket ranks
//   scan            bucket offsets
//   k_hash_scatter  entries to their sorted places; bucket counts cleared for the next call
//   k_hash_pairs    same-cell tests within buckets, exact box and shared-vertex tests, emission
constexpr int kCellBits = 21;             // signed cell coordinates packed into 63 bits
constexpr int64_t kCellLimit = 1 << 20;   // |cell index| bound

struct HashGrid {
  double org[3];
  double h;
};

__device__ __forceinline__ int64_t cell_of(double v, double org, double h) { return (int64_t)floor((v - org) / h); }

__device__ __forceinline__ uint64_t cell_key(int64_t cx, int64_t cy, int64_t cz) {
  const uint64_t m = (1ull << kCellBits) - 1;
  return (((uint64_t)cx & m) << (2 * kCellBits)) | (((uint64_t)cy & m) << kCellBits) | ((uint64_t)cz & m);
}

__device__ __forceinline__ uint32_t hash_bucket(uint64_t k, int bits) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return (uint32_t)(k >> (64 - bits));
}

__global__ void __launch_bounds__(kBpBlock) k_hash_cells(const double* __restrict__ tbox, int64_t nt,
                                                         const uint32_t* __restrict__ part,
                                                         const double* __restrict__ ext_part, int nparts, int hbits,
                                                         int32_t* __restrict__ hist, uint64_t* __restrict__ key,
                                                         int32_t* __restrict__ tri, int32_t* __restrict__ rank,
                                                         int64_t ecap, HashGrid* grid, Counters* ctr) {
  __shared__ uint32_t red[6][kBpBlock];
  __shared__ double rext[kBpBlock];
  __shared__ HashGrid sg;
  uint32_t v[6] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u};
  double e = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kBpBlock) {
    for (int c = 0; c < 6; ++c) v[c] = c < 3 ? min(v[c], part[6 * b + c]) : max(v[c], part[6 * b + c]);
    e += ext_part[b];
  }
  for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
  rext[threadIdx.x] = e;
  __syncthreads();
  for (int w = kBpBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      for (int c = 0; c < 6; ++c)
        red[c][threadIdx.x] = c < 3 ? min(red[c][threadIdx.x], red[c][threadIdx.x + w])
                                    : max(red[c][threadIdx.x], red[c][threadIdx.x + w]);
      rext[threadIdx.x] += rext[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double span = 0.0;
    for (int c = 0; c < 3; ++c) {
      sg.org[c] = (double)key2f(red[c][0]);
      span = fmax(span, (double)key2f(red[3 + c][0]) - sg.org[c]);
    }
    double h = 2.0 * rext[0] / (double)nt;
    // keep the cell indices of the scene far inside the packed range
    const double hmin = span / (double)(kCellLimit / 4);
    if (!(h > hmin)) h = hmin;
    if (!(h > 0.0) || !(h < 1.0e300)) h = 1.0;
    sg.h = h;
    if (blockIdx.x == 0) *grid = sg;
  }
  __syncthreads();
  const HashGrid g = sg;
  int status = 0;
  const int lane = __lane_id();
  for (int64_t base = (int64_t)blockIdx.x * kBpBlock; base < nt; base += (int64_t)gridDim.x * kBpBlock) {
    const int64_t t = base + threadIdx.x;
    int64_t lo[3] = {0, 0, 0}, hi[3] = {-1, -1, -1};
    uint32_t n = 0;
    if (t < nt) {
      bool ok = true;
      for (int c = 0; c < 3; ++c) {
        lo[c] = cell_of(tbox[6 * t + c], g.org[c], g.h);
        hi[c] = cell_of(tbox[6 * t + 3 + c], g.org[c], g.h);
        ok = ok && lo[c] > -kCellLimit && hi[c] < kCellLimit && hi[c] >= lo[c] && hi[c] - lo[c] < 1024;
      }
      if (ok) {
        const int64_t cnt = (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
        if (cnt <= (1 << 20)) n = (uint32_t)cnt;
        else ok = false;
      }
      if (!ok) status = STATUS_UNSUPPORTED;  // a box far outside the grid or over a million cells
    }
    // wave prefix sum of the entry counts, one atomic per wave
    uint32_t incl = n;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d);
      if (lane >= d) incl += y;
    }
    const uint32_t total = __shfl(incl, 63);
    uint64_t wbase = 0;
    if (lane == 63 && total) wbase = atomicAdd(reinterpret_cast<unsigned long long*>(&ctr->n_entries), (unsigned long long)total);
    wbase = __shfl(wbase, 63);
    int64_t slot = (int64_t)wbase + incl - n;
    for (int64_t cx = lo[0]; cx <= hi[0] && n; ++cx)
      for (int64_t cy = lo[1]; cy <= hi[1]; ++cy)
        for (int64_t cz = lo[2]; cz <= hi[2]; ++cz, ++slot) {
          if (slot >= ecap) {
            status = STATUS_CAPACITY;
            continue;
          }
          const uint64_t k = cell_key(cx, cy, cz);
          key[slot] = k;
          tri[slot] = (int32_t)t;
          rank[slot] = atomicAdd(&hist[hash_bucket(k, hbits)], 1);
        }
  }
  if (status) atomicCAS(&ctr->status, 0, status);
}

__global__ void __launch_bounds__(kBpBlock) k_hash_scatter(const Counters* ctr, int64_t ecap, int64_t nbuckets, int hbits,
                                                           const uint64_t* __restrict__ key,
                                                           const int32_t* __restrict__ tri,
                                                           const int32_t* __restrict__ rank,
                                                           const int32_t* __restrict__ offset,
                                                           uint64_t* __restrict__ skey, int32_t* __restrict__ stri,
                                                           int32_t* __restrict__ hist) {
  const int64_t ne = min((int64_t)ctr->n_entries, ecap);
  const int64_t n = ne > nbuckets ? ne : nbuckets;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < ne) {
      const uint64_t k = key[e];
      const int64_t pos = (int64_t)offset[hash_bucket(k, hbits)] + rank[e];
      skey[pos] = k;
      stri[pos] = tri[e];
    }
    if (e < nbuckets) hist[e] = 0;
  }
}

// one entry's view of its bucket: its triangle's FP64 box, lowest cell and vertices
struct HashQuery {
  uint64_t key;
  int32_t tri;
  int64_t end;  // end of the bucket in sorted order
  double lo[3], hi[3];
  int64_t cell[3];
  int32_t v[3];
};

__device__ __forceinline__ HashQuery hash_query(int64_t e, int64_t ne, int64_t nbuckets, int hbits,
                                                const int32_t* __restrict__ offset, const uint64_t* __restrict__ skey,
                                                const int32_t* __restrict__ stri, const double* __restrict__ tbox,
                                                const int32_t* __restrict__ tris, const HashGrid& g) {
  HashQuery h;
  h.key = skey[e];
  h.tri = stri[e];
  const uint32_t b = hash_bucket(h.key, hbits);
  h.end = (int64_t)b + 1 < nbuckets ? offset[b + 1] : ne;
  for (int c = 0; c < 3; ++c) {
    h.lo[c] = tbox[6 * (int64_t)h.tri + c];
    h.hi[c] = tbox[6 * (int64_t)h.tri + 3 + c];
    h.cell[c] = cell_of(h.lo[c], g.org[c], g.h);
    h.v[c] = tris[3 * (int64_t)h.tri + c];
  }
  return h;
}

// entry j of the same bucket: a candidate iff it names the same cell, the closed FP64 boxes
// overlap, this cell is the pair's reference cell, and no vertex is shared
__device__ __forceinline__ bool hash_test(const HashQuery& h, int64_t j, const uint64_t* __restrict__ skey,
                                          const int32_t* __restrict__ stri, const double* __restrict__ tbox,
                                          const int32_t* __restrict__ tris, const HashGrid& g, bool va,
                                          int32_t& other) {
  if (skey[j] != h.key) return false;
  other = stri[j];
  bool hit = true;
  int64_t ref[3];
  for (int c = 0; c < 3; ++c) {
    const double blo = tbox[6 * (int64_t)other + c], bhi = tbox[6 * (int64_t)other + 3 + c];
    hit = hit && h.lo[c] <= bhi && blo <= h.hi[c];
    const int64_t bc = cell_of(blo, g.org[c], g.h);
    ref[c] = h.cell[c] > bc ? h.cell[c] : bc;
  }
  if (!hit || cell_key(ref[0], ref[1], ref[2]) != h.key) return false;
  const int32_t vo[3] = {tris[3 * (int64_t)other], tris[3 * (int64_t)other + 1], tris[3 * (int64_t)other + 2]};
  return !is_adjacent(h.v, vo, va);
}

// A thread tests at most `hbudget` (a launch parameter, 64 by default) later entries of its
// bucket; the rest of a longer bucket
// (the cells where many triangles meet, e.g. the fan around a pole) goes to k_hash_heavy, where
// a whole wave shares it.

__global__ void __launch_bounds__(kBpBlock) k_hash_pairs(const Counters* ctr, int64_t ecap, int64_t nbuckets, int hbits,
                                                         const int32_t* __restrict__ offset,
                                                         const uint64_t* __restrict__ skey,
                                                         const int32_t* __restrict__ stri,
                                                         const double* __restrict__ tbox,
                                                         const int32_t* __restrict__ tris, const HashGrid* grid,
                                                         int hbudget, int va, int32_t* __restrict__ heavy,
                                                         int32_t* pairs,
                                                         int64_t cap,
                                                         unsigned long long* npairs, Counters* out_ctr) {
  const PairSink sink{pairs, cap, npairs, &out_ctr->status};
  __shared__ int2 stage[kBpBlock / 64][kEmitCap];
  __shared__ int wcount[kBpBlock / 64];
  __shared__ int64_t bbase;
  WaveEmitter em{stage[threadIdx.x / 64], 0};
  const int64_t ne = min((int64_t)ctr->n_entries, ecap);
  const HashGrid g = *grid;
  for (int64_t base = (int64_t)blockIdx.x * kBpBlock; base < ne; base += (int64_t)gridDim.x * kBpBlock) {
    const int64_t e = base + threadIdx.x;
    const bool active = e < ne;
    HashQuery h;
    int64_t stop = 0;
    if (active) {
      h = hash_query(e, ne, nbuckets, hbits, offset, skey, stri, tbox, tris, g);
      stop = min(h.end, e + 1 + hbudget);
    }
    const bool defer = active && h.end > stop;
    const uint32_t slot = wave_slot(defer, &out_ctr->n_heavy);
    if (defer) heavy[slot] = (int32_t)e;  // slot < ne <= ecap
    // the loop runs while any lane has work, so the emitter always sees the whole wave
    for (int64_t j = e + 1; __ballot(active && j < stop); ++j) {
      int32_t other = 0;
      const bool want = active && j < stop && hash_test(h, j, skey, stri, tbox, tris, g, va, other);
      em.push(want, h.tri, other, sink);
    }
  }
  block_flush<kBpBlock / 64>(em, wcount, &bbase, sink);
}

// one wave per deferred entry: its lanes stride over the rest of the bucket
__global__ void __launch_bounds__(kBpBlock) k_hash_heavy(const Counters* ctr, int64_t ecap, int64_t nbuckets, int hbits,
                                                         const int32_t* __restrict__ offset,
                                                         const uint64_t* __restrict__ skey,
                                                         const int32_t* __restrict__ stri,
                                                         const double* __restrict__ tbox,
                                                         const int32_t* __restrict__ tris, const HashGrid* grid,
                                                         int hbudget, int va, const int32_t* __restrict__ heavy,
                                                         int32_t* pairs,
                                                         int64_t cap, unsigned long long* npairs, Counters* out_ctr) {
  const PairSink sink{pairs, cap, npairs, &out_ctr->status};
  __shared__ int2 stage[kBpBlock / 64][kEmitCap];
  __shared__ int wcount[kBpBlock / 64];
  __shared__ int64_t bbase;
  WaveEmitter em{stage[threadIdx.x / 64], 0};
  const int64_t ne = min((int64_t)ctr->n_entries, ecap);
  const int64_t nh = min((int64_t)ctr->n_heavy, ne);
  const HashGrid g = *grid;
  const int waves = gridDim.x * (kBpBlock / 64);
  for (int64_t it = (int64_t)blockIdx.x * (kBpBlock / 64) + threadIdx.x / 64; it < nh; it += waves) {
    const int64_t e = heavy[it];
    const HashQuery h = hash_query(e, ne, nbuckets, hbits, offset, skey, stri, tbox, tris, g);
    for (int64_t jb = e + 1 + hbudget; jb < h.end; jb += 64) {
      const int64_t j = jb + __lane_id();
      int32_t other = 0;
      const bool want = j < h.end && hash_test(h, j, skey, stri, tbox, tris, g, va, other);
      em.push(want, h.tri, other, sink);
    }
  }
  block_flush<kBpBlock / 64>(em, wcount, &bbase, sink);
}



static unsigned bp_grid(int64_t n, unsigned cap = 4096) {
  int64_t g = (n + kBpBlock - 1) / kBpBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Every level is stored padded to a multiple of 4 nodes, so the four children of any node can
// be loaded together without bounds checks (padding slots are never selected: c < m[l]).
static int64_t pad4(int64_t m) { return (m + 3) & ~(int64_t)3; }

Levels make_levels(int64_t n) {
  Levels lv{};
  int64_t off = 0, m = n;
  int l = 0;
  for (;; ++l) {
    lv.m[l] = m;
    lv.off[l] = off;
    off += pad4(m);
    if (m <= 1) break;
    m = (m + 3) / 4;
  }
  lv.L = l;
  // the highest levels whose (padded) boxes fit the traversal's LDS cache, never below level 4
  int64_t cum = 0;
  lv.lt = l + 1;
  for (int k = l; k >= kSubLevels; --k) {
    if (cum + pad4(lv.m[k]) > kTopCap) break;
    cum += pad4(lv.m[k]);
    lv.lt = k;
  }
  return lv;
}

hipError_t launch_broadphase(Ctx* c, const ttie_mesh* m, int method, const double* x_end, int n_prob,
                             const int64_t* tri_off, int32_t* pairs, int64_t capacity, int64_t* n_pairs, hipStream_t s) {
  const Layout& L = c->L;
  Counters* ctr = wsp<Counters>(c, L.counters);
  const int64_t nt = m->n_tris;
  unsigned long long* npairs = reinterpret_cast<unsigned long long*>(n_pairs);
  const int va = (method & TTIE_BROAD_VERTEX_ADJACENT) ? 1 : 0;
  method &= 0xff;
  if (method == TTIE_BROAD_BRUTE || nt < 2) k_bp_init<<<1, 64, 0, s>>>(ctr, npairs);
  if (method == TTIE_BROAD_BRUTE) {
    dim3 grid(bp_grid(nt, 64), (unsigned)(nt < 8192 ? (nt > 0 ? nt : 1) : 8192));
    stage_begin(c, TTIE_STAGE_BP_TRAVERSE, s);
    k_brute<<<grid, kBpBlock, 0, s>>>(m->tris, nt, pairs, capacity, npairs, va, ctr);
    stage_end(c, TTIE_STAGE_BP_TRAVERSE, s);
  } else if (method == TTIE_BROAD_HASH && nt >= 2) {
    double* tbox = wsp<double>(c, L.bvh_tbox);
    const unsigned gb = bp_grid(nt, kBoundsBlocks);
    int hbits = 8;
    while (hbits < kMortonBucketBits && ((int64_t)1 << hbits) < 2 * nt) ++hbits;
    const int64_t nbuckets = (int64_t)1 << hbits;
    const int64_t ecap = (int64_t)kHashEntriesPerTri * c->lim.max_tris;
    int32_t* hist = wsp<int32_t>(c, L.bvh_hist);
    int32_t* offset = wsp<int32_t>(c, L.bvh_offset);
    uint64_t* key = wsp<uint64_t>(c, L.hash_key);
    int32_t* tri = wsp<int32_t>(c, L.hash_tri);
    uint64_t* skey = wsp<uint64_t>(c, L.hash_skey);
    int32_t* stri = wsp<int32_t>(c, L.hash_stri);
    HashGrid* grid = wsp<HashGrid>(c, L.hash_grid);
    stage_begin(c, TTIE_STAGE_BP_BOXES, s);
    k_tri_boxes<<<gb, kBpBlock, 0, s>>>(m->x, x_end, m->n_verts, m->tris, nt, tbox, wsp<float>(c, L.bvh_centroid),
                                        wsp<uint32_t>(c, L.bvh_part), wsp<double>(c, L.bvh_ext), npairs, ctr);
    k_hash_cells<<<bp_grid(nt), kBpBlock, 0, s>>>(tbox, nt, wsp<uint32_t>(c, L.bvh_part), wsp<double>(c, L.bvh_ext),
                                                  (int)gb, hbits, hist, key, tri, wsp<int32_t>(c, L.hash_rank), ecap,
                                                  grid, ctr);
    stage_end(c, TTIE_STAGE_BP_BOXES, s);
    stage_begin(c, TTIE_STAGE_BP_SORT, s);
    hipError_t e = launch_scan_i32(c, hist, offset, nbuckets, s);
    if (e != hipSuccess) return e;
    k_hash_scatter<<<bp_grid(std::max<int64_t>(4 * nt, nbuckets)), kBpBlock, 0, s>>>(
        ctr, ecap, nbuckets, hbits, key, tri, wsp<int32_t>(c, L.hash_rank), offset, skey, stri, hist);
    stage_end(c, TTIE_STAGE_BP_SORT, s);
    stage_begin(c, TTIE_STAGE_BP_TRAVERSE, s);
    int32_t* heavy = wsp<int32_t>(c, L.hash_rank);  // the ranks are consumed by the scatter
    const int hb = (int)ctx_param(c, TTIE_PARAM_HASH_BUDGET);
    k_hash_pairs<<<bp_grid(4 * nt, 8192), kBpBlock, 0, s>>>(ctr, ecap, nbuckets, hbits, offset, skey, stri, tbox,
                                                           m->tris, grid, hb, va, heavy, pairs, capacity, npairs, ctr);
    stage_end(c, TTIE_STAGE_BP_TRAVERSE, s);
    stage_begin(c, TTIE_STAGE_BP_HEAVY, s);
    k_hash_heavy<<<512, kBpBlock, 0, s>>>(ctr, ecap, nbuckets, hbits, offset, skey, stri, tbox, m->tris, grid, hb, va,
                                          heavy, pairs, capacity, npairs, ctr);
    stage_end(c, TTIE_STAGE_BP_HEAVY, s);
  } else if (method == TTIE_BROAD_LBVH && nt >= 2) {
    double* tbox = wsp<double>(c, L.bvh_tbox);
    float* centre = wsp<float>(c, L.bvh_centroid);
    uint32_t* k1 = wsp<uint32_t>(c, L.bvh_keys);
    int32_t* v1 = wsp<int32_t>(c, L.bvh_vals);
    int32_t* v2 = wsp<int32_t>(c, L.bvh_vals2);
    Box32* boxes = wsp<Box32>(c, L.bvh_boxes);
    LeafRec* leaves = wsp<LeafRec>(c, L.bvh_leaves);
    int32_t* qend = wsp<int32_t>(c, L.bvh_qend);
    const Levels lv = make_levels(nt);
    stage_begin(c, TTIE_STAGE_BP_BOXES, s);
    const unsigned gb = bp_grid(nt, kBoundsBlocks);
    // buckets: about two triangles per bucket; a batch spends the top bits on the problem
    int bits = 8;
    while (bits < kMortonBucketBits && ((int64_t)1 << (bits + 1)) <= nt) ++bits;
    int pbits = 0;
    if (!tri_off) n_prob = 1;
    while ((1 << pbits) < n_prob) ++pbits;
    const int mbits = std::min(std::max(bits - pbits, 3), kMortonBucketBits - pbits);
    const int64_t nbuckets = (int64_t)1 << (pbits + mbits);
    int32_t* hist = wsp<int32_t>(c, L.bvh_hist);
    int32_t* offset = wsp<int32_t>(c, L.bvh_offset);
    k_tri_boxes<<<gb, kBpBlock, 0, s>>>(m->x, x_end, m->n_verts, m->tris, nt, tbox, centre,
                                        wsp<uint32_t>(c, L.bvh_part), wsp<double>(c, L.bvh_ext), npairs, ctr);
    k_morton<<<bp_grid(nt), kBpBlock, 0, s>>>(centre, nt, wsp<uint32_t>(c, L.bvh_part), (int)gb, tri_off, n_prob,
                                              mbits, hist, k1, v1, ctr);
    stage_end(c, TTIE_STAGE_BP_BOXES, s);
    stage_begin(c, TTIE_STAGE_BP_SORT, s);
    hipError_t e = launch_scan_i32(c, hist, offset, nbuckets, s);
    if (e != hipSuccess) return e;
    k_scatter<<<bp_grid(std::max<int64_t>(nt, nbuckets)), kBpBlock, 0, s>>>(nt, nbuckets, k1, v1, offset, v2, hist);
    stage_end(c, TTIE_STAGE_BP_SORT, s);
    stage_begin(c, TTIE_STAGE_BP_BUILD, s);
    // leaves to level 4 in blocks of 256, then five levels per launch in blocks of 1024 (a
    // tree of up to 4^9 leaves takes two launches)
    for (int l0 = 0; l0 < lv.L; l0 += l0 == 0 ? 4 : 5) {
      if (l0 == 0)
        k_levels<256><<<(unsigned)((lv.m[0] + 255) / 256), 256, 0, s>>>(0, lv, tbox, v2, m->tris, boxes, leaves,
                                                                         tri_off, n_prob, mbits, offset, qend);
      else
        k_levels<1024><<<(unsigned)((lv.m[l0] + 1023) / 1024), 1024, 0, s>>>(l0, lv, tbox, v2, m->tris, boxes, leaves,
                                                                             tri_off, n_prob, mbits, offset, qend);
    }
    stage_end(c, TTIE_STAGE_BP_BUILD, s);
    stage_begin(c, TTIE_STAGE_BP_TRAVERSE, s);
    // one lane per leaf, block count rounded up to a multiple of the 8 XCDs
    const int64_t nb = ((nt + kBpBlock - 1) / kBpBlock + 7) / 8 * 8;
    TravState* heavy = wsp<TravState>(c, L.bvh_heavy);
    const int64_t heavy_cap = (int64_t)(L.bvh_heavy_bytes / sizeof(TravState));
    const int budget = (int)ctx_param(c, TTIE_PARAM_TRAV_BUDGET);
    if (va)
      k_traverse<true><<<(unsigned)nb, kTravThreads, 0, s>>>(nt, lv, boxes, leaves, tri_off ? qend : nullptr, heavy,
                                                             heavy_cap, budget, pairs, capacity, npairs, ctr);
    else
      k_traverse<false><<<(unsigned)nb, kTravThreads, 0, s>>>(nt, lv, boxes, leaves, tri_off ? qend : nullptr, heavy,
                                                              heavy_cap, budget, pairs, capacity, npairs, ctr);
    stage_end(c, TTIE_STAGE_BP_TRAVERSE, s);
    stage_begin(c, TTIE_STAGE_BP_HEAVY, s);
    k_traverse_heavy<<<1024, 64, 0, s>>>(lv, boxes, leaves, heavy, heavy_cap, va, heavy_batch(lv.L), pairs, capacity,
                                         npairs, ctr);
    stage_end(c, TTIE_STAGE_BP_HEAVY, s);
  }
  return hipGetLastError();
}

}  // namespace ttie
