// Broad phase: candidate triangle pairs for the per-pair energy (Sec. 1.2 removes redundant
// pair tests with a spatial structure; this is a linear BVH).
//
//   k_bp_init      reset the pair counter and the scene bounds
//   k_tri_boxes    exact FP64 bounding box per triangle; centroid bounds (order-preserving
//                  integer atomics, so the result does not depend on the order)
//   k_morton       30-bit Morton code of each box centre
//   radix sort     (code, triangle) pairs by code (rocPRIM), stable
//   k_build        binary radix tree over the sorted codes (Karras 2012): every internal node
//                  finds its key range from common-prefix lengths; equal codes are split by
//                  position, so the tree exists for any input
//   k_refit        bottom-up FP32 node boxes, rounded outwards from the FP64 leaf boxes; the
//                  second child to arrive at a node builds it
//   k_traverse     one lane per leaf, depth-first over the tree, reporting only leaves after
//                  itself in sorted order (every unordered pair once); a leaf is confirmed by
//                  the exact closed FP64 box test and the shared-vertex test; pairs are
//                  appended with one atomic per wave (ballot + popcount)
//   k_brute        all i < j without a shared vertex (no box test)
#include <rocprim/device/device_radix_sort.hpp>

#include "internal.h"

namespace ttie {

constexpr int kBpBlock = 256;
constexpr int32_t kLeafBit = (int32_t)0x80000000;
constexpr int kStack = 64;

__device__ __forceinline__ uint32_t f2key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void k_bp_init(Counters* c) {
  if (threadIdx.x == 0) {
    c->n_pairs = 0;
    for (int k = 0; k < 3; ++k) {
      c->bounds[k] = 0xffffffffu;  // running minimum
      c->bounds[3 + k] = 0u;       // running maximum
    }
  }
}

__global__ void __launch_bounds__(kBpBlock) k_tri_boxes(const double* __restrict__ x, int64_t nv,
                                                        const int32_t* __restrict__ tris, int64_t nt,
                                                        double* __restrict__ tbox, float* __restrict__ centre,
                                                        Counters* ctr) {
  __shared__ uint32_t smin[3][kBpBlock], smax[3][kBpBlock];
  uint32_t lmin[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, lmax[3] = {0u, 0u, 0u};
  bool bad = false;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      const int32_t v = tris[3 * t + k];
      if (v < 0 || v >= nv) {
        ok = false;
        break;
      }
      for (int c = 0; c < 3; ++c) {
        const double q = x[3 * (int64_t)v + c];
        lo[c] = k == 0 ? q : fmin(lo[c], q);
        hi[c] = k == 0 ? q : fmax(hi[c], q);
      }
    }
    if (!ok) bad = true;
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
  __syncthreads();
  for (int w = kBpBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 3; ++c) {
        smin[c][threadIdx.x] = min(smin[c][threadIdx.x], smin[c][threadIdx.x + w]);
        smax[c][threadIdx.x] = max(smax[c][threadIdx.x], smax[c][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) {
      atomicMin(&ctr->bounds[c], smin[c][0]);
      atomicMax(&ctr->bounds[3 + c], smax[c][0]);
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

__global__ void __launch_bounds__(kBpBlock) k_morton(const float* __restrict__ centre, int64_t nt, const Counters* ctr,
                                                     uint32_t* __restrict__ keys, int32_t* __restrict__ vals) {
  float lo[3], inv[3];
  for (int c = 0; c < 3; ++c) {
    lo[c] = key2f(ctr->bounds[c]);
    const float ext = key2f(ctr->bounds[3 + c]) - lo[c];
    inv[c] = ext > 0.f ? 1023.f / ext : 0.f;
  }
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
    uint32_t q[3];
    for (int c = 0; c < 3; ++c) {
      const float f = (centre[3 * t + c] - lo[c]) * inv[c];
      q[c] = (uint32_t)fminf(fmaxf(f, 0.f), 1023.f);
    }
    keys[t] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    vals[t] = (int32_t)t;
  }
}

// length of the common prefix of sorted keys i and j (positions break ties); -1 outside
__device__ __forceinline__ int prefix(const uint32_t* keys, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const uint32_t a = keys[i], b = keys[j];
  if (a == b) return 32 + __clz((uint32_t)(i ^ j));
  return __clz(a ^ b);
}

__global__ void __launch_bounds__(kBpBlock) k_build(const uint32_t* __restrict__ keys, int n, int32_t* __restrict__ left,
                                                    int32_t* __restrict__ right, int32_t* __restrict__ first,
                                                    int32_t* __restrict__ last, int32_t* __restrict__ parent,
                                                    int32_t* __restrict__ leafparent, int32_t* __restrict__ visit) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n - 1; i += gridDim.x * blockDim.x) {
    // direction of the node's range: towards the neighbour sharing the longer prefix
    const int d = prefix(keys, n, i, i + 1) > prefix(keys, n, i, i - 1) ? 1 : -1;
    const int dmin = prefix(keys, n, i, i - d);
    int lmax = 2;
    while (prefix(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
      if (prefix(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix(keys, n, i, j);
    // split: the last position sharing more than dnode bits with i
    int s = 0, t = l;
    do {
      t = (t + 1) >> 1;
      if (prefix(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int g = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    const int32_t lc = lo == g ? (g | kLeafBit) : g;
    const int32_t rc = hi == g + 1 ? ((g + 1) | kLeafBit) : g + 1;
    left[i] = lc;
    right[i] = rc;
    first[i] = lo;
    last[i] = hi;
    visit[i] = 0;
    if (lc & kLeafBit) leafparent[lc & ~kLeafBit] = i; else parent[lc] = i;
    if (rc & kLeafBit) leafparent[rc & ~kLeafBit] = i; else parent[rc] = i;
    if (i == 0) parent[0] = -1;
  }
}

__global__ void __launch_bounds__(kBpBlock) k_refit(const double* __restrict__ tbox, const int32_t* __restrict__ ids,
                                                    int n, const int32_t* __restrict__ left,
                                                    const int32_t* __restrict__ right,
                                                    const int32_t* __restrict__ parent,
                                                    const int32_t* __restrict__ leafparent, int32_t* visit,
                                                    float* leafbox, float* nodebox, Counters* ctr) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    const int64_t t = ids[s];
    for (int c = 0; c < 3; ++c) {
      leafbox[6 * s + c] = __double2float_rd(tbox[6 * t + c]);
      leafbox[6 * s + 3 + c] = __double2float_ru(tbox[6 * t + 3 + c]);
    }
    __threadfence();
    int node = leafparent[s];
    // a radix tree over 62-bit keys is at most 63 levels deep; the cap only guards a
    // malformed tree from looping
    for (int level = 0; node >= 0; ++level) {
      if (level > 2 * kStack) {
        atomicCAS(&ctr->status, 0, STATUS_CAPACITY);
        break;
      }
      if (atomicAdd(&visit[node], 1) == 0) break;  // first child to arrive: the sibling finishes
      __threadfence();
      const int32_t lc = left[node], rc = right[node];
      const float* bl = (lc & kLeafBit) ? leafbox + 6 * (lc & ~kLeafBit) : nodebox + 6 * lc;
      const float* br = (rc & kLeafBit) ? leafbox + 6 * (rc & ~kLeafBit) : nodebox + 6 * rc;
      for (int c = 0; c < 3; ++c) {
        nodebox[6 * node + c] = fminf(__builtin_nontemporal_load(bl + c), __builtin_nontemporal_load(br + c));
        nodebox[6 * node + 3 + c] =
            fmaxf(__builtin_nontemporal_load(bl + 3 + c), __builtin_nontemporal_load(br + 3 + c));
      }
      __threadfence();
      node = parent[node];
    }
  }
}

__device__ __forceinline__ bool overlap32(const float q[6], const float* b) {
  return q[0] <= b[3] && b[0] <= q[3] && q[1] <= b[4] && b[1] <= q[4] && q[2] <= b[5] && b[2] <= q[5];
}

// wave-aggregated append of (a, b) pairs: one atomic per wave
__device__ __forceinline__ void emit_pair(bool want, int32_t a, int32_t b, int32_t* pairs, int64_t cap, Counters* ctr) {
  const uint64_t mask = __ballot(want);
  if (!mask) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(&ctr->n_pairs, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  if (want) {
    const int64_t slot = (int64_t)base + __popcll(mask & ((1ull << lane) - 1ull));
    if (slot < cap) {
      pairs[2 * slot] = min(a, b);
      pairs[2 * slot + 1] = max(a, b);
    }
  }
}

__global__ void __launch_bounds__(kBpBlock) k_traverse(int n, const int32_t* __restrict__ tris,
                                                       const double* __restrict__ tbox, const int32_t* __restrict__ ids,
                                                       const float* __restrict__ leafbox,
                                                       const float* __restrict__ nodebox,
                                                       const int32_t* __restrict__ left,
                                                       const int32_t* __restrict__ right,
                                                       const int32_t* __restrict__ last, int32_t* pairs, int64_t cap,
                                                       Counters* ctr) {
  int status = 0;
  for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const int s = base + threadIdx.x;
    const bool live = s < n;
    float q[6];
    int32_t t = 0, vt[3] = {-1, -1, -1};
    double qb[6];
    int stack[kStack];
    int sp = 0;
    if (live) {
      t = ids[s];
      for (int c = 0; c < 6; ++c) {
        q[c] = leafbox[6 * s + c];
        qb[c] = tbox[6 * (int64_t)t + c];
      }
      for (int k = 0; k < 3; ++k) vt[k] = tris[3 * (int64_t)t + k];
      if (s < n - 1) stack[sp++] = 0;  // the root covers every leaf; skip if s is the last
    }
    // every lane runs the loop until the whole wave is done, so the ballots converge; a lane
    // visits each internal node at most once, so n iterations bound a well-formed tree
    for (int iter = 0; __ballot(sp > 0); ++iter) {
      if (iter > n + kStack) {
        status = STATUS_CAPACITY;
        break;
      }
      int node = -1;
      if (sp > 0) node = stack[--sp];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        bool want = false;
        int32_t t2 = 0;
        if (node >= 0) {
          const int32_t ch = side == 0 ? left[node] : right[node];
          if (ch & kLeafBit) {
            const int pos = ch & ~kLeafBit;
            if (pos > s && overlap32(q, leafbox + 6 * pos)) {
              t2 = ids[pos];
              const double* b = tbox + 6 * (int64_t)t2;
              bool ov = true;
              for (int c = 0; c < 3; ++c) ov = ov && qb[c] <= b[3 + c] && b[c] <= qb[3 + c];
              bool adj = false;
              for (int k = 0; k < 3; ++k) {
                const int32_t w = tris[3 * (int64_t)t2 + k];
                adj |= w == vt[0] || w == vt[1] || w == vt[2];
              }
              want = ov && !adj;
            }
          } else if (last[ch] > s && overlap32(q, nodebox + 6 * ch)) {
            if (sp < kStack) stack[sp++] = ch;
            else status = STATUS_CAPACITY;
          }
        }
        emit_pair(want, t, t2, pairs, cap, ctr);
      }
    }
  }
  if (status) atomicCAS(&ctr->status, 0, status);
}

__global__ void __launch_bounds__(kBpBlock) k_brute(const int32_t* __restrict__ tris, int64_t nt, int32_t* pairs,
                                                    int64_t cap, Counters* ctr) {
  for (int64_t i = blockIdx.y; i < nt; i += gridDim.y) {
    int32_t vi[3];
    for (int k = 0; k < 3; ++k) vi[k] = tris[3 * i + k];
    for (int64_t jb = (int64_t)blockIdx.x * blockDim.x; jb < nt; jb += (int64_t)gridDim.x * blockDim.x) {
      const int64_t j = jb + threadIdx.x;
      bool want = false;
      if (j > i && j < nt) {
        bool adj = false;
        for (int k = 0; k < 3; ++k) {
          const int32_t w = tris[3 * j + k];
          adj |= w == vi[0] || w == vi[1] || w == vi[2];
        }
        want = !adj;
      }
      emit_pair(want, (int32_t)i, (int32_t)j, pairs, cap, ctr);
    }
  }
}

__global__ void k_bp_finish(Counters* ctr, int64_t cap, int64_t* n_pairs) {
  if (threadIdx.x == 0) {
    const uint32_t np = ctr->n_pairs;
    *n_pairs = (int64_t)np;
    if ((int64_t)np > cap) atomicCAS(&ctr->status, 0, STATUS_CAPACITY);
  }
}

size_t sort_temp_bytes(int64_t n) {
  size_t bytes = 0;
  uint32_t* k = nullptr;
  int32_t* v = nullptr;
  if (rocprim::radix_sort_pairs(nullptr, bytes, k, k, v, v, (unsigned)n, 0, 30) != hipSuccess) return 0;
  return bytes;
}

static unsigned bp_grid(int64_t n, unsigned cap = 4096) {
  int64_t g = (n + kBpBlock - 1) / kBpBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_broadphase(Ctx* c, const ttie_mesh* m, int method, int32_t* pairs, int64_t capacity,
                             int64_t* n_pairs, hipStream_t s) {
  const Layout& L = c->L;
  Counters* ctr = wsp<Counters>(c, L.counters);
  const int64_t nt = m->n_tris;
  k_bp_init<<<1, 64, 0, s>>>(ctr);
  if (method == TTIE_BROAD_BRUTE) {
    dim3 grid(bp_grid(nt, 64), (unsigned)(nt < 8192 ? (nt > 0 ? nt : 1) : 8192));
    stage_begin(c, TTIE_STAGE_BP_TRAVERSE, s);
    k_brute<<<grid, kBpBlock, 0, s>>>(m->tris, nt, pairs, capacity, ctr);
    stage_end(c, TTIE_STAGE_BP_TRAVERSE, s);
  } else if (nt >= 2) {
    double* tbox = wsp<double>(c, L.bvh_tbox);
    float* centre = wsp<float>(c, L.bvh_centroid);
    uint32_t* k1 = wsp<uint32_t>(c, L.bvh_keys);
    uint32_t* k2 = wsp<uint32_t>(c, L.bvh_keys2);
    int32_t* v1 = wsp<int32_t>(c, L.bvh_vals);
    int32_t* v2 = wsp<int32_t>(c, L.bvh_vals2);
    int32_t* nodes = wsp<int32_t>(c, L.bvh_nodes);
    const int n = (int)nt;
    int32_t *left = nodes, *right = nodes + n, *first = nodes + 2 * (int64_t)n, *last = nodes + 3 * (int64_t)n,
            *parent = nodes + 4 * (int64_t)n;
    int32_t* leafparent = wsp<int32_t>(c, L.bvh_leafparent);
    int32_t* visit = wsp<int32_t>(c, L.bvh_visit);
    float* boxes = wsp<float>(c, L.bvh_boxes);
    float* nodebox = boxes;
    float* leafbox = boxes + 6 * (int64_t)n;
    stage_begin(c, TTIE_STAGE_BP_BOXES, s);
    k_tri_boxes<<<bp_grid(nt, 1024), kBpBlock, 0, s>>>(m->x, m->n_verts, m->tris, nt, tbox, centre, ctr);
    k_morton<<<bp_grid(nt), kBpBlock, 0, s>>>(centre, nt, ctr, k1, v1);
    stage_end(c, TTIE_STAGE_BP_BOXES, s);
    size_t bytes = L.bvh_sort_tmp_bytes;
    stage_begin(c, TTIE_STAGE_BP_SORT, s);
    hipError_t e = rocprim::radix_sort_pairs(c->ws + L.bvh_sort_tmp, bytes, k1, k2, v1, v2, (unsigned)n, 0, 30, s);
    stage_end(c, TTIE_STAGE_BP_SORT, s);
    if (e != hipSuccess) return e;
    stage_begin(c, TTIE_STAGE_BP_BUILD, s);
    k_build<<<bp_grid(n - 1), kBpBlock, 0, s>>>(k2, n, left, right, first, last, parent, leafparent, visit);
    k_refit<<<bp_grid(n), kBpBlock, 0, s>>>(tbox, v2, n, left, right, parent, leafparent, visit, leafbox, nodebox,
                                             ctr);
    stage_end(c, TTIE_STAGE_BP_BUILD, s);
    stage_begin(c, TTIE_STAGE_BP_TRAVERSE, s);
    k_traverse<<<bp_grid(n), kBpBlock, 0, s>>>(n, m->tris, tbox, v2, leafbox, nodebox, left, right, last, pairs,
                                                capacity, ctr);
    stage_end(c, TTIE_STAGE_BP_TRAVERSE, s);
  }
  k_bp_finish<<<1, 64, 0, s>>>(ctr, capacity, n_pairs);
  return hipGetLastError();
}

}  // namespace ttie
