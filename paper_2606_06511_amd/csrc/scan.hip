// Exclusive prefix sum of int32 counts in one launch: a decoupled look-back scan.
//
// Each block takes the next tile of 2048 entries from a counter (so every tile a block waits
// on belongs to a block that is already running), scans it in registers and LDS, publishes
// its aggregate, walks back over its predecessors' published words until it meets an
// inclusive prefix, and publishes its own inclusive prefix.  A published word holds the flag
// and the value together and is written and read with device-scope atomics, so the look-back
// needs no fence.  The last block to finish (counted with a release-acquire atomic, which orders
// each block's final word before its count) clears the tile words and both counters, so the state is
// zero before every scan without a separate initialisation launch, and a captured graph can
// replay the scan.  A predecessor publishes its aggregate before its own look-back, so a wait
// lasts microseconds; the waits are still bounded, and one that outlasts the bound latches
// STATUS_INTERNAL and lets the kernel finish.
#include "internal.h"

namespace ttie {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr uint32_t kSpinCap = 1u << 16;  // polls of one predecessor word (tens of ms at most)
constexpr uint64_t kAggregate = 1, kInclusive = 2;

__device__ __forceinline__ uint64_t word_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void word_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t make_word(uint64_t flag, int32_t v) { return flag << 32 | (uint32_t)v; }

__global__ void __launch_bounds__(kScanThreads) k_scan_i32(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                           int64_t n, ScanState* st, uint64_t* words,
                                                           int32_t* status_word) {
  __shared__ int32_t s_wave[kScanThreads / 64];
  __shared__ uint32_t s_tile;
  __shared__ int32_t s_excl;
  __shared__ int s_last;
  if (threadIdx.x == 0) s_tile = atomicAdd(&st->next_tile, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const int64_t base = (int64_t)tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) v[j] = base + j < n ? in[base + j] : 0;
  // exclusive within the thread
  int32_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int32_t t = v[j];
    v[j] = run;
    run += t;
  }
  // inclusive across the wave, then across the block's waves
  const int lane = __lane_id(), wave = threadIdx.x / 64;
  int32_t inc = run;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  int32_t wave_excl = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    wave_excl += w < wave ? s_wave[w] : 0;
    agg += s_wave[w];
  }
  const int32_t thread_excl = wave_excl + inc - run;
  if (wave == 0) {
    // wave-parallel look-back: lane k reads the word of tile p0 - k (a virtual inclusive 0
    // below tile 0), waits until every lane's word is published, then adds the values up to
    // and including the nearest inclusive prefix; without one in the window, it adds all 64
    // aggregates and moves the window down
    int32_t excl = 0;
    if (tile == 0) {
      if (lane == 0) word_store(&words[0], make_word(kInclusive, agg));
    } else {
      if (lane == 0) word_store(&words[tile], make_word(kAggregate, agg));
      for (int64_t p0 = (int64_t)tile - 1;; p0 -= 64) {
        const int64_t p = p0 - lane;
        uint64_t w = p >= 0 ? word_load(&words[p]) : make_word(kInclusive, 0);
        uint64_t incl;
        int first;
        for (uint32_t spins = 0;; ++spins) {
          // only the lanes up to the nearest published inclusive prefix are needed
          incl = __ballot((w >> 32) == kInclusive);
          first = incl ? __builtin_ctzll(incl) : 63;
          const uint64_t need = first == 63 ? ~0ull : (2ull << first) - 1;
          if (!(__ballot((w >> 32) == 0) & need)) break;
          if (spins == kSpinCap) {
            if (lane == 0) atomicCAS(status_word, 0, (int32_t)STATUS_INTERNAL);  // the first error wins
            if ((w >> 32) == 0) w = make_word(kInclusive, 0);
            continue;  // every lane is published now: the next pass leaves the loop
          }
          __builtin_amdgcn_s_sleep(1);
          if ((w >> 32) == 0) w = word_load(&words[p]);
        }
        int32_t add = lane <= first ? (int32_t)(uint32_t)w : 0;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) add += __shfl_xor(add, d);
        excl += add;
        if (incl) break;
      }
      if (lane == 0) word_store(&words[tile], make_word(kInclusive, excl + agg));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  const int32_t pre = s_excl + thread_excl;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) out[base + j] = pre + v[j];
  // the last block to finish clears the tile words and the counters for the next scan (every
  // other block has finished its look-back before counting itself done).  The count is taken
  // with release-acquire ordering at device scope: the tile word this thread stored above is
  // then visible before the count, so the last block's clearing comes after every block's final
  // store and no stale word survives into the next scan.
  if (threadIdx.x == 0)
    s_last = __hip_atomic_fetch_add(&st->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  for (int64_t t = threadIdx.x; t < (int64_t)gridDim.x; t += kScanThreads) word_store(&words[t], 0);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&st->next_tile, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Long scans in three launches (tile sums, one block scanning them, each tile's scan from its
// prefix): the look-back above hands each tile's prefix on through device-scope words that
// travel between the XCDs' L2s, which set its pace on long inputs (0.17 ms for 2^22 entries);
// the three passes stream the input twice at full width instead.
__global__ void __launch_bounds__(kScanThreads) k_scan_tile_sums(const int32_t* __restrict__ in, int64_t n,
                                                                 int32_t* __restrict__ tsum) {
  __shared__ int32_t s_wave[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) run += base + j < n ? in[base + j] : 0;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) run += __shfl_xor(run, d);
  if (__lane_id() == 0) s_wave[threadIdx.x / 64] = run;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) t += s_wave[w];
    tsum[blockIdx.x] = t;
  }
}

// one block: exclusive scan of the tile sums in place (each thread a contiguous run of them)
__global__ void __launch_bounds__(1024) k_scan_tile_prefix(int32_t* __restrict__ tsum, int64_t tiles) {
  __shared__ int32_t s_wave[16];
  const int64_t per = (tiles + 1023) / 1024;
  const int64_t b = (int64_t)threadIdx.x * per, e = std::min<int64_t>(tiles, b + per);
  int32_t run = 0;
  for (int64_t i = b; i < e; ++i) run += tsum[i];
  const int lane = __lane_id(), wave = threadIdx.x / 64;
  int32_t inc = run;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  int32_t excl = inc - run;
  for (int w = 0; w < wave; ++w) excl += s_wave[w];
  for (int64_t i = b; i < e; ++i) {
    const int32_t t = tsum[i];
    tsum[i] = excl;
    excl += t;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tile_apply(const int32_t* __restrict__ in,
                                                                  int32_t* __restrict__ out, int64_t n,
                                                                  const int32_t* __restrict__ tsum) {
  __shared__ int32_t s_wave[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) v[j] = base + j < n ? in[base + j] : 0;
  int32_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int32_t t = v[j];
    v[j] = run;
    run += t;
  }
  const int lane = __lane_id(), wave = threadIdx.x / 64;
  int32_t inc = run;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  int32_t pre = tsum[blockIdx.x] + inc - run;
  for (int w = 0; w < wave; ++w) pre += s_wave[w];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) out[base + j] = pre + v[j];
}

// tiles from which the three-launch form is used
constexpr int64_t kLongScanTiles = 256;

}  // namespace

// counters, then a look-back word and a tile sum per tile (separate arrays: the words must stay
// zero between one-launch scans)
size_t scan_temp_bytes(int64_t n) {
  const int64_t tiles = (std::max<int64_t>(n, 1) + kScanTile - 1) / kScanTile;
  return 256 + (size_t)tiles * (sizeof(uint64_t) + sizeof(int32_t));
}

hipError_t launch_scan_i32(Ctx* c, const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (scan_temp_bytes(n) > c->L.scan_tmp_bytes) return hipErrorInvalidValue;
  char* base = c->ws + c->L.scan_tmp;
  if (tiles >= kLongScanTiles) {
    // the tile sums after the words of the most tiles the region holds
    const int64_t tiles_cap = (int64_t)(c->L.scan_tmp_bytes - 256) / (int64_t)(sizeof(uint64_t) + sizeof(int32_t));
    int32_t* tsum = reinterpret_cast<int32_t*>(base + 256 + tiles_cap * sizeof(uint64_t));
    k_scan_tile_sums<<<(unsigned)tiles, kScanThreads, 0, s>>>(in, n, tsum);
    k_scan_tile_prefix<<<1, 1024, 0, s>>>(tsum, tiles);
    k_scan_tile_apply<<<(unsigned)tiles, kScanThreads, 0, s>>>(in, out, n, tsum);
    return hipGetLastError();
  }
  k_scan_i32<<<(unsigned)tiles, kScanThreads, 0, s>>>(in, out, n, reinterpret_cast<ScanState*>(base),
                                                      reinterpret_cast<uint64_t*>(base + 256),
                                                      &reinterpret_cast<Counters*>(c->ws + c->L.counters)->status);
  return hipGetLastError();
}

}  // namespace ttie
