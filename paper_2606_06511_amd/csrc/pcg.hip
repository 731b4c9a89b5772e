// Jacobi-preconditioned conjugate gradients on (H + mu I) x = scale * b for the inexact
// Newton consumer, with H the BSR Hessian of ttie_eval.  Everything stays on the device: the
// scalars of the iteration are reduced from fixed-size per-block partials (fixed order, so
// the result is deterministic), every kernel re-derives them from the previous kernel's
// partials, and a convergence flag written by one kernel turns the remaining launches into
// no-ops.  Three launches per iteration:
//   k_pcg_matvec  q = (H + mu I) p, partials of p.q
//   k_pcg_update  alpha = r.z / p.q; x += alpha p; r -= alpha q; z = D^-1 r; partials r.z, r.r
//   k_pcg_dir     beta = r.z(new) / r.z(old); p = z + beta p; convergence test
//
// Active rows.  H is zero outside the rows that hold blocks (those the hits touch), so there
// (H + mu I) is mu I; with b = 0 on those rows the residual, the search direction and the
// solution stay exactly 0 on them for the whole iteration.  The solve therefore runs over the
// list of active rows only (built once per solve, in row order, so the sums keep a fixed
// order), and b must vanish elsewhere: a Newton gradient does.  On a mesh of millions of
// vertices with tens of thousands touched this makes each iteration a few microseconds.
#include "internal.h"

namespace ttie {

constexpr int kPB = 256;  // threads per block (and the number of blocks)

struct PcgState {
  double mu, bb, rz, rr;
  int32_t done, iters;
};

// fixed-order sum over the kPB per-block partials of slot `slot` (every block computes it)
__device__ __forceinline__ double grid_sum(const double* __restrict__ part, int slot, double* red) {
  red[threadIdx.x] = part[4 * threadIdx.x + slot];
  __syncthreads();
  for (int w = kPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double v = red[0];
  __syncthreads();
  return v;
}

// block sums of up to two values into this block's partial slots
__device__ __forceinline__ void block_partials(double v0, double v1, double* __restrict__ part, double* red) {
  red[threadIdx.x] = v0;
  __syncthreads();
  for (int w = kPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[4 * blockIdx.x] = red[0];
  __syncthreads();
  red[threadIdx.x] = v1;
  __syncthreads();
  for (int w = kPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[4 * blockIdx.x + 1] = red[0];
}

// diagonal block of row r (columns are sorted), or -1
__device__ __forceinline__ int64_t diag_block(const int32_t* row_ptr, const int32_t* col_idx, int64_t r) {
  int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int32_t c = col_idx[mid];
    if (c == r) return mid;
    if (c < r) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}


// ---- the active rows ------------------------------------------------------------------------
// flag[v] = row v holds blocks (row_ptr) or incidences of the last evaluation's hits; x, p = 0
// on every row; a non-zero b on an inactive row latches STATUS_INVALID.  Row n's flag is 0 (the
// scan's total).  With off, each vertex's range in the evaluation's incidence lists is written
// there too: off[v] = roff[number of touched vertices below v] for v in [0, n] (the touched
// vertices are the rows, in vertex order, and roff their list starts), so that the range of v
// is [off[v], off[v + 1]), empty when no hit touches v.
template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_flags(int64_t n, const int32_t* __restrict__ row_ptr,
                                                   const uint32_t* __restrict__ bm, const uint32_t* __restrict__ wp,
                                                   const int32_t* __restrict__ roff, int32_t* __restrict__ off,
                                                   const S* __restrict__ b, S* __restrict__ x, S* __restrict__ p,
                                                   int32_t* __restrict__ flag, Counters* ctr) {
  for (int64_t v = (int64_t)blockIdx.x * kPB + threadIdx.x; v <= n; v += (int64_t)gridDim.x * kPB) {
    bool touched = false;
    if (off) {
      const int64_t w = v >> 5;
      const uint32_t word = bm[w], j = (uint32_t)v & 31u;
      off[v] = roff[wp[w] + (uint32_t)__popc(word & ((1u << j) - 1u))];
      touched = (word >> j) & 1u;
    }
    if (v == n) {
      flag[n] = 0;
      continue;
    }
    const bool act = (row_ptr && row_ptr[v + 1] > row_ptr[v]) || touched;
    flag[v] = act ? 1 : 0;
    bool nz = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * v + c] = (S)0.0;
      p[3 * v + c] = (S)0.0;
      nz |= (double)b[3 * v + c] != 0.0;
    }
    if (!act && nz) atomicCAS(&ctr->status, 0, STATUS_INVALID);
  }
}

__global__ void __launch_bounds__(kPB) k_pcg_compact(int64_t n, const int32_t* __restrict__ flag,
                                                     const int32_t* __restrict__ pos, int32_t* __restrict__ act) {
  for (int64_t v = (int64_t)blockIdx.x * kPB + threadIdx.x; v < n; v += (int64_t)gridDim.x * kPB)
    if (flag[v]) act[pos[v]] = (int32_t)v;
}

// the list of active rows and its device count (pos[n])
struct Active {
  const int32_t* rows;
  const int32_t* count;
};

template <class S>
static hipError_t pcg_active(Ctx* c, int64_t n, const int32_t* row_ptr, int32_t* off, const S* b, S* x, S* p,
                             Active& a, hipStream_t s) {
  const Layout& L = c->L;
  int32_t* flag = wsp<int32_t>(c, L.pcg_flag);
  int32_t* pos = wsp<int32_t>(c, L.pcg_pos);
  int32_t* act = wsp<int32_t>(c, L.pcg_act);
  Counters* ctr = wsp<Counters>(c, L.counters);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 1 + kPB - 1) / kPB));
  k_pcg_flags<S><<<g, kPB, 0, s>>>(n, row_ptr, wsp<uint32_t>(c, L.bm), wsp<uint32_t>(c, L.wp), wsp<int32_t>(c, L.roff),
                                   off, b, x, p, flag, ctr);
  hipError_t e = launch_scan_i32(c, flag, pos, n + 1, s);
  if (e != hipSuccess) return e;
  k_pcg_compact<<<g, kPB, 0, s>>>(n, flag, pos, act);
  a.rows = act;
  a.count = pos + n;
  return hipGetLastError();
}

#define PCG_ROWS(j, i, a)                                                                          \
  const int64_t na_ = *(a).count;                                                                  \
  for (int64_t j = (int64_t)blockIdx.x * kPB + threadIdx.x; j < na_; j += (int64_t)gridDim.x * kPB)

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_diag(Active a, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx, const S* __restrict__ vals,
                                                  double* __restrict__ part) {
  __shared__ double red[kPB];
  double sum = 0.0, cnt = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t r = a.rows[j];
    const int64_t d = diag_block(row_ptr, col_idx, r);
    if (d >= 0) {
      sum += (double)vals[9 * d] + (double)vals[9 * d + 4] + (double)vals[9 * d + 8];
      cnt += 3.0;
    }
  }
  block_partials(sum, cnt, part, red);
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_setup(Active a, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, const S* __restrict__ vals,
                                                   const S* __restrict__ b, double scale, S* __restrict__ r,
                                                   S* __restrict__ z, S* __restrict__ p, S* __restrict__ dinv,
                                                   double mu_rel, const double* __restrict__ pdiag,
                                                   double* __restrict__ pout, PcgState* st) {
  __shared__ double red[kPB];
  const double dsum = grid_sum(pdiag, 0, red), dcnt = grid_sum(pdiag, 1, red);
  // mu relative to the mean diagonal entry of the rows holding blocks (1 for an empty matrix)
  const double mu = mu_rel * (dcnt > 0.0 ? dsum / dcnt : 1.0);
  double rz = 0.0, bb = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
    const int64_t d = diag_block(row_ptr, col_idx, i);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double dg = (d >= 0 ? (double)vals[9 * d + 4 * c] : 0.0) + mu;
      const double di = dg > 0.0 ? 1.0 / dg : 1.0;
      const double ri = scale * (double)b[3 * i + c];
      const double zi = di * ri;
      dinv[3 * i + c] = (S)di;
      r[3 * i + c] = (S)ri;
      z[3 * i + c] = (S)zi;
      p[3 * i + c] = (S)zi;
      rz += ri * zi;
      bb += ri * ri;
    }
  }
  block_partials(rz, bb, pout, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->mu = mu;
    st->done = 0;
    st->iters = 0;
  }
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_matvec(Active a, const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col_idx, const S* __restrict__ vals,
                                                    const S* __restrict__ p, S* __restrict__ q,
                                                    double* __restrict__ pq_part, const PcgState* st) {
  if (st->done) return;
  __shared__ double red[kPB];
  const double mu = st->mu;
  double pq = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
    double acc[3] = {mu * (double)p[3 * i], mu * (double)p[3 * i + 1], mu * (double)p[3 * i + 2]};
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int64_t c = col_idx[k];
      const double p0 = p[3 * c], p1 = p[3 * c + 1], p2 = p[3 * c + 2];
#pragma unroll
      for (int e = 0; e < 3; ++e)
        acc[e] += (double)vals[9 * (int64_t)k + 3 * e] * p0 + (double)vals[9 * (int64_t)k + 3 * e + 1] * p1 +
                  (double)vals[9 * (int64_t)k + 3 * e + 2] * p2;
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      q[3 * i + e] = (S)acc[e];
      pq += (double)p[3 * i + e] * acc[e];
    }
  }
  block_partials(pq, 0.0, pq_part, red);
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_update(Active a, S* __restrict__ x, S* __restrict__ r,
                                                    S* __restrict__ z, const S* __restrict__ p,
                                                    const S* __restrict__ q, const S* __restrict__ dinv,
                                                    const double* __restrict__ rz_part, const double* __restrict__ pq_part,
                                                    double* __restrict__ out_part, PcgState* st) {
  if (st->done) return;
  __shared__ double red[kPB];
  const double rz = grid_sum(rz_part, 0, red), pq = grid_sum(pq_part, 0, red);
  if (!(pq > 0.0)) {  // (H + mu I) should be positive definite; stop on a breakdown
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 2;
    return;
  }
  const double alpha = rz / pq;
  double rzn = 0.0, rr = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t k = 3 * i + c;
      x[k] = (S)((double)x[k] + alpha * (double)p[k]);
      const double ri = (double)r[k] - alpha * (double)q[k];
      const double zi = (double)dinv[k] * ri;
      r[k] = (S)ri;
      z[k] = (S)zi;
      rzn += ri * zi;
      rr += ri * ri;
    }
  }
  block_partials(rzn, rr, out_part, red);
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_dir(Active a, S* __restrict__ p, const S* __restrict__ z,
                                                 const double* __restrict__ rz_old_part,
                                                 const double* __restrict__ rz_new_part,
                                                 const double* __restrict__ setup_part, double tol, int iter,
                                                 PcgState* st) {
  if (st->done) return;
  __shared__ double red[kPB];
  const double rzo = grid_sum(rz_old_part, 0, red), rzn = grid_sum(rz_new_part, 0, red);
  const double rr = grid_sum(rz_new_part, 1, red), bb = grid_sum(setup_part, 1, red);
  const bool conv = rr <= tol * tol * bb;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iters = iter + 1;
    st->rr = rr;
    st->bb = bb;
    if (conv) st->done = 1;
  }
  if (conv) return;
  const double beta = rzo > 0.0 ? rzn / rzo : 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) p[3 * i + c] = (S)((double)z[3 * i + c] + beta * (double)p[3 * i + c]);
  }
}

// ---- matrix-free variant: H applied from the last evaluation's per-hit records -------------
// H = sum over hits of J^T M J with J = [a^T; b^T] (2 x 18), the PSD core M of the
// evaluation.  Rows gather their incidences in pair-key order (the sorted lists the
// evaluation leaves behind), so the products are deterministic.

// raw diagonal of H per dof into dg, partials of (sum, count) over the active rows, as the BSR
// variant takes them over the rows holding blocks
template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_diag_mf(Active a, const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc,
                                                     const AsmRec<S>* __restrict__ recs, S* __restrict__ dg,
                                                     double* __restrict__ part) {
  __shared__ double red[kPB];
  double sum = 0.0, cnt = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
    const int32_t b = off[i], e = off[i + 1];
    double d[3] = {0.0, 0.0, 0.0};
    for (int32_t k = b; k < e; ++k) {
      const Incidence in = inc[k];
      const AsmRec<S>& r = recs[in.hit];
      const int s = in.slot;
      for (int l = 0; l < 6; ++l) {
        if (r.vid[l] != r.vid[s]) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double as = r.a[3 * s + c], bs = r.b[3 * s + c], al = r.a[3 * l + c], bl = r.b[3 * l + c];
          d[c] += (double)r.M[0] * as * al + (double)r.M[1] * (as * bl + bs * al) + (double)r.M[2] * bs * bl;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) dg[3 * i + c] = (S)d[c];
    if (e > b) {
      sum += d[0] + d[1] + d[2];
      cnt += 3.0;
    }
  }
  block_partials(sum, cnt, part, red);
}

// as k_pcg_setup, with the diagonal from dinv (holding the raw diagonal on entry)
template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_setup_mf(Active a, const S* __restrict__ b, double scale,
                                                      S* __restrict__ r, S* __restrict__ z, S* __restrict__ p,
                                                      S* __restrict__ dinv, double mu_rel,
                                                      const double* __restrict__ pdiag, double* __restrict__ pout,
                                                      PcgState* st) {
  __shared__ double red[kPB];
  const double dsum = grid_sum(pdiag, 0, red), dcnt = grid_sum(pdiag, 1, red);
  const double mu = mu_rel * (dcnt > 0.0 ? dsum / dcnt : 1.0);
  double rz = 0.0, bb = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t k = 3 * i + c;
      const double dg = (double)dinv[k] + mu;
      const double di = dg > 0.0 ? 1.0 / dg : 1.0;
      const double ri = scale * (double)b[k];
      const double zi = di * ri;
      dinv[k] = (S)di;
      r[k] = (S)ri;
      z[k] = (S)zi;
      p[k] = (S)zi;
      rz += ri * zi;
      bb += ri * ri;
    }
  }
  block_partials(rz, bb, pout, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->mu = mu;
    st->done = 0;
    st->iters = 0;
  }
}

// per hit: hv = J^T M (J p_local), 18 values
template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_hits_mf(const AsmRec<S>* __restrict__ recs, const Counters* ctr,
                                                     uint32_t max_hits, const S* __restrict__ p, S* __restrict__ hv,
                                                     const PcgState* st) {
  if (st->done) return;
  const uint32_t H = min(ctr->last_hits, max_hits);
  for (uint32_t h = blockIdx.x * kPB + threadIdx.x; h < H; h += gridDim.x * kPB) {
    const AsmRec<S>& r = recs[h];
    double ua = 0.0, ub = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double pv = p[3 * (int64_t)r.vid[k] + c];
        ua += (double)r.a[3 * k + c] * pv;
        ub += (double)r.b[3 * k + c] * pv;
      }
    const double wa = (double)r.M[0] * ua + (double)r.M[1] * ub, wb = (double)r.M[1] * ua + (double)r.M[2] * ub;
#pragma unroll
    for (int k = 0; k < 18; ++k) hv[18 * (int64_t)h + k] = (S)(wa * (double)r.a[k] + wb * (double)r.b[k]);
  }
}

// q = (H + mu I) p from the per-hit products, row by row in pair-key order; partials of p.q
template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_rows_mf(Active a, const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc, const S* __restrict__ hv,
                                                     const S* __restrict__ p, S* __restrict__ q,
                                                     double* __restrict__ pq_part, const PcgState* st) {
  if (st->done) return;
  __shared__ double red[kPB];
  const double mu = st->mu;
  double pq = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
    double acc[3] = {mu * (double)p[3 * i], mu * (double)p[3 * i + 1], mu * (double)p[3 * i + 2]};
    for (int32_t k = off[i]; k < off[i + 1]; ++k) {
      const Incidence in = inc[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += (double)hv[18 * (int64_t)in.hit + 3 * in.slot + c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q[3 * i + c] = (S)acc[c];
      pq += (double)p[3 * i + c] * acc[c];
    }
  }
  block_partials(pq, 0.0, pq_part, red);
}

// ---- coupled variant: A = K + w H + mu I, K a caller's PSD BSR matrix (FP64) --------------
// (the quasi-static objective's elastic Hessian), H applied from the hit records as above.
// Jacobi diagonal: K's diagonal entries + w times H's + mu.
__global__ void __launch_bounds__(kPB) k_pcg_setup_cp(Active a, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col_idx,
                                                      const double* __restrict__ vals, double w, double mu,
                                                      const double* __restrict__ b, double scale,
                                                      double* __restrict__ r, double* __restrict__ z,
                                                      double* __restrict__ p, double* __restrict__ dinv,
                                                      double* __restrict__ pout, PcgState* st) {
  __shared__ double red[kPB];
  double rz = 0.0, bb = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
    const int64_t d = diag_block(row_ptr, col_idx, i);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double dg = (d >= 0 ? vals[9 * d + 4 * c] : 0.0) + w * dinv[3 * i + c] + mu;
      const double di = dg > 0.0 ? 1.0 / dg : 1.0;
      const double ri = scale * b[3 * i + c];
      const double zi = di * ri;
      dinv[3 * i + c] = di;
      r[3 * i + c] = ri;
      z[3 * i + c] = zi;
      p[3 * i + c] = zi;
      rz += ri * zi;
      bb += ri * ri;
    }
  }
  block_partials(rz, bb, pout, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->mu = mu;
    st->done = 0;
    st->iters = 0;
  }
}

// q = (K + w H + mu I) p: K's row times p, plus w times the hit products gathered in pair-key
// order; partials of p.q
__global__ void __launch_bounds__(kPB) k_pcg_rows_cp(Active a, const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc, const double* __restrict__ hv,
                                                     const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx,
                                                     const double* __restrict__ vals, double w,
                                                     const double* __restrict__ p, double* __restrict__ q,
                                                     double* __restrict__ pq_part, const PcgState* st) {
  if (st->done) return;
  __shared__ double red[kPB];
  const double mu = st->mu;
  double pq = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
    double hs[3] = {0.0, 0.0, 0.0};
    for (int32_t k = off[i]; k < off[i + 1]; ++k) {
      const Incidence in = inc[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) hs[c] += hv[18 * (int64_t)in.hit + 3 * in.slot + c];
    }
    double acc[3] = {mu * p[3 * i] + w * hs[0], mu * p[3 * i + 1] + w * hs[1], mu * p[3 * i + 2] + w * hs[2]};
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int64_t c = col_idx[k];
      const double p0 = p[3 * c], p1 = p[3 * c + 1], p2 = p[3 * c + 2];
#pragma unroll
      for (int e = 0; e < 3; ++e)
        acc[e] += vals[9 * (int64_t)k + 3 * e] * p0 + vals[9 * (int64_t)k + 3 * e + 1] * p1 +
                  vals[9 * (int64_t)k + 3 * e + 2] * p2;
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      q[3 * i + e] = acc[e];
      pq += p[3 * i + e] * acc[e];
    }
  }
  block_partials(pq, 0.0, pq_part, red);
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_xb(Active a, const S* __restrict__ x, const S* __restrict__ b,
                                                double scale, double* __restrict__ part) {
  __shared__ double red[kPB];
  double xb = 0.0;
  PCG_ROWS(j, i, a) {
    const int64_t i = a.rows[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) xb += (double)x[3 * i + c] * scale * (double)b[3 * i + c];
  }
  block_partials(xb, 0.0, part, red);
}

__global__ void __launch_bounds__(kPB) k_pcg_info(const double* __restrict__ part, const PcgState* st, double* info) {
  __shared__ double red[kPB];
  const double xb = grid_sum(part, 0, red);
  if (threadIdx.x == 0) {
    info[0] = st->iters;
    info[1] = st->bb > 0.0 ? sqrt(st->rr / st->bb) : 0.0;
    info[2] = st->mu;
    info[3] = xb;
  }
}

template <class S>
__global__ void __launch_bounds__(kPB) k_axpy(int64_t n, double alpha, const double* __restrict__ x,
                                              const S* __restrict__ d, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPB) {
    const double v = x[i] + alpha * (double)d[i];
    out[i] = fabs(v) < 0x1p-200 ? 0.0 : v;  // stay in the predicates' coordinate domain
  }
}


// the vectors and partials of a solve, carved from the workspace
template <class S>
struct PcgBufs {
  S *r, *z, *p, *q, *dinv;
  double *pdiag, *pset, *pq, *pA, *pB;
  PcgState* st;
  PcgBufs(Ctx* c) {
    const Layout& L = c->L;
    S* base = wsp<S>(c, L.pcg_vec);
    const int64_t m3 = 3 * (int64_t)c->lim.max_verts;
    r = base;
    z = base + m3;
    p = base + 2 * m3;
    q = base + 3 * m3;
    dinv = base + 4 * m3;
    double* part = wsp<double>(c, L.pcg_part);  // 5 partial arrays of kPB x 4
    pdiag = part;
    pset = part + 4 * kPB;
    pq = part + 8 * kPB;
    pA = part + 12 * kPB;
    pB = part + 16 * kPB;
    st = wsp<PcgState>(c, L.pcg_state);
  }
};

template <class S>
static void pcg_finish(Ctx* c, const Active& a, const PcgBufs<S>& B, const S* x, const S* b, double scale,
                       double* info, hipStream_t s) {
  if (info) {
    k_pcg_xb<S><<<kPB, kPB, 0, s>>>(a, x, b, scale, B.pq);
    k_pcg_info<<<1, kPB, 0, s>>>(B.pq, B.st, info);
  }
}

template <class S>
static hipError_t pcg_impl(Ctx* c, int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const S* vals,
                           const S* b, double scale, S* x, double mu_rel, int max_iter, double tol, double* info,
                           hipStream_t s) {
  PcgBufs<S> B(c);
  stage_begin(c, TTIE_STAGE_PCG, s);
  Active a;
  hipError_t e = pcg_active<S>(c, n, row_ptr, nullptr, b, x, B.p, a, s);
  if (e != hipSuccess) return e;
  k_pcg_diag<S><<<kPB, kPB, 0, s>>>(a, row_ptr, col_idx, vals, B.pdiag);
  k_pcg_setup<S><<<kPB, kPB, 0, s>>>(a, row_ptr, col_idx, vals, b, scale, B.r, B.z, B.p, B.dinv, mu_rel, B.pdiag,
                                     B.pset, B.st);
  const double* rz_old = B.pset;
  for (int it = 0; it < max_iter; ++it) {
    double* rz_new = (it % 2 == 0) ? B.pA : B.pB;
    k_pcg_matvec<S><<<kPB, kPB, 0, s>>>(a, row_ptr, col_idx, vals, B.p, B.q, B.pq, B.st);
    k_pcg_update<S><<<kPB, kPB, 0, s>>>(a, x, B.r, B.z, B.p, B.q, B.dinv, rz_old, B.pq, rz_new, B.st);
    k_pcg_dir<S><<<kPB, kPB, 0, s>>>(a, B.p, B.z, rz_old, rz_new, B.pset, tol, it, B.st);
    rz_old = rz_new;
  }
  pcg_finish<S>(c, a, B, x, b, scale, info, s);
  stage_end(c, TTIE_STAGE_PCG, s);
  return hipGetLastError();
}

template <class S>
static hipError_t pcg_mf_impl(Ctx* c, int64_t n, const S* b, double scale, S* x, double mu_rel, int max_iter, double tol,
                              double* info, hipStream_t s) {
  const Layout& L = c->L;
  PcgBufs<S> B(c);
  const AsmRec<S>* recs = wsp<AsmRec<S>>(c, L.recs);
  int32_t* off = wsp<int32_t>(c, L.off);
  const Incidence* inc = wsp<Incidence>(c, L.inc2);
  S* hv = wsp<S>(c, L.hvbuf);
  const Counters* ctr = wsp<Counters>(c, L.counters);
  const uint32_t max_hits = (uint32_t)c->lim.max_hits;
  const unsigned gh = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (c->lim.max_hits + kPB - 1) / kPB));
  stage_begin(c, TTIE_STAGE_PCG, s);
  Active a;
  hipError_t e = pcg_active<S>(c, n, nullptr, off, b, x, B.p, a, s);
  if (e != hipSuccess) return e;
  k_pcg_diag_mf<S><<<kPB, kPB, 0, s>>>(a, off, inc, recs, B.dinv, B.pdiag);
  k_pcg_setup_mf<S><<<kPB, kPB, 0, s>>>(a, b, scale, B.r, B.z, B.p, B.dinv, mu_rel, B.pdiag, B.pset, B.st);
  const double* rz_old = B.pset;
  for (int it = 0; it < max_iter; ++it) {
    double* rz_new = (it % 2 == 0) ? B.pA : B.pB;
    k_pcg_hits_mf<S><<<gh, kPB, 0, s>>>(recs, ctr, max_hits, B.p, hv, B.st);
    k_pcg_rows_mf<S><<<kPB, kPB, 0, s>>>(a, off, inc, hv, B.p, B.q, B.pq, B.st);
    k_pcg_update<S><<<kPB, kPB, 0, s>>>(a, x, B.r, B.z, B.p, B.q, B.dinv, rz_old, B.pq, rz_new, B.st);
    k_pcg_dir<S><<<kPB, kPB, 0, s>>>(a, B.p, B.z, rz_old, rz_new, B.pset, tol, it, B.st);
    rz_old = rz_new;
  }
  pcg_finish<S>(c, a, B, x, b, scale, info, s);
  stage_end(c, TTIE_STAGE_PCG, s);
  return hipGetLastError();
}

hipError_t launch_pcg_coupled(Ctx* c, int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                              double w, const double* b, double scale, double* x, double mu, int max_iter, double tol,
                              double* info, hipStream_t s) {
  const Layout& L = c->L;
  PcgBufs<double> B(c);
  const AsmRec<double>* recs = wsp<AsmRec<double>>(c, L.recs);
  int32_t* off = wsp<int32_t>(c, L.off);
  const Incidence* inc = wsp<Incidence>(c, L.inc2);
  double* hv = wsp<double>(c, L.hvbuf);
  const Counters* ctr = wsp<Counters>(c, L.counters);
  const uint32_t max_hits = (uint32_t)c->lim.max_hits;
  const unsigned gh = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (c->lim.max_hits + kPB - 1) / kPB));
  stage_begin(c, TTIE_STAGE_PCG, s);
  Active a;
  hipError_t e = pcg_active<double>(c, n, row_ptr, off, b, x, B.p, a, s);
  if (e != hipSuccess) return e;
  k_pcg_diag_mf<double><<<kPB, kPB, 0, s>>>(a, off, inc, recs, B.dinv, B.pdiag);  // raw diagonal of H into dinv
  k_pcg_setup_cp<<<kPB, kPB, 0, s>>>(a, row_ptr, col_idx, vals, w, mu, b, scale, B.r, B.z, B.p, B.dinv, B.pset, B.st);
  const double* rz_old = B.pset;
  for (int it = 0; it < max_iter; ++it) {
    double* rz_new = (it % 2 == 0) ? B.pA : B.pB;
    k_pcg_hits_mf<double><<<gh, kPB, 0, s>>>(recs, ctr, max_hits, B.p, hv, B.st);
    k_pcg_rows_cp<<<kPB, kPB, 0, s>>>(a, off, inc, hv, row_ptr, col_idx, vals, w, B.p, B.q, B.pq, B.st);
    k_pcg_update<double><<<kPB, kPB, 0, s>>>(a, x, B.r, B.z, B.p, B.q, B.dinv, rz_old, B.pq, rz_new, B.st);
    k_pcg_dir<double><<<kPB, kPB, 0, s>>>(a, B.p, B.z, rz_old, rz_new, B.pset, tol, it, B.st);
    rz_old = rz_new;
  }
  pcg_finish<double>(c, a, B, x, b, scale, info, s);
  stage_end(c, TTIE_STAGE_PCG, s);
  return hipGetLastError();
}

hipError_t launch_pcg_mf(Ctx* c, int64_t n, const void* b, double scale, void* x, double mu_rel, int max_iter,
                         double tol, double* info, hipStream_t s) {
  if (c->last_precision == TTIE_FP64)
    return pcg_mf_impl<double>(c, n, (const double*)b, scale, (double*)x, mu_rel, max_iter, tol, info, s);
  return pcg_mf_impl<float>(c, n, (const float*)b, scale, (float*)x, mu_rel, max_iter, tol, info, s);
}

hipError_t launch_pcg(Ctx* c, int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                      const void* b, double scale, void* x, double mu_rel, int max_iter, double tol, int precision,
                      double* info, hipStream_t s) {
  if (precision == TTIE_FP64)
    return pcg_impl<double>(c, n, row_ptr, col_idx, (const double*)vals, (const double*)b, scale, (double*)x, mu_rel,
                            max_iter, tol, info, s);
  return pcg_impl<float>(c, n, row_ptr, col_idx, (const float*)vals, (const float*)b, scale, (float*)x, mu_rel,
                         max_iter, tol, info, s);
}

hipError_t launch_axpy(int64_t n_verts, double alpha, const double* x, const void* d, double* out, int precision,
                       hipStream_t s) {
  const int64_t n = 3 * n_verts;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kPB - 1) / kPB));
  if (precision == TTIE_FP64)
    k_axpy<double><<<g, kPB, 0, s>>>(n, alpha, x, (const double*)d, out);
  else
    k_axpy<float><<<g, kPB, 0, s>>>(n, alpha, x, (const float*)d, out);
  return hipGetLastError();
}

}  // namespace ttie
