// Jacobi-preconditioned conjugate gradients on (H + mu I) x = scale * b for the inexact
// Newton consumer, with H the BSR Hessian of ttie_eval.  Everything stays on the device: the
// scalars of the iteration are reduced from fixed-size per-block partials (fixed order, so
// the result is deterministic), every kernel re-derives them from the previous kernel's
// partials, and a convergence flag written by one kernel turns the remaining launches into
// no-ops.  Three launches per iteration:
//   k_pcg_matvec  q = (H + mu I) p, partials of p.q
//   k_pcg_update  alpha = r.z / p.q; x += alpha p; r -= alpha q; z = D^-1 r; partials r.z, r.r
//   k_pcg_dir     beta = r.z(new) / r.z(old); p = z + beta p; convergence test
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

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_diag(int64_t n, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx, const S* __restrict__ vals,
                                                  double* __restrict__ part) {
  __shared__ double red[kPB];
  double sum = 0.0, cnt = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kPB + threadIdx.x; r < n; r += (int64_t)gridDim.x * kPB) {
    const int64_t d = diag_block(row_ptr, col_idx, r);
    if (d >= 0) {
      sum += (double)vals[9 * d] + (double)vals[9 * d + 4] + (double)vals[9 * d + 8];
      cnt += 3.0;
    }
  }
  block_partials(sum, cnt, part, red);
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_setup(int64_t n, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, const S* __restrict__ vals,
                                                   const S* __restrict__ b, double scale, S* __restrict__ x,
                                                   S* __restrict__ r, S* __restrict__ z, S* __restrict__ p,
                                                   S* __restrict__ dinv, double mu_rel, const double* __restrict__ pdiag,
                                                   double* __restrict__ pout, PcgState* st) {
  __shared__ double red[kPB];
  const double dsum = grid_sum(pdiag, 0, red), dcnt = grid_sum(pdiag, 1, red);
  // mu relative to the mean diagonal entry of the rows holding blocks (1 for an empty matrix)
  const double mu = mu_rel * (dcnt > 0.0 ? dsum / dcnt : 1.0);
  double rz = 0.0, bb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPB) {
    const int64_t d = diag_block(row_ptr, col_idx, i);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double dg = (d >= 0 ? (double)vals[9 * d + 4 * c] : 0.0) + mu;
      const double di = dg > 0.0 ? 1.0 / dg : 1.0;
      const double ri = scale * (double)b[3 * i + c];
      const double zi = di * ri;
      dinv[3 * i + c] = (S)di;
      x[3 * i + c] = (S)0.0;
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
__global__ void __launch_bounds__(kPB) k_pcg_matvec(int64_t n, const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col_idx, const S* __restrict__ vals,
                                                    const S* __restrict__ p, S* __restrict__ q,
                                                    double* __restrict__ pq_part, const PcgState* st) {
  if (st->done) return;
  __shared__ double red[kPB];
  const double mu = st->mu;
  double pq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPB) {
    double acc[3] = {mu * (double)p[3 * i], mu * (double)p[3 * i + 1], mu * (double)p[3 * i + 2]};
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int64_t c = col_idx[k];
      const double p0 = p[3 * c], p1 = p[3 * c + 1], p2 = p[3 * c + 2];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        acc[a] += (double)vals[9 * (int64_t)k + 3 * a] * p0 + (double)vals[9 * (int64_t)k + 3 * a + 1] * p1 +
                  (double)vals[9 * (int64_t)k + 3 * a + 2] * p2;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      q[3 * i + a] = (S)acc[a];
      pq += (double)p[3 * i + a] * acc[a];
    }
  }
  block_partials(pq, 0.0, pq_part, red);
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_update(int64_t n, S* __restrict__ x, S* __restrict__ r,
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
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * kPB) {
    x[i] = (S)((double)x[i] + alpha * (double)p[i]);
    const double ri = (double)r[i] - alpha * (double)q[i];
    const double zi = (double)dinv[i] * ri;
    r[i] = (S)ri;
    z[i] = (S)zi;
    rzn += ri * zi;
    rr += ri * ri;
  }
  block_partials(rzn, rr, out_part, red);
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_dir(int64_t n, S* __restrict__ p, const S* __restrict__ z,
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
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * kPB)
    p[i] = (S)((double)z[i] + beta * (double)p[i]);
}

// ---- matrix-free variant: H applied from the last evaluation's per-hit records -------------
// H = sum over hits of J^T M J with J = [a^T; b^T] (2 x 18), the PSD core M of the
// evaluation.  Rows gather their incidences in pair-key order (the sorted lists the
// evaluation leaves behind), so the products are deterministic.

// raw diagonal of H per dof into dg (0 for untouched rows), partials of (sum, count) over the
// rows holding hits, as the BSR variant takes them over the rows holding blocks
template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_diag_mf(int64_t n, const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc,
                                                     const AsmRec<S>* __restrict__ recs, S* __restrict__ dg,
                                                     double* __restrict__ part) {
  __shared__ double red[kPB];
  double sum = 0.0, cnt = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPB) {
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
__global__ void __launch_bounds__(kPB) k_pcg_setup_mf(int64_t n, const S* __restrict__ b, double scale, S* __restrict__ x,
                                                      S* __restrict__ r, S* __restrict__ z, S* __restrict__ p,
                                                      S* __restrict__ dinv, double mu_rel,
                                                      const double* __restrict__ pdiag, double* __restrict__ pout,
                                                      PcgState* st) {
  __shared__ double red[kPB];
  const double dsum = grid_sum(pdiag, 0, red), dcnt = grid_sum(pdiag, 1, red);
  const double mu = mu_rel * (dcnt > 0.0 ? dsum / dcnt : 1.0);
  double rz = 0.0, bb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * kPB) {
    const double dg = (double)dinv[i] + mu;
    const double di = dg > 0.0 ? 1.0 / dg : 1.0;
    const double ri = scale * (double)b[i];
    const double zi = di * ri;
    dinv[i] = (S)di;
    x[i] = (S)0.0;
    r[i] = (S)ri;
    z[i] = (S)zi;
    p[i] = (S)zi;
    rz += ri * zi;
    bb += ri * ri;
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
__global__ void __launch_bounds__(kPB) k_pcg_rows_mf(int64_t n, const int32_t* __restrict__ off,
                                                     const Incidence* __restrict__ inc, const S* __restrict__ hv,
                                                     const S* __restrict__ p, S* __restrict__ q,
                                                     double* __restrict__ pq_part, const PcgState* st) {
  if (st->done) return;
  __shared__ double red[kPB];
  const double mu = st->mu;
  double pq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPB) {
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
__global__ void __launch_bounds__(kPB) k_pcg_setup_cp(int64_t n, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col_idx,
                                                      const double* __restrict__ vals, double w, double mu,
                                                      const double* __restrict__ b, double scale,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      double* __restrict__ z, double* __restrict__ p,
                                                      double* __restrict__ dinv, double* __restrict__ pout,
                                                      PcgState* st) {
  __shared__ double red[kPB];
  double rz = 0.0, bb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPB) {
    const int64_t d = diag_block(row_ptr, col_idx, i);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double dg = (d >= 0 ? vals[9 * d + 4 * c] : 0.0) + w * dinv[3 * i + c] + mu;
      const double di = dg > 0.0 ? 1.0 / dg : 1.0;
      const double ri = scale * b[3 * i + c];
      const double zi = di * ri;
      dinv[3 * i + c] = di;
      x[3 * i + c] = 0.0;
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
__global__ void __launch_bounds__(kPB) k_pcg_rows_cp(int64_t n, const int32_t* __restrict__ off,
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
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPB) {
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
      for (int a = 0; a < 3; ++a)
        acc[a] += vals[9 * (int64_t)k + 3 * a] * p0 + vals[9 * (int64_t)k + 3 * a + 1] * p1 +
                  vals[9 * (int64_t)k + 3 * a + 2] * p2;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      q[3 * i + a] = acc[a];
      pq += p[3 * i + a] * acc[a];
    }
  }
  block_partials(pq, 0.0, pq_part, red);
}

template <class S>
__global__ void __launch_bounds__(kPB) k_pcg_xb(int64_t n, const S* __restrict__ x, const S* __restrict__ b,
                                                double scale, double* __restrict__ part) {
  __shared__ double red[kPB];
  double xb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * kPB)
    xb += (double)x[i] * scale * (double)b[i];
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

template <class S>
static hipError_t pcg_impl(Ctx* c, int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const S* vals,
                           const S* b, double scale, S* x, double mu_rel, int max_iter, double tol, double* info,
                           hipStream_t s) {
  const Layout& L = c->L;
  S* base = wsp<S>(c, L.pcg_vec);
  const int64_t m3 = 3 * (int64_t)c->lim.max_verts;
  S *r = base, *z = base + m3, *p = base + 2 * m3, *q = base + 3 * m3, *dinv = base + 4 * m3;
  double* part = wsp<double>(c, L.pcg_part);  // 5 partial arrays of kPB x 4
  double *pdiag = part, *pset = part + 4 * kPB, *pq = part + 8 * kPB, *pA = part + 12 * kPB, *pB = part + 16 * kPB;
  PcgState* st = wsp<PcgState>(c, L.pcg_state);
  stage_begin(c, TTIE_STAGE_PCG, s);
  k_pcg_diag<S><<<kPB, kPB, 0, s>>>(n, row_ptr, col_idx, vals, pdiag);
  k_pcg_setup<S><<<kPB, kPB, 0, s>>>(n, row_ptr, col_idx, vals, b, scale, x, r, z, p, dinv, mu_rel, pdiag, pset, st);
  const double* rz_old = pset;
  for (int it = 0; it < max_iter; ++it) {
    double* rz_new = (it % 2 == 0) ? pA : pB;
    k_pcg_matvec<S><<<kPB, kPB, 0, s>>>(n, row_ptr, col_idx, vals, p, q, pq, st);
    k_pcg_update<S><<<kPB, kPB, 0, s>>>(n, x, r, z, p, q, dinv, rz_old, pq, rz_new, st);
    k_pcg_dir<S><<<kPB, kPB, 0, s>>>(n, p, z, rz_old, rz_new, pset, tol, it, st);
    rz_old = rz_new;
  }
  if (info) {
    k_pcg_xb<S><<<kPB, kPB, 0, s>>>(n, x, b, scale, pq);
    k_pcg_info<<<1, kPB, 0, s>>>(pq, st, info);
  }
  stage_end(c, TTIE_STAGE_PCG, s);
  return hipGetLastError();
}

template <class S>
static hipError_t pcg_mf_impl(Ctx* c, int64_t n, const S* b, double scale, S* x, double mu_rel, int max_iter, double tol,
                              double* info, hipStream_t s) {
  const Layout& L = c->L;
  S* base = wsp<S>(c, L.pcg_vec);
  const int64_t m3 = 3 * (int64_t)c->lim.max_verts;
  S *r = base, *z = base + m3, *p = base + 2 * m3, *q = base + 3 * m3, *dinv = base + 4 * m3;
  double* part = wsp<double>(c, L.pcg_part);
  double *pdiag = part, *pset = part + 4 * kPB, *pq = part + 8 * kPB, *pA = part + 12 * kPB, *pB = part + 16 * kPB;
  PcgState* st = wsp<PcgState>(c, L.pcg_state);
  const AsmRec<S>* recs = wsp<AsmRec<S>>(c, L.recs);
  const int32_t* off = wsp<int32_t>(c, L.off);
  const Incidence* inc = wsp<Incidence>(c, L.inc2);
  S* hv = wsp<S>(c, L.hvbuf);
  const Counters* ctr = wsp<Counters>(c, L.counters);
  const uint32_t max_hits = (uint32_t)c->lim.max_hits;
  const unsigned gh = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (c->lim.max_hits + kPB - 1) / kPB));
  stage_begin(c, TTIE_STAGE_PCG, s);
  k_pcg_diag_mf<S><<<kPB, kPB, 0, s>>>(n, off, inc, recs, dinv, pdiag);
  k_pcg_setup_mf<S><<<kPB, kPB, 0, s>>>(n, b, scale, x, r, z, p, dinv, mu_rel, pdiag, pset, st);
  const double* rz_old = pset;
  for (int it = 0; it < max_iter; ++it) {
    double* rz_new = (it % 2 == 0) ? pA : pB;
    k_pcg_hits_mf<S><<<gh, kPB, 0, s>>>(recs, ctr, max_hits, p, hv, st);
    k_pcg_rows_mf<S><<<kPB, kPB, 0, s>>>(n, off, inc, hv, p, q, pq, st);
    k_pcg_update<S><<<kPB, kPB, 0, s>>>(n, x, r, z, p, q, dinv, rz_old, pq, rz_new, st);
    k_pcg_dir<S><<<kPB, kPB, 0, s>>>(n, p, z, rz_old, rz_new, pset, tol, it, st);
    rz_old = rz_new;
  }
  if (info) {
    k_pcg_xb<S><<<kPB, kPB, 0, s>>>(n, x, b, scale, pq);
    k_pcg_info<<<1, kPB, 0, s>>>(pq, st, info);
  }
  stage_end(c, TTIE_STAGE_PCG, s);
  return hipGetLastError();
}

hipError_t launch_pcg_coupled(Ctx* c, int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                              double w, const double* b, double scale, double* x, double mu, int max_iter, double tol,
                              double* info, hipStream_t s) {
  const Layout& L = c->L;
  double* base = wsp<double>(c, L.pcg_vec);
  const int64_t m3 = 3 * (int64_t)c->lim.max_verts;
  double *r = base, *z = base + m3, *p = base + 2 * m3, *q = base + 3 * m3, *dinv = base + 4 * m3;
  double* part = wsp<double>(c, L.pcg_part);
  double *pdiag = part, *pset = part + 4 * kPB, *pq = part + 8 * kPB, *pA = part + 12 * kPB, *pB = part + 16 * kPB;
  PcgState* st = wsp<PcgState>(c, L.pcg_state);
  const AsmRec<double>* recs = wsp<AsmRec<double>>(c, L.recs);
  const int32_t* off = wsp<int32_t>(c, L.off);
  const Incidence* inc = wsp<Incidence>(c, L.inc2);
  double* hv = wsp<double>(c, L.hvbuf);
  const Counters* ctr = wsp<Counters>(c, L.counters);
  const uint32_t max_hits = (uint32_t)c->lim.max_hits;
  const unsigned gh = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (c->lim.max_hits + kPB - 1) / kPB));
  stage_begin(c, TTIE_STAGE_PCG, s);
  k_pcg_diag_mf<double><<<kPB, kPB, 0, s>>>(n, off, inc, recs, dinv, pdiag);  // raw diagonal of H into dinv
  k_pcg_setup_cp<<<kPB, kPB, 0, s>>>(n, row_ptr, col_idx, vals, w, mu, b, scale, x, r, z, p, dinv, pset, st);
  const double* rz_old = pset;
  for (int it = 0; it < max_iter; ++it) {
    double* rz_new = (it % 2 == 0) ? pA : pB;
    k_pcg_hits_mf<double><<<gh, kPB, 0, s>>>(recs, ctr, max_hits, p, hv, st);
    k_pcg_rows_cp<<<kPB, kPB, 0, s>>>(n, off, inc, hv, row_ptr, col_idx, vals, w, p, q, pq, st);
    k_pcg_update<double><<<kPB, kPB, 0, s>>>(n, x, r, z, p, q, dinv, rz_old, pq, rz_new, st);
    k_pcg_dir<double><<<kPB, kPB, 0, s>>>(n, p, z, rz_old, rz_new, pset, tol, it, st);
    rz_old = rz_new;
  }
  if (info) {
    k_pcg_xb<double><<<kPB, kPB, 0, s>>>(n, x, b, scale, pq);
    k_pcg_info<<<1, kPB, 0, s>>>(pq, st, info);
  }
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
