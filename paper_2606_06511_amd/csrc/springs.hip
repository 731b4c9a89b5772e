// Quasi-static coupling: a synthetic elastic model (springs on the mesh's edges) and the
// objective of one quasi-static step,
//
//   Phi(x) = sum over edges (k/2)(|x_i - x_j| - |r_i - r_j|)^2 + w E(x) + (m/2)|x - x_prev|^2,
//
// with E the intersection energy of the last evaluation and r the rest positions.  The paper
// pairs the energy with an elastic model in its quasi-static experiment (Fig. 2) without
// giving it; this is a stand-in.
//
// Layout: the springs' Hessian is a 3x3-block CSR matrix whose row v holds v and its
// neighbours in increasing order (the mesh's edge graph plus the diagonal), built once by
// ttie_springs_pattern.  ttie_qs_eval then works row by row over that pattern with one thread
// per vertex: every spring is seen from both ends, so gradient rows and Hessian blocks are
// written without atomics, and the energy is reduced from fixed per-block partials.
#include "internal.h"

namespace ttie {

constexpr int kSB = 256;  // threads per block

static unsigned sp_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kSB - 1) / kSB));
}

__global__ void __launch_bounds__(kSB) k_sp_zero(int32_t* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kSB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSB) a[i] = 0;
}

// half-edge counts per vertex (an interior edge is counted once from each of its triangles)
__global__ void __launch_bounds__(kSB) k_sp_count(const int32_t* __restrict__ tris, int64_t nt, int64_t nv,
                                                  int32_t* __restrict__ deg, Counters* ctr) {
  for (int64_t t = (int64_t)blockIdx.x * kSB + threadIdx.x; t < nt; t += (int64_t)gridDim.x * kSB) {
    const int32_t v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    if (v[0] < 0 || v[1] < 0 || v[2] < 0 || v[0] >= nv || v[1] >= nv || v[2] >= nv) {
      atomicCAS(&ctr->status, 0, STATUS_INDEX);
      continue;
    }
    for (int e = 0; e < 3; ++e) {
      const int32_t a = v[e], b = v[(e + 1) % 3];
      if (a == b) continue;
      atomicAdd(&deg[a], 1);
      atomicAdd(&deg[b], 1);
    }
  }
}

__global__ void __launch_bounds__(kSB) k_sp_scatter(const int32_t* __restrict__ tris, int64_t nt, int64_t nv,
                                                    const int32_t* __restrict__ off, int32_t* __restrict__ cur,
                                                    int32_t* __restrict__ adj) {
  for (int64_t t = (int64_t)blockIdx.x * kSB + threadIdx.x; t < nt; t += (int64_t)gridDim.x * kSB) {
    const int32_t v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    if (v[0] < 0 || v[1] < 0 || v[2] < 0 || v[0] >= nv || v[1] >= nv || v[2] >= nv) continue;
    for (int e = 0; e < 3; ++e) {
      const int32_t a = v[e], b = v[(e + 1) % 3];
      if (a == b) continue;
      adj[off[a] + atomicAdd(&cur[a], 1)] = b;
      adj[off[b] + atomicAdd(&cur[b], 1)] = a;
    }
  }
}

// per row: sort the neighbour list (insertion sort; rows are short on meshes), count the
// distinct neighbours plus the diagonal
__global__ void __launch_bounds__(kSB) k_sp_unique(int64_t nv, const int32_t* __restrict__ off,
                                                   int32_t* __restrict__ adj, int32_t* __restrict__ ucnt) {
  for (int64_t v = (int64_t)blockIdx.x * kSB + threadIdx.x; v <= nv; v += (int64_t)gridDim.x * kSB) {
    if (v == nv) {
      ucnt[nv] = 0;
      continue;
    }
    const int32_t b = off[v], e = off[v + 1];
    for (int32_t i = b + 1; i < e; ++i) {
      const int32_t key = adj[i];
      int32_t j = i - 1;
      while (j >= b && adj[j] > key) {
        adj[j + 1] = adj[j];
        --j;
      }
      adj[j + 1] = key;
    }
    int32_t u = 1;
    for (int32_t i = b; i < e; ++i) u += (i == b || adj[i] != adj[i - 1]);
    ucnt[v] = u;
  }
}

// column indices: the distinct sorted neighbours with v merged in
__global__ void __launch_bounds__(kSB) k_sp_cols(int64_t nv, const int32_t* __restrict__ off,
                                                 const int32_t* __restrict__ adj, const int32_t* __restrict__ row_ptr,
                                                 int32_t* __restrict__ col_idx, int64_t cap, int64_t* n_blocks,
                                                 Counters* ctr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *n_blocks = row_ptr[nv];
    if (row_ptr[nv] > cap) atomicCAS(&ctr->status, 0, STATUS_CAPACITY);
  }
  for (int64_t v = (int64_t)blockIdx.x * kSB + threadIdx.x; v < nv; v += (int64_t)gridDim.x * kSB) {
    int64_t o = row_ptr[v];
    if (row_ptr[v + 1] > cap) continue;
    bool placed = false;
    const int32_t b = off[v], e = off[v + 1];
    for (int32_t i = b; i < e; ++i) {
      if (i > b && adj[i] == adj[i - 1]) continue;
      if (!placed && adj[i] > v) {
        col_idx[o++] = (int32_t)v;
        placed = true;
      }
      col_idx[o++] = adj[i];
    }
    if (!placed) col_idx[o++] = (int32_t)v;
  }
}

hipError_t launch_springs_pattern(Ctx* c, const ttie_mesh* m, int32_t* row_ptr, int32_t* col_idx, int64_t cap,
                                  int64_t* n_blocks, hipStream_t s) {
  const Layout& L = c->L;
  const int64_t nv = m->n_verts, nt = m->n_tris;
  Counters* ctr = wsp<Counters>(c, L.counters);
  int32_t* deg = wsp<int32_t>(c, L.cnt);
  int32_t* cur = wsp<int32_t>(c, L.cur);
  int32_t* off = wsp<int32_t>(c, L.off);
  int32_t* ucnt = wsp<int32_t>(c, L.ncol);
  // borrowed buffers: the evaluation's per-vertex counters and offsets, the broad phase's
  // leaf records (6 entries per triangle, far below their size)
  int32_t* adj = wsp<int32_t>(c, L.bvh_leaves);
  k_sp_zero<<<sp_grid(nv + 1), kSB, 0, s>>>(deg, nv + 1);
  k_sp_zero<<<sp_grid(nv + 1), kSB, 0, s>>>(cur, nv + 1);
  k_sp_count<<<sp_grid(nt), kSB, 0, s>>>(m->tris, nt, nv, deg, ctr);
  hipError_t e = launch_scan_i32(c, deg, off, nv + 1, s);
  if (e != hipSuccess) return e;
  k_sp_scatter<<<sp_grid(nt), kSB, 0, s>>>(m->tris, nt, nv, off, cur, adj);
  k_sp_unique<<<sp_grid(nv + 1), kSB, 0, s>>>(nv, off, adj, ucnt);
  e = launch_scan_i32(c, ucnt, row_ptr, nv + 1, s);
  if (e != hipSuccess) return e;
  k_sp_cols<<<sp_grid(nv), kSB, 0, s>>>(nv, off, adj, row_ptr, col_idx, cap, n_blocks, ctr);
  // the evaluation expects its per-vertex counters zero on entry (it clears them on exit)
  k_sp_zero<<<sp_grid(nv + 1), kSB, 0, s>>>(deg, nv + 1);
  k_sp_zero<<<sp_grid(nv + 1), kSB, 0, s>>>(cur, nv + 1);
  k_sp_zero<<<sp_grid(nv + 1), kSB, 0, s>>>(ucnt, nv + 1);
  return hipGetLastError();
}

// ---- the objective of a quasi-static step ---------------------------------------------------
// Row v: for every neighbour c the spring (v, c) with d = x_v - x_c, l = |d|, u = d/l,
// L = |r_v - r_c|: half its energy (k/4)(l - L)^2 (the other half comes from row c), the
// gradient k (l - L) u, and the PSD block He = k [u u^T + max(0, 1 - L/l)(I - u u^T)] (k I for a
// zero-length edge, whose gradient is 0): -He at (v, c), +He summed on the diagonal block,
// which also carries m I.  The gradient row adds w times the energy's gradient and
// m (x_v - x_prev,v); the energy adds (m/2)|x_v - x_prev,v|^2.
__global__ void __launch_bounds__(kSB) k_qs_rows(int64_t nv, const int32_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col_idx, const double* __restrict__ x,
                                                 const double* __restrict__ rest, const double* __restrict__ x_prev,
                                                 double ks, double m, double w, const double* __restrict__ g_ttie,
                                                 double* __restrict__ grad, double* __restrict__ vals,
                                                 double* __restrict__ part, Counters* ctr) {
  __shared__ double red[kSB];
  double esum = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kSB + threadIdx.x; v < nv; v += (int64_t)gridDim.x * kSB) {
    const double xv[3] = {x[3 * v], x[3 * v + 1], x[3 * v + 2]};
    const double rv[3] = {rest[3 * v], rest[3 * v + 1], rest[3 * v + 2]};
    double g[3] = {0.0, 0.0, 0.0};
    double D[9] = {m, 0.0, 0.0, 0.0, m, 0.0, 0.0, 0.0, m};
    int64_t dk = -1;
    for (int64_t kk = row_ptr[v]; kk < row_ptr[v + 1]; ++kk) {
      const int64_t c = col_idx[kk];
      if (c == v) {
        dk = kk;
        continue;
      }
      if (c < 0 || c >= nv) {
        atomicCAS(&ctr->status, 0, STATUS_INDEX);
        continue;
      }
      const double d[3] = {xv[0] - x[3 * c], xv[1] - x[3 * c + 1], xv[2] - x[3 * c + 2]};
      const double q[3] = {rv[0] - rest[3 * c], rv[1] - rest[3 * c + 1], rv[2] - rest[3 * c + 2]};
      const double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double Lr = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      esum += 0.25 * ks * (l - Lr) * (l - Lr);
      double He[9];
      if (l > 0.0) {
        const double u[3] = {d[0] / l, d[1] / l, d[2] / l};
        const double f = ks * (l - Lr);
        const double sc = fmax(0.0, 1.0 - Lr / l);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          g[a] += f * u[a];
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            const double uu = u[a] * u[b];
            He[3 * a + b] = ks * (uu + sc * ((a == b ? 1.0 : 0.0) - uu));
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < 9; ++a) He[a] = (a % 4 == 0) ? ks : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        D[a] += He[a];
        if (vals) vals[9 * kk + a] = -He[a];
      }
    }
    if (vals) {
      if (dk >= 0) {
#pragma unroll
        for (int a = 0; a < 9; ++a) vals[9 * dk + a] = D[a];
      } else {
        atomicCAS(&ctr->status, 0, STATUS_INVALID);  // the pattern lacks the diagonal block
      }
    }
    double dd = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double dx = xv[a] - x_prev[3 * v + a];
      dd += dx * dx;
      if (grad) grad[3 * v + a] = g[a] + (g_ttie ? w * g_ttie[3 * v + a] : 0.0) + m * dx;
    }
    esum += 0.5 * m * dd;
  }
  red[threadIdx.x] = esum;
  __syncthreads();
  for (int s = kSB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Phi = the fixed-order sum of the row partials + w E
__global__ void __launch_bounds__(kSB) k_qs_final(const double* __restrict__ part, int nparts, double w,
                                                  const double* __restrict__ e_ttie, double* __restrict__ phi) {
  __shared__ double red[kSB];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kSB) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = kSB / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *phi = red[0] + (e_ttie ? w * *e_ttie : 0.0);
}

hipError_t launch_qs_eval(Ctx* c, int64_t nv, const int32_t* row_ptr, const int32_t* col_idx, const double* x,
                          const double* rest, const double* x_prev, double ks, double m, double w,
                          const double* e_ttie, const double* g_ttie, double* phi, double* grad, double* vals,
                          hipStream_t s) {
  Counters* ctr = wsp<Counters>(c, c->L.counters);
  double* part = wsp<double>(c, c->L.epart_v);  // one partial per block (at most 4096 <= max_verts + 1)
  const unsigned g = sp_grid(nv);
  stage_begin(c, TTIE_STAGE_ELASTIC, s);
  k_qs_rows<<<g, kSB, 0, s>>>(nv, row_ptr, col_idx, x, rest, x_prev, ks, m, w, g_ttie, grad, vals, part, ctr);
  k_qs_final<<<1, kSB, 0, s>>>(part, (int)g, w, e_ttie, phi);
  stage_end(c, TTIE_STAGE_ELASTIC, s);
  return hipGetLastError();
}

}  // namespace ttie
