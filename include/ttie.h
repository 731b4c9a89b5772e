/*
 * ttie.h -- C ABI of libttie.so, the MI355X (gfx950) hot path of the triangle-triangle
 * intersection energy (TTIE) of "Differentiable 3D Triangle-Triangle Intersection Energy".
 *
 * For every candidate pair of triangles (T_a = tris[i], T_b = tris[j]) the library runs
 * Moeller's reduction (Sec. 1, Fig. 1; appendix `intersects`) to the intervals I_a, I_b on
 * the intersection line of the two planes, forms the Minkowski interval
 * I_c = [t_c^0, t_c^1] = [t_a^0 - t_b^1, t_a^1 - t_b^0] (Eq. 1), decides the open-interval
 * criterion 0 in (t_c^0, t_c^1) exactly, and on intersecting pairs evaluates the energy
 * T = (t_c^0 t_c^1)^2 (Eq. 2), its 18-dof gradient (Eq. 3) and the inexact Hessian of Eq. 4
 * made positive semi-definite from the eigenanalysis of Sec. 1.1.  The per-pair pieces are
 * assembled into a global energy, a dense gradient and a 3x3-block CSR (BSR) Hessian.
 *
 * Conventions shared by every call
 *  - All array arguments are DEVICE pointers (memory of the current HIP device) unless the
 *    parameter name ends in `_host`.  The caller owns every buffer; the library never
 *    allocates device memory: its scratch space is one caller-provided workspace
 *    (ttie_workspace_size / ttie_set_workspace).
 *  - `stream` is a hipStream_t passed as void* (0 = the null stream).  Calls enqueue work
 *    on it and return without waiting, except where a call says it synchronizes.
 *  - A context's workspace carries state from call to call (the last evaluation's hits, the
 *    broad phase's tree, counters kept zero between calls), so the calls on one context must
 *    be ordered: one stream, or streams ordered by events.  Unordered calls on one context
 *    race; work that runs concurrently takes one context each.  The library keeps no
 *    global state, so separate contexts are independent (also on one device).
 *  - Positions x: n_verts x 3 float64, row-major (x0,y0,z0,x1,...).  Triangles: n_tris x 3
 *    int32 vertex indices.  Pairs: n_pairs x 2 int32 triangle indices (i, j), i != j; the
 *    degrees of freedom of a pair are ordered (u0,u1,u2,v0,v1,v2) with u = tris[i] (T_a)
 *    and v = tris[j] (T_b).
 *  - Every call returns a ttie_status and never aborts or throws.  Errors detected on the
 *    host return immediately; errors found by kernels (an index out of range, a non-finite
 *    or out-of-domain coordinate, an overflowed capacity) are latched in a device status
 *    word read by ttie_get_status.  ttie_last_error() describes the last host-side error
 *    of the calling thread.
 *  - Coordinates must be finite and each either 0 or of magnitude in [2^-200, 2^200]: on
 *    that domain the exact orientation predicates below are exact and never overflow.
 *
 * Readings of the paper fixed by this library (the paper is silent on them)
 *  - plane sides and the intersection flag are exact (sign of orientation determinants,
 *    semi-static FP64 filter, exact fixed-point fallback); pairs sharing a vertex index are
 *    "adjacent" and carry no energy (Sec. 1 excludes topologically adjacent pairs);
 *  - T is gated by the flag: T = (t_c^0 t_c^1)^2 on intersecting pairs, 0 otherwise;
 *  - I_c follows Eq. 1 by default; TTIE_INTERVAL_APPENDIX_HALF halves both ends as the
 *    appendix does (T scales by exactly 1/16);
 *  - the Eq. 4 Hessian is J^T M J with J = [dt_c^0; dt_c^1] (2 x 18) and a 2x2 core M chosen
 *    by the PSD mode (see ttie_options).
 */
#ifndef TTIE_H
#define TTIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ttie_status {
  TTIE_OK = 0,
  TTIE_ERR_INVALID_ARGUMENT = 1,   /* null pointer, negative size, bad enum, i == j */
  TTIE_ERR_INDEX_OUT_OF_RANGE = 2, /* a pair or triangle index outside its array */
  TTIE_ERR_NONFINITE_INPUT = 3,    /* NaN or Inf coordinate */
  TTIE_ERR_CAPACITY = 4,           /* an output or the workspace is too small */
  TTIE_ERR_HIP = 5,                /* a HIP runtime call failed */
  TTIE_ERR_NO_DEVICE = 6,          /* no usable GPU */
  TTIE_ERR_UNSUPPORTED = 7,        /* coordinate outside the exact-predicate domain */
  TTIE_ERR_INTERNAL = 8            /* a bounded device-side wait ran out (a library fault) */
} ttie_status;

/* precision policy */
enum { TTIE_FP64 = 0, TTIE_MIXED = 1 };
/* 2x2 core of the per-pair Hessian J^T M J (s = t_c^0 t_c^1, a = dt_c^0, b = dt_c^1):
 *  PER_PART      parts 1 and 2 of Eq. 4 (PSD, Sec. 1.1) plus the non-negative eigencomponent
 *                of part 3: M = [[2 t1^2 + 2|s||b|/|a|, 2 s/|s|*|s|], [.., 2 t0^2 + 2|s||a|/|b|]]
 *  NEAREST       Eq. 4 with its negative eigenvalues clamped to 0 (nearest PSD matrix)
 *  PAPER_LITERAL parts 1 and 2, plus part 3 only when its trace 8 s a.b is positive
 *                (not PSD in general)
 *  RAW_EQ4       Eq. 4 unchanged (indefinite on every intersecting pair) */
enum { TTIE_PSD_PER_PART = 0, TTIE_PSD_NEAREST = 1, TTIE_PSD_PAPER_LITERAL = 2, TTIE_PSD_RAW_EQ4 = 3 };
enum { TTIE_INTERVAL_EQ1 = 0, TTIE_INTERVAL_APPENDIX_HALF = 1 };
enum { TTIE_BROAD_BRUTE = 0, TTIE_BROAD_LBVH = 1, TTIE_BROAD_HASH = 2 };
/* Pairs sharing a vertex index are adjacent (Sec. 1): the broad phase never lists them and the
 * evaluation gives them T = 0.  The paper leaves aside triangles that share a vertex and still
 * cross each other beyond it (a fan folded over itself).  With these bits -- OR'ed into the
 * broad phase's method, set in ttie_options.flags -- a pair sharing exactly one vertex is
 * listed and evaluated like any other pair: the shared vertex lies exactly on both planes
 * (an on-plane endpoint of both segments), so two triangles that only touch there have
 * intervals meeting in a point and T = 0, while triangles that cross beyond it get T > 0.
 * Pairs sharing two vertices (an edge) stay adjacent. */
enum { TTIE_BROAD_VERTEX_ADJACENT = 0x100 };
enum { TTIE_EVAL_VERTEX_ADJACENT = 1 };
enum { TTIE_HVP_EXACT = 0, TTIE_HVP_PSD = 1 };
/* per-pair flag codes written by ttie_eval.  TTIE_PAIR_COPLANAR: the two triangles lie in one
 * plane and their interiors overlap (decided exactly).  Such a pair has no intersection
 * segment, so T = 0 as for every non-crossing pair (the paper sets coplanar pairs aside); the
 * flag tells the caller where the energy cannot see an overlap. */
enum { TTIE_PAIR_NONE = 0, TTIE_PAIR_HIT = 1, TTIE_PAIR_ADJACENT = 2, TTIE_PAIR_DEGENERATE_FRAME = 3,
       TTIE_PAIR_COPLANAR = 4 };

typedef struct ttie_ctx ttie_ctx;

typedef struct ttie_mesh {
  const double* x;      /* n_verts x 3 float64 */
  int64_t n_verts;
  const int32_t* tris;  /* n_tris x 3 int32 */
  int64_t n_tris;
} ttie_mesh;

typedef struct ttie_options {
  int32_t precision; /* TTIE_FP64: everything in float64.  TTIE_MIXED: plane sides,
                        endpoints, intervals, flag and T in float64; derivatives, gradient
                        and Hessian in float32 on pair-local coordinates */
  int32_t psd_mode;  /* TTIE_PSD_* */
  int32_t interval;  /* TTIE_INTERVAL_* */
  int32_t flags;     /* TTIE_EVAL_* bits (0: the paper's definition) */
} ttie_options;

/* Upper bounds that size the workspace.  max_pairs bounds the candidate list of
 * ttie_broadphase and of ttie_eval; max_hits bounds the intersecting pairs per evaluation;
 * max_blocks bounds the non-zero 3x3 blocks of the assembled Hessian. */
typedef struct ttie_limits {
  int64_t max_verts, max_tris, max_pairs, max_hits, max_blocks;
} ttie_limits;

/* ---- library and context ------------------------------------------------------------ */
const char* ttie_version(void);
/* Host-side description of the last error returned on this thread ("" if none). */
const char* ttie_last_error(void);

/* Creates a context bound to HIP device `device`.  TTIE_ERR_NO_DEVICE when no GPU is
 * visible (safe to call on a machine without one).  *out receives the context. */
ttie_status ttie_create(int device, ttie_ctx** out);
ttie_status ttie_destroy(ttie_ctx* ctx);

/* Bytes of device workspace needed for the given limits on the context's device. */
ttie_status ttie_workspace_size(ttie_ctx* ctx, const ttie_limits* limits, size_t* bytes_host);
/* Hands the context a caller-owned device buffer of `bytes` (>= ttie_workspace_size) and
 * the limits it was sized for; clears the buffer's persistent counters on `stream`.  The
 * buffer must stay alive and unused by the caller until the next ttie_set_workspace or
 * ttie_destroy. */
ttie_status ttie_set_workspace(ttie_ctx* ctx, const ttie_limits* limits, void* dptr, size_t bytes, void* stream);

/* Device status word latched by kernels since the last call to this function.  Waits for
 * `stream` to finish, returns the latched status in *status_host and clears it. */
ttie_status ttie_get_status(ttie_ctx* ctx, void* stream, ttie_status* status_host);

/* ---- broad phase (candidate pairs) ---------------------------------------------------
 * Writes the canonical candidate set {(i, j) : i < j, no shared vertex index} of the mesh
 * -- for TTIE_BROAD_LBVH and TTIE_BROAD_HASH restricted to pairs whose closed float64
 * bounding boxes overlap on all three axes -- into pairs (capacity x 2 int32, 8-byte aligned)
 * in an unspecified order, and the number of candidates into *n_pairs (device int64).
 * TTIE_BROAD_LBVH: a BVH over 30-bit Morton codes.  TTIE_BROAD_HASH: the spatial hashing of
 * Sec. 1.2 -- a uniform grid (cell size twice the mean largest box extent) whose cells are
 * hashed into buckets; it suits meshes of even triangle size: a box covering more than
 * 2^20 cells or lying far outside the grid latches TTIE_ERR_UNSUPPORTED, and more than
 * 8 (cell, triangle) entries per triangle of limits.max_tris latch TTIE_ERR_CAPACITY.  x_end (nullable,
 * n_verts x 3 float64) makes every box cover the triangle at both x and x_end, so the list
 * holds every pair that can intersect anywhere on the straight path from x to x_end (the
 * line search of the Newton consumer).  When the count exceeds `capacity` only the first
 * `capacity` pairs are written, *n_pairs still receives the full count and
 * TTIE_ERR_CAPACITY is latched.  capacity must not exceed limits.max_pairs. */
ttie_status ttie_broadphase(ttie_ctx* ctx, const ttie_mesh* mesh, int method, const double* x_end, int32_t* pairs,
                            int64_t capacity, int64_t* n_pairs, void* stream);

/* ---- evaluation -----------------------------------------------------------------------
 * Evaluates the candidate pairs and assembles the energy, gradient and Hessian: per pair the
 * screening and intervals of Sec. 1 and Eq. 1, T of Eq. 2, its gradient (Eq. 3) and the Eq. 4
 * Hessian made PSD as in Sec. 1.1; then the sums over the pairs into one energy, one gradient
 * and one block-sparse matrix (Sec. 1.2).
 *  pairs      pair_capacity x 2 int32 candidate list (8-byte aligned); the number of pairs evaluated is
 *             n = min(*n_pairs, pair_capacity), *n_pairs being a device int64 (so the output of
 *             ttie_broadphase can be passed directly); pair_capacity <= limits.max_pairs
 *  energy     device float64 scalar: E = sum of T over the pairs (accumulated in float64)
 *  grad       n_verts x 3, float64 (TTIE_FP64) or float32 (TTIE_MIXED); every row written
 *  flags      optional (may be NULL): pair_capacity bytes, TTIE_PAIR_* for the first n
 *  pair_T     optional (may be NULL): pair_capacity float64, T of each of the first n pairs
 *  row_ptr, col_idx, vals   optional BSR Hessian (all NULL to skip assembly): row_ptr is
 *             n_verts + 1 int32, col_idx holds up to block_capacity int32 (sorted per row),
 *             vals block_capacity x 3 x 3 (row-major blocks; float64 or float32 by
 *             precision).  The pattern is the union over intersecting pairs of their 6x6
 *             vertex blocks, stored symmetric in full.
 *  n_blocks   optional device int64: number of non-zero blocks (nnzb); on overflow the
 *             full count is written and TTIE_ERR_CAPACITY latched
 *  n_hits     optional device int64: number of intersecting pairs
 * The intersecting pairs and their derivative records are kept in the workspace for
 * ttie_hvp and ttie_get_hits until the next ttie_eval.  No host synchronization. */
ttie_status ttie_eval(ttie_ctx* ctx, const ttie_mesh* mesh, const int32_t* pairs, const int64_t* n_pairs,
                      int64_t pair_capacity, const ttie_options* opts, double* energy, void* grad, uint8_t* flags, double* pair_T,
                      int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity, int64_t* n_blocks,
                      int64_t* n_hits, void* stream);

/* ---- evaluation without a workspace --------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  The same evaluation as ttie_eval (same
 * kernels, same results bit for bit), run in a file-scope device array of
 * TTIE_STATIC_SCRATCH_BYTES that every GPU the library runs on holds until the process ends,
 * in place of the caller's workspace: it needs a context (ttie_create looks the array's
 * address up on the context's device) but no ttie_set_workspace, and calls no allocating
 * routine (no hipMalloc, no events).
 *  max_hits   the intersecting-pair capacity the array is laid out for (as limits.max_hits)
 *  status     optional device int32: 0, or the TTIE_ERR_* code the kernels of this call
 *             detected (index out of range, non-finite coordinate, capacity) -- the status
 *             word that ttie_get_status reads for ttie_eval, which this call does not touch
 *  the other arguments as ttie_eval; pair_capacity and block_capacity also size the layout.
 * Returns TTIE_ERR_CAPACITY, before anything runs, when n_verts, pair_capacity, max_hits and
 * block_capacity need more than TTIE_STATIC_SCRATCH_BYTES (about 9 B per vertex, 10 B per
 * listed pair and 2 KB per hit).  Every call on one GPU uses that GPU's one array and finds
 * the last call's contents in it (the counts that must start at zero are cleared by fill
 * kernels at the start of each call): calls that overlap on one GPU -- two streams, two
 * threads, two contexts -- race, and the caller must order them.  ttie_get_hits, ttie_hvp and
 * the ttie_bsr_* calls refer to the context's last ttie_eval, never to this call. */
#define TTIE_STATIC_SCRATCH_BYTES (64ll << 20)
ttie_status ttie_eval_static(ttie_ctx* ctx, const ttie_mesh* mesh, const int32_t* pairs, const int64_t* n_pairs,
                             int64_t pair_capacity, int64_t max_hits, const ttie_options* opts, double* energy,
                             void* grad, uint8_t* flags, double* pair_T, int32_t* row_ptr, int32_t* col_idx, void* vals,
                             int64_t block_capacity, int64_t* n_blocks, int64_t* n_hits, int32_t* status,
                             void* stream);

/* ---- batches of independent problems --------------------------------------------------
 * Many independent problems (each a mesh, or the union of several meshes, whose pairs are
 * evaluated among themselves only) in one call: the hot path of Sec. 1 applied problem by
 * problem, with every stage one launch for the whole batch.  The caller concatenates the
 * problems into one ttie_mesh: problem p owns vertices [vert_off[p], vert_off[p+1]) and
 * triangles [tri_off[p], tri_off[p+1]), and its triangles index vertices with global ids.
 * vert_off and tri_off are DEVICE int64 arrays of n_problems + 1 entries, non-decreasing, from
 * 0 to n_verts and n_tris.  1 <= n_problems <= TTIE_MAX_PROBLEMS. */
#define TTIE_MAX_PROBLEMS 4096

/* LBVH broad phase of a batch: as ttie_broadphase with TTIE_BROAD_LBVH, except that no pair
 * joins triangles of two problems (one tree over the batch; each query searches only the
 * sorted range of its own problem).  tri_off that does not tile [0, n_tris) latches
 * TTIE_ERR_INVALID_ARGUMENT. */
ttie_status ttie_batch_broadphase(ttie_ctx* ctx, const ttie_mesh* mesh, int n_problems, const int64_t* tri_off,
                                  const double* x_end, int32_t* pairs, int64_t capacity, int64_t* n_pairs,
                                  void* stream);

/* Evaluation of a batch: exactly ttie_eval over the concatenated mesh (the Hessian of a
 * batch is block diagonal, problem by problem, when no pair joins two problems), plus
 * energies (device float64, n_problems): energies[p] is the sum of T over the intersecting
 * pairs whose first vertex (vertex 0 of the pair's first triangle) lies in problem p, summed
 * per vertex and then in vertex order.  vert_off that does not tile [0, n_verts) latches
 * TTIE_ERR_INVALID_ARGUMENT. */
ttie_status ttie_batch_eval(ttie_ctx* ctx, const ttie_mesh* mesh, int n_problems, const int64_t* vert_off,
                            const int32_t* pairs, const int64_t* n_pairs, int64_t pair_capacity,
                            const ttie_options* opts, double* energies, double* energy, void* grad, uint8_t* flags,
                            double* pair_T, int32_t* row_ptr, int32_t* col_idx, void* vals, int64_t block_capacity,
                            int64_t* n_blocks, int64_t* n_hits, void* stream);

/* Copies the last evaluation's intersecting pairs, sorted by (i, j), to HOST buffers of
 * `capacity` entries: pair indices (i, j) int32 x 2, t_c (float64 x 2, Eq. 1), T (float64,
 * Eq. 2), the interval gradients a = dt_c^0, b = dt_c^1 and the pair's energy gradient
 * g = 2 t0 t1^2 a + 2 t0^2 t1 b (Eq. 3) (float64 x 18 each, converted from the evaluation's
 * precision), and the 2x2 core M of the pair's Hessian J^T M J (float64 x 3: M00, M01, M11;
 * Eq. 4 as projected by the evaluation's PSD mode).  Synchronizes `stream`; *count_host
 * receives the hit count (TTIE_ERR_CAPACITY if it exceeds capacity).  Any output pointer may be
 * NULL.  A diagnostic call (host copies): it is in no timed path. */
ttie_status ttie_get_hits(ttie_ctx* ctx, int64_t capacity, int32_t* ij_host, double* tc_host, double* T_host,
                          double* a_host, double* b_host, double* g_host, double* M_host, int64_t* count_host,
                          void* stream);

/* ---- the Hessian as two calls: pattern, then values --------------------------------------
 * The BSR Hessian of the last ttie_eval (Eq. 4 per pair as projected by its PSD mode, summed
 * over the intersecting pairs; Sec. 1.2 records each pair's derivatives to build the global
 * matrix), split so that a caller can size the pattern before taking the values and refresh the
 * values on a pattern it keeps.  Both read the hit records and incidence lists that ttie_eval
 * leaves in the workspace (valid until the next ttie_eval or ttie_springs_pattern); the ttie_eval
 * call itself may have skipped its own BSR output.
 *
 * ttie_bsr_symbolic: the pattern -- the union over intersecting pairs of their 6 x 6 vertex
 * blocks, full symmetric storage, columns sorted per row.  row_ptr: n_verts + 1 int32 (every
 * entry written); col_idx: up to `capacity` int32; *n_blocks (device int64, 8-byte aligned)
 * receives nnzb.  When nnzb exceeds capacity only the columns that fit are written and
 * TTIE_ERR_CAPACITY is latched (row_ptr and *n_blocks are still complete, so the caller can
 * size col_idx from them and call again). */
ttie_status ttie_bsr_symbolic(ttie_ctx* ctx, int32_t* row_ptr, int32_t* col_idx, int64_t capacity,
                              int64_t* n_blocks, void* stream);

/* ttie_bsr_numeric: the values on a caller's pattern (row_ptr, col_idx with sorted columns, over
 * the last evaluation's n_verts rows), e.g. one from ttie_bsr_symbolic of an earlier evaluation.
 * vals: row_ptr[n_verts] x 3 x 3 in the last evaluation's precision, every block written: the
 * blocks the hits give, summed in the order of ttie_eval's own assembly (identical values on
 * the same pattern), and 0 elsewhere.  A pattern that misses a block the hits need latches
 * TTIE_ERR_INVALID_ARGUMENT (the values are then incomplete). */
ttie_status ttie_bsr_numeric(ttie_ctx* ctx, const int32_t* row_ptr, const int32_t* col_idx, void* vals,
                             void* stream);

/* Hessian-vector product of the energy at the positions of the last ttie_eval (same mesh
 * and x): Hv = H v, v and Hv n_verts x 3 in the evaluation's precision (the second derivative
 * of the summed Eq. 2 energy, or the Eq. 4 / Sec. 1.1 PSD form).  mode
 * TTIE_HVP_EXACT: the exact Hessian of the summed energy (forward-mode differentiation of
 * the gradient along v, through the line direction and the lerp weights); TTIE_HVP_PSD:
 * the assembled Hessian of the evaluation's PSD mode applied matrix-free. */
ttie_status ttie_hvp(ttie_ctx* ctx, const ttie_mesh* mesh, const void* v, void* Hv, int mode, void* stream);

/* y = H x with a BSR matrix from ttie_eval (the summed Eq. 4 blocks of Sec. 1.2; precision as
 * in opts->precision); n_rows = n_verts.  Used by the Newton consumer. */
ttie_status ttie_bsr_mv(ttie_ctx* ctx, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                        const void* vals, const void* x, void* y, int precision, void* stream);

/* ---- inexact Newton consumer (the abstract's GPU inexact-Newton route) -----------------
 * Jacobi-preconditioned conjugate gradients on (H + mu I) x = scale * b, entirely on the
 * device (no host synchronization): H is a BSR matrix from ttie_eval (n_rows = n_verts),
 * mu = mu_rel * (mean diagonal entry of H over the rows that hold blocks), the Jacobi
 * preconditioner is the diagonal of H + mu I, x starts at 0, and the iteration stops after
 * max_iter steps or when |r| <= tol |scale b|.  b and x are n_rows x 3 in the precision of
 * vals; reductions accumulate in float64 in a fixed order.  info (device, 4 float64, may be
 * NULL) receives {iterations, |r| / |b|, mu, x . (scale b)}.
 * The iteration runs over the rows that hold blocks: elsewhere H + mu I is mu I, and b must be
 * 0 there (a gradient from ttie_eval is), so the solution is 0 there too; a non-zero b on such
 * a row latches TTIE_ERR_INVALID_ARGUMENT.  Each iteration thus costs in proportion to the rows
 * the hits touch, not to n_rows. */
ttie_status ttie_pcg(ttie_ctx* ctx, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                     const void* b, double scale, void* x, double mu_rel, int max_iter, double tol, int precision,
                     double* info, void* stream);

/* Matrix-free variant of ttie_pcg (the same iteration, mu and preconditioner, over the rows
 * the last evaluation's hits touch; b must be 0 on the others): H is the PSD
 * Hessian of the last ttie_eval, applied from its per-hit records as the sum over hits of
 * J^T M J (J = [a^T; b^T], Eq. 4 with the evaluation's PSD core) without assembling the BSR
 * matrix; its diagonal comes from the same records.  n_rows must equal the last evaluation's
 * n_verts; b and x are in that evaluation's precision.  Valid until the next ttie_eval. */
ttie_status ttie_pcg_mf(ttie_ctx* ctx, int64_t n_rows, const void* b, double scale, void* x, double mu_rel,
                        int max_iter, double tol, double* info, void* stream);

/* ---- quasi-static coupling with a synthetic elastic model -----------------------------
 * The paper's quasi-static simulation (Fig. 2) drives an intersecting state to an
 * intersection-free one with the energy paired with an elastic model it does not give.  The
 * stand-in: springs on the mesh's edges, and the objective of one quasi-static step
 *   Phi(x) = sum over edges (k/2)(|x_i - x_j| - |r_i - r_j|)^2 + w E(x) + (m/2)|x - x_prev|^2
 * (r: rest positions, x_prev: positions at the step's start), minimised by inexact Newton with
 * A = K + w H, K the springs' Hessian with each edge block projected to PSD plus m I, H the PSD
 * Hessian of the energy applied from the hit records (ttie_pcg_coupled).
 *
 * ttie_springs_pattern: the 3x3-block CSR pattern of K, row v holding v and its neighbours in
 * the mesh's edge graph in increasing order.  row_ptr: n_verts + 1 int32; col_idx: up to
 * block_capacity int32; *n_blocks (device int64) receives the block count, and a count above
 * block_capacity latches TTIE_ERR_CAPACITY (rows that fit are still written).  Vertex indices
 * outside [0, n_verts) latch TTIE_ERR_INDEX_OUT_OF_RANGE.  Uses the evaluation's incidence
 * buffers, so the last evaluation is no longer available to ttie_hvp / ttie_pcg_mf. */
ttie_status ttie_springs_pattern(ttie_ctx* ctx, const ttie_mesh* mesh, int32_t* row_ptr, int32_t* col_idx,
                                 int64_t block_capacity, int64_t* n_blocks, void* stream);

/* ttie_qs_eval: Phi, its gradient and K at x (all device float64; n_verts x 3 arrays).
 *  row_ptr, col_idx  the pattern from ttie_springs_pattern
 *  x, rest, x_prev   positions, rest positions, positions at the step's start
 *  k, m, w           spring stiffness (>= 0), proximal weight (>= 0), weight of the energy (>= 0)
 *  e_ttie, g_ttie    E (device scalar) and its gradient (n_verts x 3, float64) from a
 *                    TTIE_FP64 ttie_eval at x; both NULL when w = 0
 *  phi               device scalar: Phi(x)
 *  grad, vals        optional (NULL skips): grad Phi, and K's blocks in the pattern's order
 * Per edge with d = x_i - x_j, l = |d|, u = d / l, L = |r_i - r_j|: the PSD block is
 * k [u u^T + max(0, 1 - L/l)(I - u u^T)], or k I for a zero-length edge (whose gradient is 0).
 * Deterministic: rows are summed in column order, Phi in a fixed order. */
ttie_status ttie_qs_eval(ttie_ctx* ctx, int64_t n_verts, const int32_t* row_ptr, const int32_t* col_idx,
                         const double* x, const double* rest, const double* x_prev, double k, double m, double w,
                         const double* e_ttie, const double* g_ttie, double* phi, double* grad, double* vals,
                         void* stream);

/* ttie_pcg_coupled: Jacobi-PCG (the iteration of ttie_pcg, over the rows where K holds blocks
 * or the hits touch; b must be 0 on the others) on (K + w H + mu I) x = scale * b,
 * with K a PSD 3x3-block CSR matrix in float64 (columns sorted per row, e.g. from
 * ttie_qs_eval) and H the PSD Hessian of the last ttie_eval, which must be TTIE_FP64 and
 * have n_verts = n_rows.  mu >= 0 is absolute.  info as for ttie_pcg (info[2] = mu). */
ttie_status ttie_pcg_coupled(ttie_ctx* ctx, int64_t n_rows, const int32_t* row_ptr, const int32_t* col_idx,
                             const double* vals, double w, const double* b, double scale, double* x, double mu,
                             int max_iter, double tol, double* info, void* stream);

/* ---- launch parameters (what an autotuner varies) ------------------------------------
 * Launch shapes and work budgets of the kernels.  Every value in range gives the same results
 * bit for bit (the evaluation sums in pair-key order and a candidate set does not depend on
 * the order of emission); only the speed changes.  A value of 0 restores the default. */
enum {
  TTIE_PARAM_SCREEN_BLOCKS = 0, /* blocks of the screening kernels: 64 .. 65536 (default 4096) */
  TTIE_PARAM_ROW_BLOCKS = 1,    /* blocks of ttie_bsr_symbolic's row kernel: 64 .. 65536 (default 2048) */
  TTIE_PARAM_TRAV_BUDGET = 2,   /* nodes a traversal lane visits before a whole wave takes over its
                                   query: 16 .. 2^20 (default 128) */
  TTIE_PARAM_HASH_BUDGET = 3,   /* later bucket entries a hash thread tests before a whole wave takes
                                   over the rest: 16 .. 2^20 (default 64) */
  TTIE_PARAM_SCREEN_TILE = 4,   /* candidates per tile of the screening's tile queue: a multiple of
                                   64 in 64 .. 2^20, raised if needed so that a list has at most
                                   2^18 tiles; the screening grid (TTIE_PARAM_SCREEN_BLOCKS) then
                                   stays resident and each wave takes the next tile from a
                                   device counter until the list is done.  Default 0: no queue,
                                   one contiguous chunk of the list per wave. */
  TTIE_PARAM_COUNT = 5
};
ttie_status ttie_set_param(ttie_ctx* ctx, int param, int64_t value);
ttie_status ttie_get_param(ttie_ctx* ctx, int param, int64_t* value_host);

/* out = x + alpha * d for n_verts x 3 positions: x and out float64, d in `precision`.  A result
 * of magnitude below 2^-200 is set to 0, so positions stay in the coordinate domain of the exact
 * predicates (0, or magnitude in [2^-200, 2^200]); a truncated solve can leave vanishing
 * components at far vertices. */
ttie_status ttie_axpy(ttie_ctx* ctx, int64_t n_verts, double alpha, const double* x, const void* d, double* out,
                      int precision, void* stream);

/* ---- stage timers ---------------------------------------------------------------------
 * When enabled (mask of 1 << TTIE_STAGE_*), the following calls record a HIP event pair on
 * their stream around every kernel of the selected stages.  ttie_read_timers waits for the
 * recorded events and returns, for stages 0..n_stages-1, the number of timed launches and
 * their summed duration in milliseconds since the previous read, then resets them. */
enum {
  TTIE_STAGE_BP_BOXES = 0,    /* triangle boxes, scene bounds, Morton bucket ranks (spatial hash: cells) */
  TTIE_STAGE_BP_SORT = 1,     /* counting sort by Morton bucket (spatial hash: by cell hash) */
  TTIE_STAGE_BP_BUILD = 2,    /* leaf records and the implicit 4-ary tree's boxes, bottom up */
  TTIE_STAGE_BP_TRAVERSE = 3, /* tree self-traversal / hash buckets / brute force, pair emission
                                 (the queries over the traversal budget go on in TTIE_STAGE_BP_HEAVY) */
  TTIE_STAGE_SCREEN = 4,      /* per-candidate screening with FP64 filters */
  TTIE_STAGE_SCREEN_EXACT = 5,/* re-screening of the deferred candidates with exact predicates */
  TTIE_STAGE_DERIVS = 6,      /* per-hit interval gradients, energy, gradient, Hessian core */
  TTIE_STAGE_ASSEMBLY = 7,    /* incidence lists, BSR pattern, rows of gradient and Hessian */
  TTIE_STAGE_HVP = 8,         /* Hessian-vector products */
  TTIE_STAGE_PCG = 9,         /* the preconditioned conjugate-gradient solve */
  TTIE_STAGE_ELASTIC = 10,    /* the quasi-static objective (springs, proximal term) */
  TTIE_STAGE_BP_HEAVY = 11,   /* broad-phase queries handed to a whole wave each (tree or hash) */
  TTIE_STAGE_COUNT = 12
};
ttie_status ttie_set_timing(ttie_ctx* ctx, uint32_t stage_mask);
ttie_status ttie_read_timers(ttie_ctx* ctx, int n_stages, int64_t* launches_host, double* total_ms_host);

#ifdef __cplusplus
}
#endif

#endif /* TTIE_H */
