"""Quasi-static coupling of the energy with a synthetic elastic model -- TEST INFRASTRUCTURE ONLY.

Only the test-suite and the benchmark's CPU-baseline leg use this module; the GPU path shares
no code with it.

The paper's quasi-static simulation (Fig. 2) starts from an intersecting state and ends
intersection-free, with the energy paired with an elastic model that the paper does not
give.  The stand-in here is a reading, stated in full so that it can be checked:

    Phi(x) = sum over mesh edges e = (i, j) of (k/2) (|x_i - x_j| - L_e)^2
             + w E(x) + (m/2) |x - x_prev|^2

with L_e = |r_i - r_j| from rest positions r, E the intersection energy (Eq. 2 summed over the
candidate pairs) and x_prev the positions at the start of the quasi-static step.  A step runs
inexact Newton on Phi from x_prev:
  * A d = -grad Phi with A = K + w H: K is the springs' Hessian with every edge block projected
    to PSD (the transverse eigenvalue k (1 - L/l) clamped at 0), plus m I; H is the PSD
    Hessian of Eq. 4 (the evaluation's PSD mode);
  * Jacobi-preconditioned CG from d = 0, the iteration of the Newton loop (relative residual
    tolerance, iteration cap);
  * Armijo backtracking on Phi along d, with candidates from boxes swept from x to x + d.
The simulation repeats steps until one starts with E = 0 (an intersection-free state).
"""

from __future__ import annotations

import numpy as np

from . import evaluate, pairs, pairs_swept


def spring_edges(tris):
    """The mesh's undirected edges (i < j), unique, in increasing (i, j) order."""
    t = np.asarray(tris, np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = e[e[:, 0] != e[:, 1]]
    return np.unique(e, axis=0)


def springs(x, rest, edges, k):
    """Energy, gradient (N, 3) and the PSD 3x3 Hessian block of every edge (ne, 3, 3).

    Per edge with d = x_i - x_j, l = |d|, u = d / l and L = |r_i - r_j|: energy
    (k/2)(l - L)^2, gradient k (l - L) u at i and its negative at j, and the block
    k [u u^T + max(0, 1 - L/l) (I - u u^T)] (the exact Hessian k [u u^T + (1 - L/l)(I - u u^T)]
    with its transverse eigenvalue clamped at 0).  A zero-length edge has no direction: its
    gradient is 0 and its block k I (a reading)."""
    x, rest = np.asarray(x, np.float64), np.asarray(rest, np.float64)
    d = x[edges[:, 0]] - x[edges[:, 1]]
    l = np.linalg.norm(d, axis=1)
    L = np.linalg.norm(rest[edges[:, 0]] - rest[edges[:, 1]], axis=1)
    E = 0.5 * k * float(np.sum((l - L) ** 2))
    ok = l > 0
    u = np.zeros_like(d)
    u[ok] = d[ok] / l[ok, None]
    f = (k * (l - L))[:, None] * u
    G = np.zeros_like(x)
    np.add.at(G, edges[:, 0], f)
    np.add.at(G, edges[:, 1], -f)
    uu = u[:, :, None] * u[:, None, :]
    s = np.zeros_like(l)
    s[ok] = np.maximum(0.0, 1.0 - L[ok] / l[ok])
    I = np.eye(3)
    He = k * (uu + s[:, None, None] * (I - uu))
    He[~ok] = k * I
    return E, G, He


def stiffness_bsr(n_verts, edges, He, m):
    """K = sum over edges of [[He, -He], [-He, He]] at (i, j), plus m I, as 3x3-block CSR:
    row v holds v and its neighbours in increasing order.  Returns (row_ptr, col_idx, vals)."""
    n = int(n_verts)
    i, j = edges[:, 0], edges[:, 1]
    v = np.arange(n)
    rows = np.concatenate([v, i, j])
    cols = np.concatenate([v, j, i])
    key = rows * n + cols
    uk = np.unique(key)
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, uk // n + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    col_idx = uk % n
    vals = np.zeros((len(uk), 3, 3))
    diag = np.searchsorted(uk, v * n + v)
    vals[diag] += m * np.eye(3)
    np.add.at(vals, np.searchsorted(uk, i * n + i), He)
    np.add.at(vals, np.searchsorted(uk, j * n + j), He)
    np.add.at(vals, np.searchsorted(uk, i * n + j), -He)
    np.add.at(vals, np.searchsorted(uk, j * n + i), -He)
    return row_ptr.astype(np.int32), col_idx.astype(np.int32), vals


def bsr_matvec(row_ptr, col_idx, vals, v):
    """y = M v for a 3x3-block CSR matrix and v of shape (N, 3)."""
    v = np.asarray(v, np.float64).reshape(-1, 3)
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    y = np.zeros_like(v)
    np.add.at(y, rows, np.einsum("kab,kb->ka", vals, v[col_idx]))
    return y


def bsr_diagonal(row_ptr, col_idx, vals, n_verts):
    """The diagonal entries (N, 3) of a 3x3-block CSR matrix (0 where a row has no diagonal block)."""
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    out = np.zeros((n_verts, 3))
    on = rows == col_idx
    out[rows[on]] = np.einsum("kaa->ka", vals[on])
    return out


def objective(x, rest, x_prev, tris, edges, pair_list, k, m, w, hessian=True):
    """Phi, grad Phi (N, 3), K as BSR (or None) and the evaluation of the energy E."""
    r = evaluate(x, tris, pair_list, hessian=hessian)
    Es, Gs, He = springs(x, rest, edges, k)
    dx = np.asarray(x, np.float64) - np.asarray(x_prev, np.float64)
    phi = Es + w * r["E"] + 0.5 * m * float(np.sum(dx * dx))
    grad = Gs + w * r["G"] + m * dx
    K = stiffness_bsr(len(x), edges, He, m) if hessian else None
    return phi, grad, K, r


def pcg(apply, b, diag, max_iter, tol):
    """Jacobi-preconditioned CG on A d = b from d = 0 (the Newton loop's iteration)."""
    b = b.ravel()
    dinv = np.where(diag.ravel() > 0, 1.0 / np.where(diag.ravel() > 0, diag.ravel(), 1.0), 1.0)
    d = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    bb = b @ b
    it = 0
    while it < max_iter:
        q = apply(p)
        pq = p @ q
        if not pq > 0:
            break
        a = rz / pq
        d += a * p
        r -= a * q
        z = dinv * r
        rzn, rr = r @ z, r @ r
        it += 1
        if rr <= tol * tol * bb:
            break
        p = z + (rzn / rz if rz > 0 else 0.0) * p
        rz = rzn
    return d, it


def flush_tiny(x):
    """Coordinates of magnitude below 2^-200 set to 0: trial positions stay in the exact
    predicates' coordinate domain (0, or magnitude in [2^-200, 2^200]), as in the Newton loop."""
    x = np.asarray(x, np.float64)
    return np.where(np.abs(x) < 2.0 ** -200, 0.0, x)


def qs_step(x_prev, rest, tris, k, m, w, newton_iters=4, pcg_iters=50, pcg_tol=1e-6, armijo_c=1e-4, beta=0.5,
            max_halvings=30, solve=None):
    """One quasi-static step: ``newton_iters`` inexact Newton iterations on Phi from x_prev.
    ``solve(K, H_bsr, w, b)`` replaces the PCG when given (tests use a dense solve).
    Returns the new positions and one record per iteration."""
    edges = spring_edges(tris)
    x_prev = np.asarray(x_prev, np.float64)
    x = x_prev.copy()
    recs = []
    for _ in range(newton_iters):
        pl = pairs(x, tris)
        phi, g, K, r = objective(x, rest, x_prev, tris, edges, pl, k, m, w)
        H = (r["row_ptr"], r["col_idx"], r["vals"])
        if solve is not None:
            d, its = solve(K, H, w, -g), 0
        else:
            diag = bsr_diagonal(*K, len(x)) + w * bsr_diagonal(*H, len(x))

            def apply(p):
                return (bsr_matvec(*K, p) + w * bsr_matvec(*H, p)).ravel()

            d, its = pcg(apply, -g.ravel(), diag, pcg_iters, pcg_tol)
        d = d.reshape(-1, 3)
        gd = float(np.sum(g * d))
        sw = pairs_swept(x, flush_tiny(x + d), tris)
        alpha = 1.0
        for h in range(max_halvings):
            xt = flush_tiny(x + alpha * d)
            phit = objective(xt, rest, x_prev, tris, edges, sw, k, m, w, hessian=False)[0]
            if phit <= phi + armijo_c * alpha * gd:
                break
            if h + 1 < max_halvings:
                alpha *= beta
        recs.append({"phi": phi, "E": r["E"], "hits": len(r["hit_pair"]), "alpha": alpha, "pcg_iters": its,
                     "phi_new": phit})
        x = xt
    return x, recs


def quasi_static(x0, rest, tris, steps, k, m, w, **kw):
    """Quasi-static steps from x0 until a step starts intersection-free (E = 0) or ``steps``
    steps ran.  Returns the final positions and the list of per-step records
    {E (at the step's start), hits, newton: [...]}."""
    x = np.asarray(x0, np.float64).copy()
    hist = []
    for _ in range(steps):
        r = evaluate(x, tris, pairs(x, tris), hessian=False)
        if r["E"] == 0.0:
            hist.append({"E": 0.0, "hits": 0, "newton": []})
            return x, hist
        x, recs = qs_step(x, rest, tris, k, m, w, **kw)
        hist.append({"E": r["E"], "hits": len(r["hit_pair"]), "newton": recs})
    r = evaluate(x, tris, pairs(x, tris), hessian=False)
    hist.append({"E": r["E"], "hits": len(r["hit_pair"]), "newton": []})
    return x, hist
