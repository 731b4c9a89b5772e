"""CPU oracle for the triangle-triangle intersection energy -- TEST INFRASTRUCTURE ONLY.

Plain FP64 reference implementation written from the paper (Sec. 1: Moeller reduction,
Eq. 1 interval, Eq. 2 energy; Sec. 1.1: Eq. 3 gradient, Eq. 4 inexact Hessian and its
eigenanalysis; appendix: the dual-number algorithm).  Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does.

``libttie_oracle.so`` (``ttie_oracle.cpp``) does the arithmetic; this module only marshals
numpy arrays.  ``exact_moller`` is a separate, exact-rational implementation used to pin the
oracle's intersection flags and interval values.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build_oracle

INTERVAL_EQ1, INTERVAL_APPENDIX_HALF = 0, 1
PSD_PER_PART, PSD_NEAREST, PSD_PAPER_LITERAL, PSD_RAW_EQ4 = 0, 1, 2, 3
ST_NONE, ST_HIT, ST_ADJACENT, ST_BAD_FRAME, ST_COPLANAR = 0, 1, 2, 3, 4
BROAD_BRUTE, BROAD_BOXES = 0, 1

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_bp = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.LIB
        if not os.path.exists(path):
            build_oracle.build()
        L = ctypes.CDLL(path)
        L.ttie_oracle_threads.argtypes = []
        L.ttie_oracle_threads.restype = ctypes.c_int
        L.ttie_oracle_orient_sign.argtypes = [_dp] * 4
        L.ttie_oracle_orient_sign.restype = ctypes.c_int
        L.ttie_oracle_pair.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.ttie_oracle_pair.restype = ctypes.c_int
        L.ttie_oracle_pair_hvp.argtypes = [_dp, ctypes.c_int, _dp, _dp]
        L.ttie_oracle_pair_hvp.restype = ctypes.c_int
        L.ttie_oracle_eig.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.ttie_oracle_eig.restype = None
        L.ttie_oracle_pairs.argtypes = [_dp, ctypes.c_int64, _ip, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _lp]
        L.ttie_oracle_pairs.restype = ctypes.c_void_p
        L.ttie_oracle_free.argtypes = [ctypes.c_void_p]
        L.ttie_oracle_free.restype = None
        L.ttie_oracle_pairs_swept.argtypes = [_dp, _dp, ctypes.c_int64, _ip, ctypes.c_int64, _lp]
        L.ttie_oracle_pairs_swept.restype = ctypes.c_void_p
        L.ttie_oracle_newton.argtypes = [_dp, ctypes.c_int64, _ip, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp,
                                         ctypes.POINTER(ctypes.c_int)]
        L.ttie_oracle_newton.restype = ctypes.c_int
        L.ttie_oracle_eval.argtypes = [_dp, ctypes.c_int64, _ip, ctypes.c_int64, _ip, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.ttie_oracle_eval.restype = ctypes.c_void_p
        L.ttie_oracle_eval_sizes.argtypes = [ctypes.c_void_p, _lp, _lp]
        L.ttie_oracle_eval_sizes.restype = ctypes.c_int
        L.ttie_oracle_eval_fetch.argtypes = [ctypes.c_void_p, _bp, _dp, _dp, _dp, _dp, _lp, _dp, _dp, _dp,
                                             _dp, _dp, _ip, _ip, _dp]
        L.ttie_oracle_eval_fetch.restype = None
        L.ttie_oracle_eval_free.argtypes = [ctypes.c_void_p]
        L.ttie_oracle_eval_free.restype = None
        L.ttie_oracle_hvp.argtypes = [_dp, ctypes.c_int64, _ip, ctypes.c_int64, _ip, ctypes.c_int64, _dp,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int]
        L.ttie_oracle_hvp.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def threads() -> int:
    """Threads the oracle's parallel loops use (OMP_NUM_THREADS or all cores)."""
    return lib().ttie_oracle_threads()


def orient_sign(a, b, c, p) -> int:
    """Exact sign of det[b-a, c-a, p-a] (which side of plane (a,b,c) point p lies on)."""
    a, b, c, p = (_f64(v) for v in (a, b, c, p))
    return lib().ttie_oracle_orient_sign(_d(a), _d(b), _d(c), _d(p))


def pair(X, interval=INTERVAL_EQ1, psd=PSD_PER_PART):
    """One triangle pair; X is (6,3): u0,u1,u2 (T_a) then v0,v1,v2 (T_b).

    Returns dict(status, t0, t1, T, a, b, g, H) with a = dt_c^0/dX, b = dt_c^1/dX,
    g = dT/dX (18-vectors in (u0,u1,u2,v0,v1,v2) order) and H the 18x18 Hessian of ``psd``.
    """
    X = _f64(X).reshape(18)
    t01 = np.zeros(2)
    T = np.zeros(1)
    a, b, g = np.zeros(18), np.zeros(18), np.zeros(18)
    H = np.zeros((18, 18))
    st = lib().ttie_oracle_pair(_d(X), interval, psd, _d(t01), _d(T), _d(a), _d(b), _d(g), _d(H))
    return dict(status=st, t0=t01[0], t1=t01[1], T=T[0], a=a, b=b, g=g, H=H)


def pair_hvp(X, v, interval=INTERVAL_EQ1):
    """Exact (nested-dual) Hessian-vector product of T for one pair; zeros if not a hit."""
    X = _f64(X).reshape(18)
    v = _f64(v).reshape(18)
    out = np.zeros(18)
    lib().ttie_oracle_pair_hvp(_d(X), interval, _d(v), _d(out))
    return out


def eig(A):
    """Jacobi eigen-decomposition used inside the oracle (exposed so it can be pinned)."""
    A = _f64(A)
    n = A.shape[0]
    w, Q = np.zeros(n), np.zeros((n, n))
    lib().ttie_oracle_eig(n, _d(A), _d(w), _d(Q))
    return w, Q


def pairs(x, tris, method=BROAD_BOXES, vertex_adjacent=False):
    """Canonical sorted candidate list (P, 2) int32: i < j, no shared vertex (with
    ``vertex_adjacent``: at most one shared vertex), and for BROAD_BOXES closed FP64 bounding
    boxes overlapping."""
    x, tris = _f64(x), _i32(tris)
    n = ctypes.c_int64(0)
    ptr = lib().ttie_oracle_pairs(_d(x), len(x), _i(tris), len(tris), method, 1 if vertex_adjacent else 0,
                                  ctypes.byref(n))
    try:
        out = np.ctypeslib.as_array(ctypes.cast(ptr, _ip), shape=(max(1, 2 * n.value),))[: 2 * n.value].copy()
    finally:
        lib().ttie_oracle_free(ptr)
    return out.reshape(-1, 2)


def pairs_swept(x, x_end, tris):
    """Candidates whose boxes, swept from x to x_end, overlap (canonical sorted list)."""
    x, x_end, tris = _f64(x), _f64(x_end), _i32(tris)
    n = ctypes.c_int64(0)
    ptr = lib().ttie_oracle_pairs_swept(_d(x), _d(x_end), len(x), _i(tris), len(tris), ctypes.byref(n))
    try:
        out = np.ctypeslib.as_array(ctypes.cast(ptr, _ip), shape=(max(1, 2 * n.value),))[: 2 * n.value].copy()
    finally:
        lib().ttie_oracle_free(ptr)
    return out.reshape(-1, 2)


def newton(x, tris, steps=20, pcg_iters=50, pcg_tol=1e-6, mu_rel=1e-3, armijo_c=1e-4, beta=0.5, max_halvings=30,
           interval=INTERVAL_EQ1, psd=PSD_PER_PART, threads=0):
    """Inexact Newton with the PSD Hessian, Jacobi-PCG and Armijo backtracking (FP64).
    Returns (x_final, energies (steps+1,), step lengths (steps,), PCG iterations (steps,))."""
    x = _f64(x).copy()
    tris = _i32(tris)
    E = np.zeros(steps + 1)
    al = np.zeros(steps)
    its = np.zeros(steps, np.int32)
    lib().ttie_oracle_newton(_d(x), len(x), _i(tris), len(tris), steps, pcg_iters, pcg_tol, mu_rel, armijo_c, beta,
                             max_halvings, interval, psd, threads, _d(E), _d(al),
                             its.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return x, E, al, its


def evaluate(x, tris, pair_list, interval=INTERVAL_EQ1, psd=PSD_PER_PART, hessian=True, threads=0,
             vertex_adjacent=False):
    """Energy, gradient and block-sparse Hessian over a candidate list.

    Returns a dict with per-pair ``flags`` (0 none, 1 hit, 2 adjacent, 3 hit with a
    degenerate line frame, 4 coplanar with overlapping interiors, T = 0), ``t`` (P,2), ``T`` (P,), and totals ``E``, ``G`` (N_v,3), the
    hit records (``hit_pair``, ``hit_t``, ``hit_a``, ``hit_b``, ``hit_g``, ``hit_H``) and the
    BSR Hessian ``row_ptr``, ``col_idx``, ``vals`` (nnzb,3,3).  With ``vertex_adjacent`` a pair
    sharing exactly one vertex is evaluated instead of flagged adjacent.
    """
    x, tris, pl = _f64(x), _i32(tris), _i32(pair_list).reshape(-1, 2)
    L = lib()
    h = L.ttie_oracle_eval(_d(x), len(x), _i(tris), len(tris), _i(pl), len(pl), interval, psd,
                           1 if hessian else 0, threads, 1 if vertex_adjacent else 0)
    try:
        nh, nb = ctypes.c_int64(0), ctypes.c_int64(0)
        err = L.ttie_oracle_eval_sizes(h, ctypes.byref(nh), ctypes.byref(nb))
        if err:
            raise ValueError("oracle: pair index out of range or i == j")
        nh, nb = nh.value, nb.value
        np_ = len(pl)
        out = dict(
            flags=np.zeros(np_, np.uint8), t=np.zeros((np_, 2)), T=np.zeros(np_), E=np.zeros(1),
            G=np.zeros((len(x), 3)), hit_pair=np.zeros(nh, np.int64), hit_t=np.zeros((nh, 2)),
            hit_a=np.zeros((nh, 18)), hit_b=np.zeros((nh, 18)), hit_g=np.zeros((nh, 18)),
            hit_H=np.zeros((nh, 18, 18)) if hessian else None,
            row_ptr=np.zeros(len(x) + 1, np.int32) if hessian else None,
            col_idx=np.zeros(nb, np.int32) if hessian else None,
            vals=np.zeros((nb, 3, 3)) if hessian else None,
        )
        nul_d, nul_i = ctypes.cast(None, _dp), ctypes.cast(None, _ip)
        L.ttie_oracle_eval_fetch(
            h, out["flags"].ctypes.data_as(_bp), _d(out["t"]), _d(out["T"]), _d(out["E"]), _d(out["G"]),
            out["hit_pair"].ctypes.data_as(_lp), _d(out["hit_t"]), _d(out["hit_a"]), _d(out["hit_b"]),
            _d(out["hit_g"]), _d(out["hit_H"]) if hessian else nul_d,
            _i(out["row_ptr"]) if hessian else nul_i, _i(out["col_idx"]) if hessian else nul_i,
            _d(out["vals"]) if hessian else nul_d)
    finally:
        L.ttie_oracle_eval_free(h)
    out["E"] = float(out["E"][0])
    return out


def hvp(x, tris, pair_list, v, interval=INTERVAL_EQ1, exact=True, psd=PSD_PER_PART, threads=0,
        vertex_adjacent=False):
    """H v summed over the candidate list: the exact Hessian (nested duals) when ``exact``,
    else the ``psd`` Hessian of Eq. 4."""
    x, tris, pl, v = _f64(x), _i32(tris), _i32(pair_list).reshape(-1, 2), _f64(v).reshape(-1, 3)
    out = np.zeros_like(x)
    lib().ttie_oracle_hvp(_d(x), len(x), _i(tris), len(tris), _i(pl), len(pl), _d(v), interval,
                          0 if exact else 1, psd, _d(out), threads, 1 if vertex_adjacent else 0)
    return out


def bsr_to_dense(row_ptr, col_idx, vals, n_verts):
    """Dense (3N,3N) matrix from a 3x3-block CSR triple (for small test problems)."""
    H = np.zeros((3 * n_verts, 3 * n_verts))
    for r in range(n_verts):
        for k in range(row_ptr[r], row_ptr[r + 1]):
            c = col_idx[k]
            H[3 * r:3 * r + 3, 3 * c:3 * c + 3] += np.asarray(vals[k]).reshape(3, 3)
    return H
