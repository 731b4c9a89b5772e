"""Element-wise parity checks of the GPU path against the CPU oracle, shared by the GPU tests.

Every check compares per element (per pair, per hit, per gradient row, per Hessian block), never
only a global norm, so one wrong pair cannot hide behind many right ones.  The bars:

* flags, candidate lists, hit lists and BSR patterns: identical;
* per pair: |T - T*| <= tol_T max(|T*|, 1e-10 max T*)  (T is float64 on both paths);
* per hit: both interval ends within tol_t of the larger of |t_c^0*|, |t_c^1*|; the 18-vectors
  a = dt_c^0, b = dt_c^1 and g = dT each within tol of their own largest entry; the pair's
  18 x 18 Hessian J^T M J within tol of its own largest entry;
* per gradient row: |G_v - G*_v| <= tol S_v with S_v the sum, over the hits touching v, of the
  largest entry of each hit's gradient (the scale a row sum's rounding error is relative to);
* per BSR block: |B - B*| <= tol times the largest entry of its block row;
* the energy: |E - E*| <= tol_T |E*|.

tol is 1e-10 on the float64 path and 1e-4 on the mixed path (float32 per-hit algebra); t_c and
T are float64 on both paths, so tol_t = tol_T = 1e-10 on both.
"""

from __future__ import annotations

import numpy as np

import oracle

FP64_TOL = 1e-10
MIXED_TOL = 1e-4


def tol_for(precision):
    return FP64_TOL if precision == 0 else MIXED_TOL


def _fail(what, worst, bar, where):
    raise AssertionError(f"{what}: worst error {worst:.3e} exceeds {bar:.3e} at {where}")


def check_pair_T(pair_T, ref_T, tol=FP64_TOL, what="pair T"):
    pair_T = np.asarray(pair_T, np.float64)
    ref_T = np.asarray(ref_T, np.float64)
    assert pair_T.shape == ref_T.shape
    if ref_T.size == 0:
        return
    floor = 1e-10 * np.abs(ref_T).max()
    bar = tol * np.maximum(np.abs(ref_T), floor)
    err = np.abs(pair_T - ref_T)
    bad = err > bar
    if bad.any():
        k = int(np.argmax(np.where(bad, err / np.maximum(bar, 1e-300), 0)))
        _fail(what, err[k], bar[k], f"pair {k} (T* = {ref_T[k]:.6e})")


def ref_hits_sorted(ref, pairs):
    """The oracle's hit records reordered by pair key (i, j), as the GPU returns them."""
    ij = np.asarray(pairs)[ref["hit_pair"]].astype(np.int64)
    order = np.lexsort((ij[:, 1], ij[:, 0]))
    out = {"ij": ij[order], "t": ref["hit_t"][order], "a": ref["hit_a"][order], "b": ref["hit_b"][order],
           "g": ref["hit_g"][order]}
    if ref.get("hit_H") is not None:
        out["H"] = ref["hit_H"][order]
    return out


def per_hit_hessian(a, b, M):
    """J^T M J per hit from the GPU's own factors (a, b: (H, 18); M: (H, 3) = M00, M01, M11)."""
    aa = a[:, :, None] * a[:, None, :]
    ab = a[:, :, None] * b[:, None, :]
    bb = b[:, :, None] * b[:, None, :]
    return M[:, 0, None, None] * aa + M[:, 1, None, None] * (ab + ab.transpose(0, 2, 1)) + M[:, 2, None, None] * bb


def _vec_check(got, want, tol, what):
    got = np.asarray(got, np.float64).reshape(len(want), -1)
    want = np.asarray(want, np.float64).reshape(len(want), -1)
    scale = np.abs(want).max(axis=1)
    err = np.abs(got - want).max(axis=1)
    bar = tol * np.maximum(scale, 1e-300)
    bad = err > bar
    if bad.any():
        k = int(np.argmax(np.where(bad, err / bar, 0)))
        _fail(what, err[k], bar[k], f"hit {k}")


def check_hits(h, ref, pairs, precision, hessian=True, what=""):
    """h: ``Context.hits()`` (sorted by (i, j)); ref: ``oracle.evaluate`` on ``pairs``."""
    tol = tol_for(precision)
    r = ref_hits_sorted(ref, pairs)
    np.testing.assert_array_equal(np.asarray(h["ij"], np.int64), r["ij"], err_msg=f"{what} hit list")
    if len(r["ij"]) == 0:
        return
    tmax = np.abs(r["t"]).max(axis=1)
    err = np.abs(np.asarray(h["t"]) - r["t"]).max(axis=1)
    bad = err > FP64_TOL * tmax
    if bad.any():
        k = int(np.argmax(np.where(bad, err / tmax, 0)))
        _fail(f"{what} t_c", err[k], FP64_TOL * tmax[k], f"hit {k} {r['ij'][k]}")
    check_pair_T(h["T"], np.prod(r["t"], axis=1) ** 2, FP64_TOL, f"{what} hit T")
    _vec_check(h["a"], r["a"], tol, f"{what} a")
    _vec_check(h["b"], r["b"], tol, f"{what} b")
    _vec_check(h["g"], r["g"], tol, f"{what} g")
    if hessian and "H" in r:
        _vec_check(per_hit_hessian(np.asarray(h["a"]), np.asarray(h["b"]), np.asarray(h["M"])), r["H"], tol,
                   f"{what} per-hit Hessian")


def row_scales(ref, pairs, tris, n_verts):
    """S_v: the sum over the hits touching vertex v of the magnitude (largest entry) of their
    gradients -- the scale of the rounding error of row v's sum, since each hit's 18 entries are
    computed together and carry errors relative to the largest of them."""
    ij = np.asarray(pairs)[ref["hit_pair"]]
    vid = np.concatenate([np.asarray(tris)[ij[:, 0]], np.asarray(tris)[ij[:, 1]]], axis=1)  # (H, 6)
    mag = np.abs(ref["hit_g"]).max(axis=1) if len(ij) else np.zeros(0)
    S = np.zeros(n_verts)
    np.add.at(S, vid.reshape(-1), np.repeat(mag, 6))
    return np.repeat(S[:, None], 3, axis=1)


def check_grad(G, ref, pairs, tris, precision, what="gradient"):
    tol = tol_for(precision)
    G = np.asarray(G, np.float64)
    want = ref["G"]
    S = row_scales(ref, pairs, tris, len(want))
    err = np.abs(G - want)
    bar = tol * S
    bad = err > bar
    if bad.any():
        v, c = np.unravel_index(int(np.argmax(np.where(bad, err / np.maximum(bar, 1e-300), 0))), err.shape)
        _fail(what, err[v, c], bar[v, c], f"vertex {v} coordinate {c}")


def check_bsr(row_ptr, col_idx, vals, ref, precision, what="BSR"):
    tol = tol_for(precision)
    np.testing.assert_array_equal(np.asarray(row_ptr), ref["row_ptr"], err_msg=f"{what} row_ptr")
    np.testing.assert_array_equal(np.asarray(col_idx), ref["col_idx"], err_msg=f"{what} col_idx")
    nb = len(ref["col_idx"])
    if nb == 0:
        return
    v = np.asarray(vals, np.float64).reshape(nb, 9)
    want = ref["vals"].reshape(nb, 9)
    nv = len(ref["row_ptr"]) - 1
    row = np.repeat(np.arange(nv), np.diff(ref["row_ptr"]))
    rmax = np.zeros(nv)
    np.maximum.at(rmax, row, np.abs(want).max(axis=1))
    err = np.abs(v - want).max(axis=1)
    bar = tol * rmax[row]
    bad = err > bar
    if bad.any():
        k = int(np.argmax(np.where(bad, err / np.maximum(bar, 1e-300), 0)))
        _fail(what, err[k], bar[k], f"block {k} (row {row[k]}, column {ref['col_idx'][k]})")


def check_energy(E, ref_E, what="energy"):
    if abs(E - ref_E) > FP64_TOL * abs(ref_E):
        _fail(what, abs(E - ref_E), FP64_TOL * abs(ref_E), "the total")


def check_vector(got, want, scale, precision, what):
    """Per-entry check of an N x 3 result against the oracle with an explicit per-entry scale."""
    tol = tol_for(precision)
    got = np.asarray(got, np.float64)
    err = np.abs(got - want)
    bar = tol * scale
    bad = err > bar
    if bad.any():
        v, c = np.unravel_index(int(np.argmax(np.where(bad, err / np.maximum(bar, 1e-300), 0))), err.shape)
        _fail(what, err[v, c], bar[v, c], f"vertex {v} coordinate {c}")


def check_eval_outputs(out, ref, pairs, tris, precision, flags=True, hessian=True, what=""):
    """Every output of ``Context.evaluate`` against ``oracle.evaluate`` on the same list."""
    if flags and "flags" in out:
        np.testing.assert_array_equal(out["flags"].cpu().numpy()[: len(pairs)], ref["flags"],
                                      err_msg=f"{what} flags")
    if "pair_T" in out:
        check_pair_T(out["pair_T"].cpu().numpy()[: len(pairs)], ref["T"], FP64_TOL, f"{what} pair T")
    assert int(out["n_hits"].item()) == len(ref["hit_pair"]), what
    check_energy(out["energy"].item(), ref["E"], f"{what} energy")
    check_grad(out["grad"].cpu().numpy(), ref, pairs, tris, precision, f"{what} gradient")
    if hessian and "row_ptr" in out:
        nb = int(out["n_blocks"].item())
        check_bsr(out["row_ptr"].cpu().numpy(), out["col_idx"][:nb].cpu().numpy(), out["vals"][:nb].cpu().numpy(),
                  ref, precision, f"{what} BSR")


def hvp_row_scales(x, tris, pairs, v, exact, ref=None, vertex_adjacent=False):
    """Per vertex: the sum over the hits touching it of the largest entry of the hit's own
    Hessian-vector product (each computed by the oracle for that pair alone) -- the scale of the
    rounding error of a row of H v."""
    if ref is None or (not exact and ref.get("hit_H") is None):
        ref = oracle.evaluate(x, tris, pairs, hessian=not exact, vertex_adjacent=vertex_adjacent)
    S = np.zeros(len(x))
    for k, p in enumerate(ref["hit_pair"]):
        vid = np.concatenate([tris[pairs[p, 0]], tris[pairs[p, 1]]])
        if exact:
            hv = oracle.pair_hvp(x[vid], v[vid].reshape(18))
        else:
            hv = ref["hit_H"][k] @ v[vid].reshape(18)
        np.add.at(S, vid, np.abs(hv).max())
    return np.repeat(S[:, None], 3, axis=1)
