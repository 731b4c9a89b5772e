"""Element-wise parity checks of the GPU path against the CPU oracle, shared by the GPU tests.

Every check compares per element (per pair, per hit, per gradient row, per Hessian block), never
only a global norm, so one wrong pair cannot hide behind many right ones.

The bars follow the arithmetic.  tol is 1e-10 on the float64 path and 1e-4 on the mixed path
(float32 per-hit algebra); the interval ends t_c and T are float64 on both paths, so their
tolerance tol_t is 1e-10 on both.  Two independent float64 evaluations of an interval end agree
to a multiple of the unit roundoff times the size of the quantities it is formed from, not
times its own size: an end close to zero is the difference of two nearly equal positions on
the line.  So each bar is a tolerance times an error scale, and a derived result's scale is
the first-order propagation of its inputs' bars through its formula (Eq. 1-4):

* flags, candidate lists, hit lists and BSR patterns: identical;
* interval ends (Eq. 1): |dt_i| <= tol_t m, with m = max(|t_c^0|, |t_c^1|) of the oracle;
* per pair, T = s^2 with s = t_c^0 t_c^1 (Eq. 2): |ds| <= tol_t m (|t_c^0| + |t_c^1|) (ends taken
  plus their bars), so |dT| <= tol_t T + 2 |s| ds + ds^2; T is exactly 0 off the hits (flags agree);
* per hit, the interval Jacobian [a b] (a = dt_c^0, b = dt_c^1): every entry within
  tol J + 2 c dJ, with J the largest entry of the pair's 18 x 2 Jacobian and dJ the pair's own
  sensitivity: the largest change of the oracle's [a b] when the pair's coordinates, taken
  relative to its first vertex, are rounded to float32 or moved by a relative 2^-24
  (``hit_sensitivity``); c = 1 on the mixed path and 2^-29 (the ratio of the unit roundoffs) on
  the float64 one.  Near-parallel planes or an edge almost in the other plane amplify rounding
  of the inputs: such a pair's Jacobian cannot be computed in float32 to 1e-4 by any method;
* per hit, g = 2 s (t_c^1 a + t_c^0 b) (Eq. 3): the propagation of the bars above,
  2 [ds (|t1| A + |t0| B) + |s| (dt (A + B) + dab (|t0| + |t1|))] + (tol + r) 2 |s| (|t1| A + |t0| B),
  with A, B the largest entries of a, b, dab the Jacobian's bar below and r = dab / J (every
  magnitude taken plus its own bar, which covers the second-order terms);
* per hit, the 18 x 18 block J^T M J: within 4 r of its largest entry, r being the Jacobian's
  relative bar above (the block is quadratic in [a b] and M is homogeneous in it);
* per gradient row and per BSR block row: a row is a sum over the hits touching it, so its
  bar is the sum of those hits' bars (the hit's g bar; tol times the largest entry of the hit's
  Hessian);
* the energy: the sum of the per-hit T bars.
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


def _check(err, bar, what, where):
    """err <= bar everywhere (both arrays of one shape); ``where(k)`` names the flat index k."""
    err = np.asarray(err, np.float64)
    bar = np.asarray(bar, np.float64)
    bad = err > bar
    if bad.any():
        k = int(np.argmax(np.where(bad, err / np.maximum(bar, 1e-300), 0).ravel()))
        _fail(what, err.ravel()[k], bar.ravel()[k], where(k))


U32 = 2.0 ** -24
FP64_PER_FP32 = 2.0 ** -29  # float64 unit roundoff over float32's


def hit_sensitivity(x, tris, pairs, ref, copies=6, seed=0, **kw):
    """Per hit (the oracle's order): the largest entry-wise change of the oracle's [a b] when the
    pair's coordinates relative to its first vertex are rounded to float32 (after scaling by a
    power of two to order 1), or multiplied by
    1 + 2^-24 r with r uniform in [-1, 1] (``copies`` draws).  Every copy of every hit goes into
    one oracle evaluation of a soup of disjoint pairs (a vertex the two triangles share stays
    one vertex).  A copy whose flag changes carries no derivative and is left out; a hit with no
    copy left gets its Jacobian's largest entry."""
    hp = np.asarray(pairs)[ref["hit_pair"]]
    n = len(hp)
    if n == 0:
        return np.zeros(0)
    tris = np.asarray(tris)
    ta, tb = tris[hp[:, 0]], tris[hp[:, 1]]
    X = np.concatenate([x[ta], x[tb]], axis=1)  # (n, 6, 3)
    X0 = X - X[:, :1, :]
    # float32 rounding of the coordinates brought to order 1 by a power of two (as the mixed
    # path scales them), so that it neither overflows nor underflows
    e = np.ldexp(1.0, -np.frexp(np.abs(X0).max(axis=(1, 2)))[1])[:, None, None]
    rng = np.random.default_rng(seed)
    reps = [X0, (X0 * e).astype(np.float32).astype(np.float64) / e]
    reps += [X0 * (1.0 + U32 * rng.uniform(-1.0, 1.0, X0.shape)) for _ in range(copies)]
    nc = len(reps)
    xs = np.ascontiguousarray(np.stack(reps).reshape(-1, 3))
    # local vertex index of each slot of T_b: its slot in T_a when the vertex is shared
    loc_b = np.tile(np.arange(3, 6), (n, 1))
    for k in range(3):
        for m in range(3):
            loc_b[:, k] = np.where(tb[:, k] == ta[:, m], m, loc_b[:, k])
    base = 6 * np.arange(nc * n).reshape(nc, n, 1)
    soup_a = base + np.arange(3)
    soup_b = base + loc_b[None]
    ts = np.stack([soup_a, soup_b], axis=2).reshape(-1, 3).astype(np.int32)
    pl = np.arange(2 * nc * n, dtype=np.int32).reshape(-1, 2)
    r = oracle.evaluate(xs, ts, pl, hessian=False, **kw)
    ab = np.full((nc * n, 36), np.nan)
    ab[r["hit_pair"]] = np.concatenate([r["hit_a"], r["hit_b"]], axis=1)
    ab = ab.reshape(nc, n, 36)
    J = np.maximum(np.abs(ref["hit_a"]).max(axis=1), np.abs(ref["hit_b"]).max(axis=1))
    dev = np.abs(ab[1:] - ab[0][None]).max(axis=2)  # (nc - 1, n), nan where a copy is no hit
    ok = ~np.isnan(dev)
    out = np.where(ok, dev, 0.0).max(axis=0)
    return np.where(ok.any(axis=0) & ~np.isnan(ab[0, :, 0]), out, J)


def reference(x, tris, pairs, **kw):
    """``oracle.evaluate`` plus each hit's float32 sensitivity (``hit_dJ``), which the bars of
    the per-hit Jacobian and of everything derived from it use."""
    ref = oracle.evaluate(x, tris, pairs, **kw)
    skw = {k: v for k, v in kw.items() if k in ("interval", "vertex_adjacent")}
    ref["hit_dJ"] = hit_sensitivity(x, tris, pairs, ref, **skw)
    return ref


def _dJ(ref):
    if "hit_dJ" not in ref:
        raise KeyError("the oracle result needs hit_dJ: build it with parity_checks.reference")
    return ref["hit_dJ"]


def hit_bars(t, a, b, dJ, precision):
    """Absolute bars (arrays over hits) of T, of the Jacobian entries and of g, and the
    Jacobian's relative bar, from the oracle's t_c, a, b and the hits' sensitivities dJ."""
    tol = tol_for(precision)
    tt = FP64_TOL
    c = 1.0 if precision else FP64_PER_FP32
    m = np.abs(t).max(axis=1) if len(t) else np.zeros(0)
    t0 = np.abs(t[:, 0]) + tt * m
    t1 = np.abs(t[:, 1]) + tt * m
    s = t0 * t1
    A = np.abs(a).max(axis=1) if len(a) else np.zeros(0)
    B = np.abs(b).max(axis=1) if len(b) else np.zeros(0)
    J = np.maximum(A, B)
    bar_ab = tol * J + 2 * c * np.asarray(dJ)
    rel = bar_ab / np.maximum(J, 1e-300)
    A, B = A + bar_ab, B + bar_ab
    ds = tt * m * (t0 + t1)
    bar_T = tt * s * s + 2 * s * ds + ds * ds
    mag = t1 * A + t0 * B
    bar_g = 2 * (ds * mag + s * (tt * m * (A + B) + bar_ab * (t0 + t1))) + (tol + rel) * 2 * s * mag
    return bar_T, bar_ab, bar_g, rel


def check_pair_T(pair_T, ref, pairs, what="pair T"):
    """Per pair against the oracle's T; off the hits both must be exactly 0."""
    pair_T = np.asarray(pair_T, np.float64)
    want = np.asarray(ref["T"], np.float64)
    assert pair_T.shape == want.shape
    bar = np.zeros(len(want))
    if len(ref["hit_pair"]):
        bar_T = hit_bars(ref["hit_t"], ref["hit_a"], ref["hit_b"], np.zeros(len(ref["hit_pair"])), 0)[0]
        bar[ref["hit_pair"]] = bar_T
    _check(np.abs(pair_T - want), bar, what, lambda k: f"pair {k} {np.asarray(pairs)[k]} (T* = {want[k]:.6e})")


def ref_hits_sorted(ref, pairs):
    """The oracle's hit records reordered by pair key (i, j), as the GPU returns them."""
    ij = np.asarray(pairs)[ref["hit_pair"]].astype(np.int64)
    order = np.lexsort((ij[:, 1], ij[:, 0]))
    out = {"ij": ij[order], "t": ref["hit_t"][order], "a": ref["hit_a"][order], "b": ref["hit_b"][order],
           "g": ref["hit_g"][order], "dJ": _dJ(ref)[order]}
    if ref.get("hit_H") is not None:
        out["H"] = ref["hit_H"][order]
    return out


def per_hit_hessian(a, b, M):
    """J^T M J per hit from the GPU's own factors (a, b: (H, 18); M: (H, 3) = M00, M01, M11)."""
    aa = a[:, :, None] * a[:, None, :]
    ab = a[:, :, None] * b[:, None, :]
    bb = b[:, :, None] * b[:, None, :]
    return M[:, 0, None, None] * aa + M[:, 1, None, None] * (ab + ab.transpose(0, 2, 1)) + M[:, 2, None, None] * bb


def check_hits(h, ref, pairs, precision, hessian=True, what=""):
    """h: ``Context.hits()`` (sorted by (i, j)); ref: ``oracle.evaluate`` on ``pairs``."""
    r = ref_hits_sorted(ref, pairs)
    np.testing.assert_array_equal(np.asarray(h["ij"], np.int64), r["ij"], err_msg=f"{what} hit list")
    n = len(r["ij"])
    if n == 0:
        return
    m = np.abs(r["t"]).max(axis=1)
    _check(np.abs(np.asarray(h["t"]) - r["t"]).max(axis=1), FP64_TOL * m, f"{what} t_c",
           lambda k: f"hit {k} {r['ij'][k]} (t* = {r['t'][k]})")
    bar_T, bar_ab, bar_g, rel = hit_bars(r["t"], r["a"], r["b"], r["dJ"], precision)
    _check(np.abs(np.asarray(h["T"]) - np.prod(r["t"], axis=1) ** 2), bar_T, f"{what} hit T",
           lambda k: f"hit {k} {r['ij'][k]} (t* = {r['t'][k]})")
    for name in ("a", "b"):
        err = np.abs(np.asarray(h[name], np.float64).reshape(n, 18) - r[name]).max(axis=1)
        _check(err, bar_ab, f"{what} {name}", lambda k: f"hit {k} {r['ij'][k]} (t* = {r['t'][k]})")
    err = np.abs(np.asarray(h["g"], np.float64).reshape(n, 18) - r["g"]).max(axis=1)
    _check(err, bar_g, f"{what} g", lambda k: f"hit {k} {r['ij'][k]} (t* = {r['t'][k]})")
    if hessian and "H" in r:
        Hg = per_hit_hessian(np.asarray(h["a"], np.float64).reshape(n, 18),
                             np.asarray(h["b"], np.float64).reshape(n, 18), np.asarray(h["M"], np.float64))
        err = np.abs(Hg - r["H"]).reshape(n, -1).max(axis=1)
        _check(err, 4 * rel * np.abs(r["H"]).reshape(n, -1).max(axis=1), f"{what} per-hit Hessian",
               lambda k: f"hit {k} {r['ij'][k]}")


def _hit_vertices(ref, pairs, tris):
    ij = np.asarray(pairs)[ref["hit_pair"]]
    return np.concatenate([np.asarray(tris)[ij[:, 0]], np.asarray(tris)[ij[:, 1]]], axis=1)  # (H, 6)


def _row_sums(vid, per_hit, n_verts):
    """Per vertex, the sum over the hit slots that hold it of the hit's scale."""
    S = np.zeros(n_verts)
    if len(vid):
        np.add.at(S, vid.reshape(-1), np.repeat(per_hit, 6))
    return S


def check_grad(G, ref, pairs, tris, precision, what="gradient"):
    G = np.asarray(G, np.float64)
    want = ref["G"]
    vid = _hit_vertices(ref, pairs, tris)
    bar_g = hit_bars(ref["hit_t"], ref["hit_a"], ref["hit_b"], _dJ(ref), precision)[2]
    bar = np.repeat(_row_sums(vid, bar_g, len(want))[:, None], 3, axis=1)
    _check(np.abs(G - want), bar, what, lambda k: f"vertex {k // 3} coordinate {k % 3}")


def bsr_row_bars(ref, pairs, tris, precision, n_verts):
    """Per vertex row: the sum, over the hit slots holding the vertex, of the hit's Hessian bar
    (4 r times the largest entry of its 18 x 18 Hessian)."""
    vid = _hit_vertices(ref, pairs, tris)
    if len(vid) == 0:
        return np.zeros(n_verts)
    rel = hit_bars(ref["hit_t"], ref["hit_a"], ref["hit_b"], _dJ(ref), precision)[3]
    hmax = np.abs(ref["hit_H"]).reshape(len(vid), -1).max(axis=1)
    return _row_sums(vid, 4 * rel * hmax, n_verts)


def check_bsr(row_ptr, col_idx, vals, ref, pairs, tris, precision, what="BSR"):
    np.testing.assert_array_equal(np.asarray(row_ptr), ref["row_ptr"], err_msg=f"{what} row_ptr")
    np.testing.assert_array_equal(np.asarray(col_idx), ref["col_idx"], err_msg=f"{what} col_idx")
    nb = len(ref["col_idx"])
    if nb == 0:
        return
    v = np.asarray(vals, np.float64).reshape(nb, 9)
    want = ref["vals"].reshape(nb, 9)
    nv = len(ref["row_ptr"]) - 1
    row = np.repeat(np.arange(nv), np.diff(ref["row_ptr"]))
    bar = bsr_row_bars(ref, pairs, tris, precision, nv)[row]
    _check(np.abs(v - want).max(axis=1), bar, what,
           lambda k: f"block {k} (row {row[k]}, column {ref['col_idx'][k]})")


def check_energy(E, ref, what="energy"):
    """E against the oracle's; ``ref`` is the oracle's result (bar: the sum of the hits' T bars)
    or a bare float64 (bar: tol_t |E*|)."""
    if isinstance(ref, dict):
        want = ref["E"]
        bar = FP64_TOL * abs(want)
        if len(ref["hit_pair"]):
            nh = len(ref["hit_pair"])
            bar = max(bar, hit_bars(ref["hit_t"], ref["hit_a"], ref["hit_b"], np.zeros(nh), 0)[0].sum())
    else:
        want = float(ref)
        bar = FP64_TOL * abs(want)
    if abs(E - want) > bar:
        _fail(what, abs(E - want), bar, "the total")


def check_vector(got, want, scale, precision, what):
    """Per-entry check of an N x 3 result against the oracle with an explicit per-entry scale."""
    tol = tol_for(precision)
    got = np.asarray(got, np.float64)
    _check(np.abs(got - want), tol * scale, what, lambda k: f"vertex {k // 3} coordinate {k % 3}")


def check_eval_outputs(out, ref, pairs, tris, precision, flags=True, hessian=True, what=""):
    """Every output of ``Context.evaluate`` against ``oracle.evaluate`` on the same list."""
    if flags and "flags" in out:
        np.testing.assert_array_equal(out["flags"].cpu().numpy()[: len(pairs)], ref["flags"],
                                      err_msg=f"{what} flags")
    if "pair_T" in out:
        check_pair_T(out["pair_T"].cpu().numpy()[: len(pairs)], ref, pairs, f"{what} pair T")
    assert int(out["n_hits"].item()) == len(ref["hit_pair"]), what
    check_energy(out["energy"].item(), ref, f"{what} energy")
    check_grad(out["grad"].cpu().numpy(), ref, pairs, tris, precision, f"{what} gradient")
    if hessian and "row_ptr" in out:
        nb = int(out["n_blocks"].item())
        check_bsr(out["row_ptr"].cpu().numpy(), out["col_idx"][:nb].cpu().numpy(), out["vals"][:nb].cpu().numpy(),
                  ref, pairs, tris, precision, f"{what} BSR")


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
