"""Pins of the oracle's coplanar-overlap status against exact rational geometry.

Two triangles in one plane have no intersection segment, so their energy is 0; the oracle
reports the pair with status 4 when their interiors overlap.  Here the overlap is decided by a
different computation: one triangle is clipped by the other's three closed half-planes
(Sutherland-Hodgman, in Python fractions on the plane's integer (u, v) coordinates), and the
interiors overlap exactly when the clipped polygon has positive area.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2606_06511_amd import workloads

PLANES = np.asarray(workloads._SOUP_PLANES, np.float64)


def _orient(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def clip_area(P, Q):
    """Area of the intersection of the closed triangles P and Q, given by (u, v) corners."""
    sq = _orient(*Q)
    if sq == 0 or _orient(*P) == 0:
        return Fraction(0)
    poly = [(Fraction(p[0]), Fraction(p[1])) for p in P]
    for e in range(3):
        a, b = Q[e], Q[(e + 1) % 3]
        side = [sq * _orient(a, b, p) for p in poly]
        out = []
        for i, cur in enumerate(poly):
            k = (i + 1) % len(poly)
            nxt = poly[k]
            if side[i] >= 0:
                out.append(cur)
            if (side[i] > 0 and side[k] < 0) or (side[i] < 0 and side[k] > 0):
                t = side[i] / (side[i] - side[k])
                out.append((cur[0] + t * (nxt[0] - cur[0]), cur[1] + t * (nxt[1] - cur[1])))
        poly = out
        if not poly:
            return Fraction(0)
    n = len(poly)
    return abs(sum(poly[i][0] * poly[(i + 1) % n][1] - poly[(i + 1) % n][0] * poly[i][1] for i in range(n))) / 2


def embed(uv, plane):
    o, e1, e2 = PLANES[plane]
    uv = np.asarray(uv, np.float64)
    return o + uv[..., :1] * e1 + uv[..., 1:] * e2


def _eval_pairs(tri_uv, planes):
    """One triangle per row of tri_uv (n, 3, 2) on its plane; pairs (2k, 2k+1)."""
    x = np.concatenate([embed(t, p) for t, p in zip(tri_uv, planes)])
    tris = np.arange(len(x), dtype=np.int32).reshape(-1, 3)
    pairs = np.arange(len(tris), dtype=np.int32).reshape(-1, 2)
    return oracle.evaluate(x, tris, pairs)


def test_clip_area_self_check():
    # the rational clipper itself, on cases with known areas
    big = [(0, 0), (4, 0), (0, 4)]
    assert clip_area(big, big) == 8
    assert clip_area([(1, 1), (2, 1), (1, 2)], big) == Fraction(1, 2)   # contained
    assert clip_area(big, [(0, 0), (0, 4), (-4, 0)]) == 0              # shared edge line
    assert clip_area(big, [(2, 2), (4, 4), (2, 4)]) == 0               # touches at a vertex
    assert clip_area(big, [(2, 0), (6, 0), (2, 4)]) == 2                # half-overlap
    assert clip_area([(0, 0), (2, 2), (4, 4)], big) == 0               # no area


@pytest.mark.parametrize("plane", range(len(PLANES)))
def test_random_coplanar_pairs_match_clipping(plane):
    rng = np.random.default_rng(10 + plane)
    n = 600
    uv = rng.integers(0, 5, (2 * n, 3, 2))
    ref = _eval_pairs(uv, [plane] * (2 * n))
    got = ref["flags"]
    want = np.array([clip_area(uv[2 * k].tolist(), uv[2 * k + 1].tolist()) > 0 for k in range(n)])
    np.testing.assert_array_equal(got == oracle.ST_COPLANAR, want)
    assert np.all((got == oracle.ST_COPLANAR) | (got == oracle.ST_NONE))
    assert 0.2 * n < want.sum() < 0.8 * n  # both outcomes well represented
    assert ref["E"] == 0.0 and np.all(ref["T"] == 0.0)


def test_pairs_on_different_planes_never_coplanar():
    rng = np.random.default_rng(3)
    n = 400
    uv = rng.integers(0, 5, (2 * n, 3, 2))
    planes = np.stack([rng.integers(0, 2, n), rng.integers(2, 4, n)], 1).reshape(-1)
    ref = _eval_pairs(uv, planes)
    assert not np.any(ref["flags"] == oracle.ST_COPLANAR)


CASES = [  # (A, B, overlap)
    ([(0, 0), (4, 0), (0, 4)], [(0, 0), (4, 0), (0, 4)], True),    # the same triangle
    ([(0, 0), (4, 0), (0, 4)], [(0, 4), (4, 0), (0, 0)], True),    # same, other orientation
    ([(0, 0), (4, 0), (0, 4)], [(1, 1), (2, 1), (1, 2)], True),    # contained
    ([(1, 1), (2, 1), (1, 2)], [(0, 0), (4, 0), (0, 4)], True),    # containing
    ([(0, 0), (4, 0), (0, 4)], [(2, 0), (6, 0), (2, 4)], True),    # partial overlap
    ([(0, 0), (4, 0), (0, 4)], [(0, 0), (0, 4), (-4, 0)], False),  # touching along an edge
    ([(0, 0), (4, 0), (0, 4)], [(2, 2), (4, 4), (2, 4)], False),   # touching at a vertex
    ([(0, 0), (4, 0), (0, 4)], [(1, 0), (3, 0), (2, -2)], False),  # edge on edge, outside
    ([(0, 0), (4, 0), (0, 4)], [(5, 5), (6, 5), (5, 6)], False),   # apart
    ([(0, 0), (4, 0), (0, 4)], [(0, 1), (4, 1), (8, 1)], False),   # no area, across A
    ([(0, 0), (0, 0), (0, 0)], [(0, 0), (4, 0), (0, 4)], False),   # a point
    ([(0, 0), (4, 0), (0, 4)], [(1, 1), (5, -1), (5, 3)], True),   # vertex inside, edges crossing
]


@pytest.mark.parametrize("plane", range(len(PLANES)))
def test_special_cases(plane):
    uv = np.array([c for A, B, _ in CASES for c in (A, B)])
    ref = _eval_pairs(uv, [plane] * len(uv))
    want = np.array([ov for _, _, ov in CASES])
    np.testing.assert_array_equal(ref["flags"] == oracle.ST_COPLANAR, want)
    for A, B, ov in CASES:
        assert (clip_area(A, B) > 0) == ov


def test_invariant_under_order_translation_and_scale():
    rng = np.random.default_rng(5)
    n = 300
    uv = rng.integers(0, 5, (2 * n, 3, 2))
    x = np.concatenate([embed(t, 2) for t in uv])
    tris = np.arange(len(x), dtype=np.int32).reshape(-1, 3)
    pairs = np.arange(len(tris), dtype=np.int32).reshape(-1, 2)
    f0 = oracle.evaluate(x, tris, pairs)["flags"]
    assert np.any(f0 == oracle.ST_COPLANAR)
    # swapped roles, reversed vertex order of the first triangle
    np.testing.assert_array_equal(oracle.evaluate(x, tris, pairs[:, ::-1].copy())["flags"], f0)
    np.testing.assert_array_equal(oracle.evaluate(x, tris[:, ::-1].copy(), pairs)["flags"], f0)
    # exact similarity maps: a power-of-two scale and an integer shift
    np.testing.assert_array_equal(oracle.evaluate(x * 0.125 + np.array([3.0, -7.0, 11.0]), tris, pairs)["flags"], f0)
    # lifting one triangle of each pair off the plane along the normal removes every status 4
    o, e1, e2 = PLANES[2]
    lift = x.copy()
    lift[tris[pairs[:, 1]].reshape(-1)] += np.cross(e1, e2)
    assert not np.any(oracle.evaluate(lift, tris, pairs)["flags"] == oracle.ST_COPLANAR)


def test_soup_statuses_match_clipping():
    """The generator's pairs: coplanar statuses exactly where same-plane clipping has area."""
    x, tris = workloads.coplanar_soup(1, n_tris=600, grid=8, span=4)
    pairs = oracle.pairs(x, tris)
    ref = oracle.evaluate(x, tris, pairs)
    # recover each triangle's plane and (u, v) corners from the generator's own recipe
    rng = np.random.default_rng(1)
    pl = rng.integers(0, 4, 600)
    uv = rng.integers(0, 5, (600, 1, 2)) + rng.integers(0, 5, (600, 3, 2))
    np.testing.assert_array_equal(np.concatenate([embed(uv[t], pl[t]) for t in range(600)]), x)
    same = pl[pairs[:, 0]] == pl[pairs[:, 1]]
    want = np.array([s and clip_area(uv[i].tolist(), uv[j].tolist()) > 0 for (i, j), s in zip(pairs, same)])
    np.testing.assert_array_equal(ref["flags"] == oracle.ST_COPLANAR, want)
    assert want.sum() > 100 and np.sum(ref["flags"] == oracle.ST_HIT) > 100
