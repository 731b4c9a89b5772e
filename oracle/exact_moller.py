"""Exact-rational Moeller test -- TEST INFRASTRUCTURE ONLY.

A second, independent statement of Sec. 1 (Moeller's reduction, Eq. 1 and the
open-interval criterion) in exact arithmetic, used to pin the oracle's intersection flags and
interval values.  Every FP64 input is converted to a ``fractions.Fraction`` exactly, so every
sign and comparison below is exact.

It deliberately builds the segments differently from the appendix's case table: the part of
a triangle lying on the other triangle's plane is taken as the set {vertices on the plane}
together with {crossing points of edges whose endpoints lie strictly on opposite sides}.
The line parameter is t(P) = D.P with the unnormalised D = n_a x n_b, i.e. the paper's t
times |D| plus a common offset, which changes no comparison.
"""

from __future__ import annotations

from fractions import Fraction


def _vec(p):
    return tuple(c if isinstance(c, Fraction) else Fraction(float(c)) for c in p)


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _sign(x):
    return (x > 0) - (x < 0)


def orient_sign(a, b, c, p) -> int:
    a, b, c, p = (_vec(v) for v in (a, b, c, p))
    return _sign(_dot(_cross(_sub(b, a), _sub(c, a)), _sub(p, a)))


def _cut(tri, n, o):
    """Points of triangle ``tri`` on the plane through ``o`` with normal ``n``: on-plane
    vertices and crossing points of edges with strictly opposite sides.  Returns (points,
    straddles)."""
    d = [_dot(n, _sub(p, o)) for p in tri]
    s = [_sign(x) for x in d]
    straddles = (1 in s) and (-1 in s)
    pts = [tri[k] for k in range(3) if s[k] == 0]
    for i, j in ((0, 1), (1, 2), (2, 0)):
        if s[i] * s[j] < 0:
            lam = d[i] / (d[i] - d[j])
            pts.append(tuple(tri[i][c] + lam * (tri[j][c] - tri[i][c]) for c in range(3)))
    return pts, straddles


def pair(u, v):
    """Exact Moeller evaluation of T_a = u (3x3) against T_b = v (3x3).

    Returns dict(straddle, flag, tc0, tc1, DD): ``tc0``/``tc1`` are Eq. 1's interval ends
    multiplied by |D| (exact Fractions; None when a triangle does not straddle the other's
    plane) and ``DD`` = |D|^2, so the paper's values are tc/sqrt(DD).
    """
    U = [_vec(p) for p in u]
    V = [_vec(p) for p in v]
    na = _cross(_sub(U[1], U[0]), _sub(U[2], U[0]))
    nb = _cross(_sub(V[1], V[0]), _sub(V[2], V[0]))
    pa, sa = _cut(U, nb, V[0])
    pb, sb = _cut(V, na, U[0])
    out = dict(straddle=bool(sa and sb), flag=False, tc0=None, tc1=None, DD=None)
    if not (sa and sb):
        return out
    D = _cross(na, nb)
    ta = [_dot(D, p) for p in pa]
    tb = [_dot(D, p) for p in pb]
    tc0 = min(ta) - max(tb)
    tc1 = max(ta) - min(tb)
    out.update(flag=bool(tc0 < 0 < tc1), tc0=tc0, tc1=tc1, DD=_dot(D, D))
    return out


def shares_vertex(ti, tj) -> bool:
    return len(set(int(a) for a in ti) & set(int(b) for b in tj)) > 0
