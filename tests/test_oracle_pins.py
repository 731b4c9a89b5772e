"""Pins for the CPU oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is a closed form worked
out by hand, an exact-rational evaluation (``oracle.exact_moller``), a finite difference, an
invariance of the definition, or a library routine.
"""

import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import exact_moller

# ---------------------------------------------------------------------------------------
# The worked example.  T_a = (0,0,0),(2,0,0),(0,2,0) lies in z = 0; T_b = (.5,.5,-1),
# (.5,.5,1),(1.5,.5,1) lies in y = .5.  n_a = (0,0,4), n_b = (0,2,0), D = n_a x n_b =
# (-8,0,0) so the line parameter is t = -x.  T_a meets y = .5 in x in [0, 1.5]; T_b meets
# z = 0 in x in [.5, 1] (edge v0v1 at x = .5, edge v0v2 at its midpoint x = 1).  Hence
# I_a = [-1.5, 0], I_b = [-1, -.5] and Eq. 1 gives t_c = [-1.5 + .5, 0 + 1] = [-1, 1],
# so T = (t0 t1)^2 = 1 (Eq. 2).
# ---------------------------------------------------------------------------------------
# the hand-derived values of this example, with their derivation, are the fixture
# tests/golden/worked_example.json
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")))
WORKED = np.array(GOLDEN["X"], float)
A_WORKED = np.array(GOLDEN["a"], float)
B_WORKED = np.array(GOLDEN["b"], float)


def test_worked_example_values():
    r = oracle.pair(WORKED)
    assert r["status"] == oracle.ST_HIT
    assert r["t0"] == GOLDEN["t0"] and r["t1"] == GOLDEN["t1"] and r["T"] == GOLDEN["T"]
    np.testing.assert_allclose(r["a"].reshape(6, 3), A_WORKED, atol=1e-15)
    np.testing.assert_allclose(r["b"].reshape(6, 3), B_WORKED, atol=1e-15)
    np.testing.assert_allclose(r["g"].reshape(6, 3), np.array(GOLDEN["g"]), atol=1e-15)
    # exact dyadic sums of the rows above
    a, b = r["a"], r["b"]
    assert a @ a == GOLDEN["a_dot_a"] and b @ b == GOLDEN["b_dot_b"] and a @ b == GOLDEN["a_dot_b"]
    h = oracle.pair(WORKED, interval=oracle.INTERVAL_APPENDIX_HALF)
    assert h["T"] == GOLDEN["T_appendix_half"]


def test_worked_example_eigenanalysis():
    # Sec. 1.1: part 1 eigenvalue 2 t1^2 |a|^2 = 6.5, part 2: 2 t0^2 |b|^2 = 2.6875; the
    # stated part-3 value 8 t0 t1 a.b = -2.5 is the trace of part 3, whose two eigenvalues
    # are 4 t0 t1 (a.b -+ |a||b|).
    raw = oracle.pair(WORKED, psd=oracle.PSD_RAW_EQ4)["H"]
    per = oracle.pair(WORKED, psd=oracle.PSD_PER_PART)["H"]
    assert np.trace(raw) == pytest.approx(
        GOLDEN["part1_eigenvalue"] + GOLDEN["part2_eigenvalue"] + GOLDEN["part3_stated_value"], abs=1e-13)
    na, nb = np.sqrt(13 / 4), np.sqrt(43 / 32)
    p3_neg = 4 * -1 * (5 / 16 + na * nb)      # the negative eigenvalue of part 3
    w = np.linalg.eigvalsh(raw - per)          # raw - per_part = the removed negative part of part 3
    assert np.sum(np.abs(w) > 1e-10) == 1
    assert w[0] == pytest.approx(p3_neg, rel=1e-12)
    # the full Eq. 4 matrix is indefinite: core det = -12 t0^2 t1^2 < 0
    wr = np.linalg.eigvalsh(raw)
    assert wr[0] < -1.0 and wr[-1] > 1.0
    assert np.linalg.eigvalsh(per)[0] > -1e-12


def test_appendix_half_interval_is_exact_sixteenth():
    # the appendix halves both ends of I_c; T scales by exactly 1/16 (power of two)
    for X in [WORKED] + [p for p, _ in _random_hits(np.random.default_rng(3), 20)]:
        f = oracle.pair(X)
        h = oracle.pair(X, interval=oracle.INTERVAL_APPENDIX_HALF)
        assert h["status"] == f["status"] == oracle.ST_HIT
        assert h["T"] * 16 == f["T"]
        assert h["t0"] * 2 == f["t0"] and h["t1"] * 2 == f["t1"]
        np.testing.assert_array_equal(h["g"] * 16, f["g"])


def test_translation_closed_form():
    # moving T_b by delta along x shifts I_b by -delta in t = -x: t_c = (delta-1, delta+1),
    # T(delta) = (1 - delta^2)^2 for |delta| < 1 and 0 beyond (the open interval excludes 0)
    for delta in [-1.5, -1.0, -0.75, -0.3, 0.0, 0.2, 0.6, 0.999, 1.0, 1.25]:
        X = WORKED.copy()
        X[3:, 0] += delta
        r = oracle.pair(X)
        if abs(delta) < 1:
            assert r["status"] == oracle.ST_HIT
            assert r["t0"] == pytest.approx(delta - 1, abs=1e-15)
            assert r["t1"] == pytest.approx(delta + 1, abs=1e-15)
            assert r["T"] == pytest.approx((1 - delta * delta) ** 2, rel=1e-14, abs=1e-15)
        else:
            assert r["T"] == 0.0 and r["status"] != oracle.ST_HIT


def test_translation_second_derivative():
    # along v = d/d(delta) (x-motion of T_b) t is linear in delta, so both v^T (Eq. 4) v and
    # the exact v^T H v equal T''(delta) = 12 delta^2 - 4
    v = np.zeros((6, 3))
    v[3:, 0] = 1.0
    v = v.ravel()
    for delta in [-0.6, -0.1, 0.0, 0.35, 0.8]:
        X = WORKED.copy()
        X[3:, 0] += delta
        raw = oracle.pair(X, psd=oracle.PSD_RAW_EQ4)
        assert raw["a"] @ v == pytest.approx(1.0, abs=1e-14) and raw["b"] @ v == pytest.approx(1.0, abs=1e-14)
        expect = 12 * delta * delta - 4
        assert v @ raw["H"] @ v == pytest.approx(expect, rel=1e-12, abs=1e-12)
        assert v @ oracle.pair_hvp(X, v) == pytest.approx(expect, rel=1e-12, abs=1e-12)


# ---------------------------------------------------------------------------------------
# Exact flags: brute force against the exact-rational Moeller test.
# ---------------------------------------------------------------------------------------
def _check_against_exact(x, tris, pairs, check_values=True):
    res = oracle.evaluate(x, tris, pairs, hessian=False)
    n_hits = 0
    for k, (i, j) in enumerate(pairs):
        if exact_moller.shares_vertex(tris[i], tris[j]):
            assert res["flags"][k] == oracle.ST_ADJACENT
            continue
        ex = exact_moller.pair(x[tris[i]], x[tris[j]])
        assert (res["flags"][k] == oracle.ST_HIT) == ex["flag"], (k, i, j, ex)
        if ex["flag"]:
            n_hits += 1
            if check_values:
                nd = np.sqrt(float(ex["DD"]))
                t0, t1 = float(ex["tc0"]) / nd, float(ex["tc1"]) / nd
                scale = max(abs(t0), abs(t1))
                assert abs(res["t"][k, 0] - t0) <= 1e-12 * scale + 1e-300
                assert abs(res["t"][k, 1] - t1) <= 1e-12 * scale + 1e-300
                # |t - t*| <= d for both ends bounds |t0 t1 - t0* t1*| by dp, hence T's error
                d = 1e-12 * scale
                dp = (abs(t0) + abs(t1)) * d + d * d
                assert abs(res["T"][k] - (t0 * t1) ** 2) <= (2 * abs(t0 * t1) + dp) * dp + 1e-300
        else:
            assert res["T"][k] == 0.0
    return n_hits


@pytest.mark.parametrize("seed", range(4))
def test_flags_integer_grid_brute_force(seed):
    # integer vertices in {-3..3}^3: dense in coplanar, touching and vertex-on-plane cases
    x, tris = _integer_triangles(seed, 70)
    pairs = np.array(list(itertools.combinations(range(len(tris)), 2)), np.int32)
    hits = _check_against_exact(x, tris, pairs)
    assert hits > 20


def test_flags_near_degenerate_perturbed():
    # integer configurations nudged by 2^-45: FP64 signs become unreliable, exact ones decide
    rng = np.random.default_rng(11)
    x, tris = _integer_triangles(7, 60)
    x = x + rng.integers(-1, 2, size=x.shape) * 2.0 ** -45
    pairs = np.array(list(itertools.combinations(range(len(tris)), 2)), np.int32)
    # flags only: with every vertex within 2^-45 of the other plane the FP64 lerp weights
    # (and so t) are ill-conditioned by construction; the exact flag is not
    assert _check_against_exact(x, tris, pairs, check_values=False) > 10


def test_values_vs_exact_random_floats():
    # generic (well-conditioned) float triangles: t_c^0, t_c^1 and T against exact rationals
    rng = np.random.default_rng(12)
    x = rng.normal(size=(3 * 150, 3)) * 0.7
    x[75 * 3:] += 0.3
    tris = np.arange(3 * 150, dtype=np.int32).reshape(150, 3)
    pairs = np.array(list(itertools.combinations(range(len(tris)), 2)), np.int32)
    assert _check_against_exact(x, tris, pairs) > 100


def test_flags_shared_vertex_meshes():
    # small noisy sphere: adjacency detection plus exact flags over all pairs
    from paper_2606_06511_amd import workloads

    x, tris = workloads.noisy_sphere(seed=1, n_lon=12, n_bands=7, amplitude=0.3)
    pairs = oracle.pairs(x, tris, oracle.BROAD_BRUTE)
    _check_against_exact(x, tris, pairs, check_values=True)


def test_orient_sign_exact():
    rng = np.random.default_rng(5)
    for _ in range(300):
        pts = rng.integers(-4, 5, size=(4, 3)).astype(float)
        if rng.random() < 0.5:
            pts[3] = pts[0] + rng.integers(-2, 3) * (pts[1] - pts[0]) + rng.integers(-2, 3) * (pts[2] - pts[0])
        pts = pts * 0.1  # non-dyadic values: the FP64 determinant is no longer exact
        assert oracle.orient_sign(*pts) == exact_moller.orient_sign(*pts)


# ---------------------------------------------------------------------------------------
# Derivatives: Eq. 3 and finite differences
# ---------------------------------------------------------------------------------------
def _integer_triangles(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.integers(-3, 4, size=(3 * n, 3)).astype(np.float64)
    return x, np.arange(3 * n, dtype=np.int32).reshape(n, 3)


def _random_hits(rng, n):
    out = []
    while len(out) < n:
        u = rng.normal(size=(3, 3))
        v = u.mean(0) + 0.8 * rng.normal(size=(3, 3))
        X = np.concatenate([u, v])
        r = oracle.pair(X)
        if r["status"] == oracle.ST_HIT and abs(r["t0"]) > 1e-3 and abs(r["t1"]) > 1e-3:
            out.append((X, r))
    return out


def _signature(X):
    """Branch signature: exact side signs of both cuts (what selects the formula)."""
    u, v = X[:3], X[3:]
    return tuple(oracle.orient_sign(*v, p) for p in u) + tuple(oracle.orient_sign(*u, p) for p in v)


def test_gradient_is_eq3():
    for X, r in _random_hits(np.random.default_rng(0), 40):
        t0, t1 = r["t0"], r["t1"]
        np.testing.assert_allclose(r["g"], 2 * t0 * t1 * t1 * r["a"] + 2 * t1 * t0 * t0 * r["b"],
                                   rtol=1e-13, atol=1e-13 * np.abs(r["g"]).max())


def test_gradient_and_interval_derivatives_fd():
    h = 1e-6
    checked = 0
    for X, r in _random_hits(np.random.default_rng(1), 30):
        sig = _signature(X)
        for k in range(18):
            Xp, Xm = X.copy().ravel(), X.copy().ravel()
            Xp[k] += h
            Xm[k] -= h
            Xp, Xm = Xp.reshape(6, 3), Xm.reshape(6, 3)
            if _signature(Xp) != sig or _signature(Xm) != sig:
                continue
            rp, rm = oracle.pair(Xp), oracle.pair(Xm)
            if rp["status"] != oracle.ST_HIT or rm["status"] != oracle.ST_HIT:
                continue
            # the min/max picks must not change either (a kink of t)
            if np.sign(rp["t0"] - r["t0"]) * np.sign(r["t0"] - rm["t0"]) < 0:
                continue
            for key, fd in (("a", (rp["t0"] - rm["t0"]) / (2 * h)), ("b", (rp["t1"] - rm["t1"]) / (2 * h)),
                            ("g", (rp["T"] - rm["T"]) / (2 * h))):
                ref = r[key][k]
                scale = max(1.0, np.abs(r[key]).max())
                assert abs(fd - ref) <= 2e-6 * scale, (key, k, fd, ref)
            checked += 1
    assert checked > 400


def _exact_t_derivative(X, v):
    """Directional derivatives of the exact (t_c^0, t_c^1) along v: exact rational difference
    quotients of tc and |D|^2 over a step of 2^-120 (far below any kink of these inputs, so
    the truncation error is O(2^-120)), then t = tc / |D|."""
    from fractions import Fraction

    h = Fraction(1, 2 ** 120)
    Xq = [[Fraction(float(c)) for c in row] for row in X]
    Xh = [[Xq[i][c] + h * Fraction(float(v[3 * i + c])) for c in range(3)] for i in range(6)]
    e0, e1 = exact_moller.pair(Xq[:3], Xq[3:]), exact_moller.pair(Xh[:3], Xh[3:])
    assert e0["flag"] and e1["flag"]
    DD, dDD = float(e0["DD"]), float((e1["DD"] - e0["DD"]) / h)
    out = []
    for key in ("tc0", "tc1"):
        tc, dtc = float(e0[key]), float((e1[key] - e0[key]) / h)
        out.append(dtc / np.sqrt(DD) - tc * dDD / (2 * DD ** 1.5))
    return out


def test_interval_derivatives_at_near_tied_ends():
    """A vertex within 2^-60..2^-48 of the other triangle's plane makes its two crossing
    points (one segment's ends) nearly coincide: their t values differ by less than their
    rounding error, and picking the wrong one as the minimum swaps the derivatives of two
    different edge crossings.  The oracle's dt_c^0/dX and dt_c^1/dX must be those of the
    exact interval; both triangles take the near vertex in every position."""
    rng = np.random.default_rng(21)
    checked = 0
    for trial in range(48):
        # T_b in the plane y = 0, T_a with a lone vertex just above it and two below
        tb = np.array([[-1.0, 0.0, -1.0], [2.0, 0.0, -1.0], [0.5, 0.0, 2.0]])
        tb[:, [0, 2]] += rng.normal(0, 0.05, size=(3, 2))
        near = np.array([0.4 + 0.2 * rng.random(), 2.0 ** -rng.uniform(48, 60), 0.1 + 0.2 * rng.random()])
        far = np.array([[rng.uniform(-0.2, 0.3), -1 - rng.random(), rng.uniform(0.3, 0.9)],
                        [rng.uniform(0.8, 1.3), -1 - rng.random(), rng.uniform(-0.6, 0.0)]])
        ta = np.concatenate([near[None], far])[np.roll(np.arange(3), trial % 3)]
        if trial % 6 >= 3:
            ta = ta[[0, 2, 1]]  # the other orientation
        X = np.concatenate([ta, tb]) if trial % 2 == 0 else np.concatenate([tb, ta])
        r = oracle.pair(X)
        assert r["status"] == oracle.ST_HIT
        v = rng.normal(size=18)
        da, db = _exact_t_derivative(X, v)
        scale = max(1.0, np.abs(r["a"]).max(), np.abs(r["b"]).max()) * np.linalg.norm(v)
        assert abs(r["a"] @ v - da) <= 1e-9 * scale, (trial, r["a"] @ v, da)
        assert abs(r["b"] @ v - db) <= 1e-9 * scale, (trial, r["b"] @ v, db)
        checked += 1
    assert checked == 48


def test_exact_hvp_fd():
    h = 1e-6
    rng = np.random.default_rng(2)
    for X, r in _random_hits(rng, 25):
        v = rng.normal(size=18)
        v /= np.linalg.norm(v)
        Xp, Xm = (X.ravel() + h * v).reshape(6, 3), (X.ravel() - h * v).reshape(6, 3)
        if _signature(Xp) != _signature(X) or _signature(Xm) != _signature(X):
            continue
        gp, gm = oracle.pair(Xp)["g"], oracle.pair(Xm)["g"]
        fd = (gp - gm) / (2 * h)
        hv = oracle.pair_hvp(X, v)
        np.testing.assert_allclose(hv, fd, atol=2e-5 * max(1.0, np.abs(hv).max()))


def test_exact_hessian_differs_from_eq4_by_curvature():
    # Eq. 4 drops 2 t0 t1 (t1 H(t0) + t0 H(t1)); with t linear along the worked-example
    # translation they agree, for generic directions they do not
    rng = np.random.default_rng(4)
    diffs = []
    for X, r in _random_hits(rng, 10):
        H = np.stack([oracle.pair_hvp(X, e) for e in np.eye(18)])
        np.testing.assert_allclose(H, H.T, atol=1e-9 * np.abs(H).max())
        raw = oracle.pair(X, psd=oracle.PSD_RAW_EQ4)["H"]
        diffs.append(np.abs(H - raw).max() / np.abs(raw).max())
    assert max(diffs) > 1e-3


# ---------------------------------------------------------------------------------------
# Hessian variants
# ---------------------------------------------------------------------------------------
def test_psd_variants_closed_forms():
    for X, r in _random_hits(np.random.default_rng(6), 30):
        t0, t1, a, b = r["t0"], r["t1"], r["a"], r["b"]
        raw = oracle.pair(X, psd=oracle.PSD_RAW_EQ4)["H"]
        per = oracle.pair(X, psd=oracle.PSD_PER_PART)["H"]
        lit = oracle.pair(X, psd=oracle.PSD_PAPER_LITERAL)["H"]
        near = oracle.pair(X, psd=oracle.PSD_NEAREST)["H"]
        scale = np.abs(raw).max()
        # Eq. 4 term by term
        eq4 = 2 * t1 * t1 * np.outer(a, a) + 2 * t0 * t0 * np.outer(b, b) + 4 * t0 * t1 * (np.outer(b, a) + np.outer(a, b))
        np.testing.assert_allclose(raw, eq4, atol=1e-13 * scale)
        # trace = sum of the three "eigenvalues" named in the eigenanalysis
        assert np.trace(raw) == pytest.approx(2 * t1 * t1 * a @ a + 2 * t0 * t0 * b @ b + 8 * t0 * t1 * a @ b, rel=1e-12)
        # per-part: parts 1 and 2 kept; part 3 keeps only 4|t0 t1|(|a||b| - a.b) along a/|a| - b/|b|
        na, nb = np.linalg.norm(a), np.linalg.norm(b)
        w = nb * a - na * b
        p3plus = 2 * abs(t0 * t1) / (na * nb) * np.outer(w, w)
        np.testing.assert_allclose(per, 2 * t1 * t1 * np.outer(a, a) + 2 * t0 * t0 * np.outer(b, b) + p3plus,
                                   atol=1e-11 * scale)
        for M in (per, near):
            ev = np.linalg.eigvalsh(M)
            assert ev[0] >= -1e-11 * scale
            assert np.sum(ev > 1e-9 * scale) <= 2
            np.testing.assert_allclose(M, M.T, atol=1e-12 * scale)
            # rigid translations are in the null space
            for c in range(3):
                tvec = np.zeros((6, 3))
                tvec[:, c] = 1
                assert np.abs(M @ tvec.ravel()).max() <= 1e-10 * scale
        # nearest: Frobenius projection keeps the positive eigenpairs of Eq. 4
        ev, Q = np.linalg.eigh(raw)
        np.testing.assert_allclose(near, (Q * np.maximum(ev, 0)) @ Q.T, atol=1e-10 * scale)
        # paper-literal keeps part 3 only when 8 t0 t1 a.b > 0
        keep = 8 * t0 * t1 * (a @ b) > 0
        expect = eq4 if keep else eq4 - 4 * t0 * t1 * (np.outer(b, a) + np.outer(a, b))
        np.testing.assert_allclose(lit, expect, atol=1e-12 * scale)


def test_jacobi_eigen_against_lapack():
    rng = np.random.default_rng(8)
    for n in (2, 5, 18):
        A = rng.normal(size=(n, n))
        A = A + A.T
        w, Q = oracle.eig(A)
        np.testing.assert_allclose(np.sort(w), np.linalg.eigvalsh(A), atol=1e-12 * np.abs(A).max())
        np.testing.assert_allclose((Q * w) @ Q.T, A, atol=1e-12 * np.abs(A).max())


# ---------------------------------------------------------------------------------------
# Invariances of the definition
# ---------------------------------------------------------------------------------------
def _rotation(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_invariances():
    rng = np.random.default_rng(9)
    for X, r in _random_hits(rng, 25):
        T = r["T"]
        g = r["g"].reshape(6, 3)
        # rigid motion: T invariant, gradient rotates with the frame
        R, t = _rotation(rng), rng.normal(size=3)
        rr = oracle.pair(X @ R.T + t)
        assert rr["T"] == pytest.approx(T, rel=1e-9)
        np.testing.assert_allclose(rr["g"].reshape(6, 3), g @ R.T, atol=1e-8 * np.abs(g).max())
        # scaling: T(sX) = s^4 T(X)
        assert oracle.pair(2.5 * X)["T"] == pytest.approx(2.5 ** 4 * T, rel=1e-12)
        # relabelling vertices within a triangle (either orientation)
        for perm in itertools.permutations(range(3)):
            Y = np.concatenate([X[list(perm)], X[3 + np.array(perm[::-1])]])
            assert oracle.pair(Y)["T"] == pytest.approx(T, rel=1e-9)
        # swapping the triangles swaps I_a and I_b but also flips D = n_a x n_b (t -> -t),
        # so t_c^0 = min I_a - max I_b and t_c^1 are unchanged
        s = oracle.pair(np.concatenate([X[3:], X[:3]]))
        assert s["t0"] == pytest.approx(r["t0"], rel=1e-9) and s["t1"] == pytest.approx(r["t1"], rel=1e-9)
        np.testing.assert_allclose(s["g"].reshape(6, 3), np.concatenate([g[3:], g[:3]]), atol=1e-8 * np.abs(g).max())
        # zero net force and torque per pair
        assert np.abs(g.sum(0)).max() <= 1e-12 * np.abs(g).max()
        assert np.abs(np.cross(X, g).sum(0)).max() <= 1e-11 * np.abs(g).max() * np.abs(X).max()
        # the interval derivatives ignore the motion of the line direction: both t's move
        # with the endpoints' gradients projected on D, which is translation-free as well
        assert np.abs(r["a"].reshape(6, 3).sum(0)).max() <= 1e-12 * np.abs(r["a"]).max()


# ---------------------------------------------------------------------------------------
# Broad phase and assembly
# ---------------------------------------------------------------------------------------
def test_brute_force_candidate_count_closed_form():
    from paper_2606_06511_amd import workloads

    x, tris = workloads.two_icospheres(0)
    p = oracle.pairs(x, tris, oracle.BROAD_BRUTE)
    # C(2560,2) minus pairs sharing a vertex: per sphere sum_v C(val_v,2) - #edges
    # = 12*C(5,2) + 630*C(6,2) - 1920 = 7650
    assert len(p) == 2560 * 2559 // 2 - 2 * 7650 == 3_260_220
    assert np.all(p[:, 0] < p[:, 1])


@pytest.mark.parametrize("which", ["sphere", "cloth"])
def test_box_pairs_match_all_pairs_box_test(which):
    from paper_2606_06511_amd import workloads

    if which == "sphere":
        x, tris = workloads.noisy_sphere(seed=2, n_lon=48, n_bands=25)
    else:
        x, tris = workloads.folded_cloth(seed=3, n=32)
    got = oracle.pairs(x, tris, oracle.BROAD_BOXES)
    V = x[tris]
    lo, hi = V.min(1), V.max(1)
    ov = np.all((lo[:, None, :] <= hi[None, :, :]) & (lo[None, :, :] <= hi[:, None, :]), axis=2)
    shared = np.zeros_like(ov)
    for a in range(3):
        for b in range(3):
            shared |= tris[:, a][:, None] == tris[:, b][None, :]
    i, j = np.nonzero(np.triu(ov & ~shared, 1))
    np.testing.assert_array_equal(got, np.stack([i, j], 1))


def test_assembly_consistency():
    from paper_2606_06511_amd import workloads

    x, tris = workloads.folded_cloth(seed=0, n=40)
    pairs = oracle.pairs(x, tris)
    res = oracle.evaluate(x, tris, pairs)
    assert len(res["hit_pair"]) > 5
    nv = len(x)
    # energy is the plain sum of the per-pair energies
    assert res["E"] == pytest.approx(res["T"].sum(), rel=1e-14)
    # gradient and Hessian are the scatter of the per-hit pieces
    G = np.zeros((nv, 3))
    H = np.zeros((3 * nv, 3 * nv))
    for k, p in enumerate(res["hit_pair"]):
        vid = np.concatenate([tris[pairs[p, 0]], tris[pairs[p, 1]]])
        dof = (3 * vid[:, None] + np.arange(3)).ravel()
        G[vid] += res["hit_g"][k].reshape(6, 3)
        H[np.ix_(dof, dof)] += res["hit_H"][k]
    np.testing.assert_allclose(res["G"], G, atol=1e-14 * np.abs(G).max())
    Hb = oracle.bsr_to_dense(res["row_ptr"], res["col_idx"], res["vals"], nv)
    np.testing.assert_allclose(Hb, H, atol=1e-13 * np.abs(H).max())
    np.testing.assert_allclose(Hb, Hb.T, atol=1e-13 * np.abs(H).max())
    # block structure: sorted unique columns per row, and every block is touched by a hit
    for r in range(nv):
        cols = res["col_idx"][res["row_ptr"][r]:res["row_ptr"][r + 1]]
        assert np.all(np.diff(cols) > 0)
    # the PSD Hessian-vector product agrees with the assembled matrix
    v = np.random.default_rng(0).normal(size=(nv, 3))
    hv = oracle.hvp(x, tris, pairs, v, exact=False)
    np.testing.assert_allclose(hv.ravel(), Hb @ v.ravel(), atol=1e-12 * np.abs(Hb).max() * np.abs(v).max())
    # the global gradient matches central differences of the global energy
    rng = np.random.default_rng(1)
    d = rng.normal(size=x.shape)
    h = 1e-7
    Ep = oracle.evaluate(x + h * d, tris, pairs, hessian=False)["E"]
    Em = oracle.evaluate(x - h * d, tris, pairs, hessian=False)["E"]
    assert (Ep - Em) / (2 * h) == pytest.approx(np.sum(res["G"] * d), rel=1e-4)


def test_swept_pairs_brute_force():
    # swept candidates: every non-adjacent pair whose boxes over both positions overlap, by an
    # O(N^2) numpy test
    from paper_2606_06511_amd import workloads

    x, tris = workloads.folded_cloth(3, n=20)
    x_end = x + 0.02 * np.random.default_rng(4).normal(size=x.shape)
    got = oracle.pairs_swept(x, x_end, tris)
    lo = np.minimum(x[tris].min(1), x_end[tris].min(1))
    hi = np.maximum(x[tris].max(1), x_end[tris].max(1))
    ov = np.all((lo[:, None, :] <= hi[None, :, :]) & (lo[None, :, :] <= hi[:, None, :]), axis=2)
    shared = (tris[:, None, :, None] == tris[None, :, None, :]).any(axis=(2, 3))
    i, j = np.nonzero(np.triu(ov & ~shared, 1))
    np.testing.assert_array_equal(got, np.stack([i, j], 1).astype(got.dtype))
    assert len(got) > len(oracle.pairs(x, tris))


def test_newton_matches_dense_newton():
    """The oracle's inexact Newton against the same iteration written with dense linear algebra:
    (H + mu I) d = -g solved exactly (PCG run to convergence must agree), mu = 1e-3 * mean
    diagonal of the rows holding blocks, Armijo halving on E over the swept candidates."""
    from paper_2606_06511_amd import workloads

    x, tris = workloads.folded_cloth(0, n=24)
    steps = 3
    _, E_or, al_or, _ = oracle.newton(x, tris, steps=steps, pcg_iters=5000, pcg_tol=1e-14)
    xc = x.copy()
    E_ref, al_ref = [], []
    for _ in range(steps):
        r = oracle.evaluate(xc, tris, oracle.pairs(xc, tris), hessian=True)
        E = r["E"]
        E_ref.append(E)
        H = oracle.bsr_to_dense(r["row_ptr"], r["col_idx"], r["vals"], len(xc))
        g = r["G"].ravel()
        rows = np.repeat(np.diff(r["row_ptr"]) > 0, 3)
        mu = 1e-3 * np.diag(H)[rows].mean()
        d = np.linalg.solve(H + mu * np.eye(len(g)), -g).reshape(-1, 3)
        cand = oracle.pairs_swept(xc, xc + d, tris)
        alpha = 1.0
        for h in range(30):
            Et = oracle.evaluate(xc + alpha * d, tris, cand, hessian=False)["E"]
            if Et <= E + 1e-4 * alpha * float(g @ d.ravel()) or h == 29:
                break
            alpha *= 0.5
        al_ref.append(alpha)
        xc = xc + alpha * d
    E_ref.append(oracle.evaluate(xc, tris, oracle.pairs(xc, tris), hessian=False)["E"])
    assert E_ref[0] > 0
    np.testing.assert_allclose(E_or, E_ref, rtol=1e-7)
    assert list(al_or) == al_ref


# ---------------------------------------------------------------------------------------
# Pairs sharing exactly one vertex (an option; the paper excludes every adjacent pair).
# T_a in z = 0 and T_b = (0,0,0), (1,.5,1), (1,.5,-1) in the plane y = x/2 share the origin.
# D = n_a x n_b = (0,0,4) x (-1,2,0) = (-8,-4,0), so t = -(2x + y)/sqrt(5).  T_a meets the
# plane from the origin to (4/3, 2/3, 0) (edge u1u2), T_b meets z = 0 from the origin to
# (1, 1/2, 0) (edge v1v2): I_a = [-10/3, 0]/sqrt(5), I_b = [-5/2, 0]/sqrt(5), and Eq. 1 gives
# t_c = [-10/3, 5/2]/sqrt(5): T = ((10/3)(5/2)/5)^2 = 25/9.  Mirroring T_b through the origin
# makes the two cuts leave the shared vertex in opposite directions: they only touch, T = 0.
# ---------------------------------------------------------------------------------------
VA = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0], [0, 0, 0], [1, .5, 1], [1, .5, -1]], float)


def test_vertex_adjacent_closed_form():
    r = oracle.pair(VA)
    assert r["status"] == oracle.ST_HIT
    assert r["t0"] == pytest.approx(-10 / 3 / np.sqrt(5), rel=1e-14)
    assert r["t1"] == pytest.approx(5 / 2 / np.sqrt(5), rel=1e-14)
    assert r["T"] == pytest.approx(25 / 9, rel=1e-14)
    mirror = VA.copy()
    mirror[4:] *= [-1, -1, 1]
    assert oracle.pair(mirror)["status"] == oracle.ST_NONE
    # at the mesh level the shared index makes the pair adjacent unless vertex_adjacent is set
    x = VA[[0, 1, 2, 4, 5]]
    tris = np.array([[0, 1, 2], [0, 3, 4]], np.int32)
    assert len(oracle.pairs(x, tris)) == 0
    pl = oracle.pairs(x, tris, vertex_adjacent=True)
    np.testing.assert_array_equal(pl, [[0, 1]])
    assert oracle.evaluate(x, tris, pl)["E"] == 0.0
    r = oracle.evaluate(x, tris, pl, vertex_adjacent=True)
    assert r["E"] == pytest.approx(25 / 9, rel=1e-14)
    # pairs sharing an edge stay adjacent
    tris_e = np.array([[0, 1, 2], [0, 1, 3]], np.int32)
    assert len(oracle.pairs(x, tris_e, oracle.BROAD_BRUTE, vertex_adjacent=True)) == 0


def test_vertex_adjacent_flags_vs_exact():
    rng = np.random.default_rng(11)
    n_hit = 0
    for _ in range(1500):
        P = rng.integers(-3, 4, size=(5, 3)).astype(float)
        tris = np.array([[0, 1, 2], [0, 3, 4]], np.int32)
        r = oracle.evaluate(P, tris, np.array([[0, 1]], np.int32), hessian=False, vertex_adjacent=True)
        e = exact_moller.pair(P[[0, 1, 2]], P[[0, 3, 4]])
        # small integers: every normal and D is exact, so a hit never has a zero line direction
        assert r["flags"][0] != 3
        assert (r["flags"][0] == 1) == bool(e["flag"])
        n_hit += r["flags"][0] == 1
    assert n_hit > 100


def test_vertex_adjacent_gradient_fd():
    # the shared vertex is one vertex: its gradient collects both slots
    from paper_2606_06511_amd import workloads

    x, tris = workloads.crumpled_fans(3, n_fans=2, blades=12)
    pl = oracle.pairs(x, tris, vertex_adjacent=True)
    r = oracle.evaluate(x, tris, pl, hessian=False, vertex_adjacent=True)
    assert len(r["hit_pair"]) > 5
    h = 1e-6
    fd = np.zeros_like(x)
    for v in range(len(x)):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[v, c] += h
            xm[v, c] -= h
            fd[v, c] = (oracle.evaluate(xp, tris, pl, hessian=False, vertex_adjacent=True)["E"] -
                        oracle.evaluate(xm, tris, pl, hessian=False, vertex_adjacent=True)["E"]) / (2 * h)
    assert np.abs(fd - r["G"]).max() <= 1e-6 * max(1.0, np.abs(r["G"]).max())
    assert np.abs(r["G"][0]).max() > 0  # the centre vertex of the first fan feels the crossings


def test_vertex_adjacent_pairs_definition():
    from paper_2606_06511_amd import workloads

    x, tris = workloads.crumpled_fans(2, n_fans=3, blades=10)
    got = oracle.pairs(x, tris, vertex_adjacent=True)
    lo, hi = x[tris].min(1), x[tris].max(1)
    ov = np.all((lo[:, None, :] <= hi[None, :, :]) & (lo[None, :, :] <= hi[:, None, :]), axis=2)
    shared = (tris[:, None, :, None] == tris[None, :, None, :]).any(axis=3).sum(axis=2)
    i, j = np.nonzero(np.triu(ov & (shared <= 1), 1))
    np.testing.assert_array_equal(got, np.stack([i, j], 1).astype(got.dtype))


# ---------------------------------------------------------------------------------------
# The line frame at the edges of float64.  Eq. 1-2 are homogeneous: scaling every coordinate
# by s = 2^k (exact in float64) scales t_c by s and T by s^4, and leaves a = dt_c^0/dX and
# b = dt_c^1/dX unchanged.  At s = 2^-150 the direction D = n_a x n_b is of order 2^-600, so
# |D|^2 would underflow to 0; at s = 2^150 it would overflow.  The oracle scales D by a power of
# two before normalising it, so both give the worked example's values exactly.
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("k", [-150, 150])
def test_worked_example_at_extreme_scale(k):
    s = 2.0 ** k
    r = oracle.pair(WORKED * s)
    assert r["status"] == oracle.ST_HIT
    assert r["t0"] == GOLDEN["t0"] * s and r["t1"] == GOLDEN["t1"] * s
    assert r["T"] == GOLDEN["T"] * s ** 4
    np.testing.assert_allclose(r["a"].reshape(6, 3), A_WORKED, atol=1e-15)
    np.testing.assert_allclose(r["b"].reshape(6, 3), B_WORKED, atol=1e-15)
    np.testing.assert_allclose(r["g"].reshape(6, 3) / s ** 3, np.array(GOLDEN["g"]), atol=1e-15)
    # every operation is a power-of-two multiple of the unscaled one: bit-identical a and b
    u = oracle.pair(WORKED)
    np.testing.assert_array_equal(r["a"], u["a"])
    np.testing.assert_array_equal(r["b"], u["b"])
    e = exact_moller.pair(WORKED[:3] * s, WORKED[3:] * s)
    assert e["flag"]


# ---------------------------------------------------------------------------------------
# The degenerate line frame (status 3).  An exact hit always has a non-zero line direction:
# both triangles straddle the other's plane, so the planes are not parallel.  Only rounding can
# make the float64 D = n_a x n_b vanish, and tests/golden/degenerate_frame.json holds a pair
# built by hand for that: the two products of each component of n_b round to the same double.
# The exact-rational Moeller test finds the intersection; the oracle reports status 3, T = 0.
# ---------------------------------------------------------------------------------------
DEGENERATE = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "degenerate_frame.json")))


def test_degenerate_frame_pair():
    X = np.array([[float.fromhex(c) for c in p] for p in DEGENERATE["X_hex"]])
    np.testing.assert_array_equal(X, np.array(DEGENERATE["X"], float))
    e = exact_moller.pair(X[:3], X[3:])
    assert e["straddle"] and e["flag"]
    assert e["DD"] > 0  # the exact direction is not zero
    r = oracle.pair(X)
    assert r["status"] == DEGENERATE["status"] == oracle.ST_BAD_FRAME
    assert r["T"] == 0.0 and not np.any(r["g"]) and not np.any(r["H"])
    # the same pair inside a mesh: flag 3, no energy, no gradient, no Hessian block
    tris = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    m = oracle.evaluate(X, tris, np.array([[0, 1]], np.int32))
    assert m["flags"][0] == 3 and m["E"] == 0.0 and not np.any(m["G"]) and len(m["vals"]) == 0
    # nudging the tilt so that the products no longer round together gives an ordinary hit
    Y = X.copy()
    Y[5, 2] += 2.0 ** -90  # v2.z - v0.z = 2^-40 (1 + 2^-51 + 2^-50), exact; n_b.x = 2^-90
    assert oracle.pair(Y)["status"] == oracle.ST_HIT and exact_moller.pair(Y[:3], Y[3:])["flag"]
