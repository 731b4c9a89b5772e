"""Seeded synthetic triangle meshes shaped like the workloads the TTIE hot path runs on.

This module holds mesh construction only: vertex positions, triangle index arrays and the
seeded random draws that perturb them.  It contains none of the intersection-energy
arithmetic, so both the GPU path and the CPU oracle can be fed from it.

Every generator returns ``(x, tris)`` with ``x`` a C-contiguous float64 array of shape
``(n_verts, 3)`` and ``tris`` a C-contiguous int32 array of shape ``(n_tris, 3)``.  All
randomness comes from ``numpy.random.default_rng(seed)`` in a fixed draw order, so a
(generator, seed) pair always yields the same bytes.

Workloads (sizes as stated in the method's evaluation plan; the paper itself gives none):

* ``two_icospheres``   two radius-1 icospheres (3 subdivisions, 642 verts / 1280 tris
  each), the second translated by (0.5, 0.13, 0.07), all vertices jittered by N(0, 1e-3).
  Used with the brute-force all-pairs candidate list.
* ``folded_cloth``     a 256x256 vertex grid on [0,1]^2 (130,050 tris) with a height
  field of 8 Gaussian bumps, folded so that x > 0.5 maps to 1 - x; the two layers cross.
* ``noisy_sphere``     a UV sphere (n_lon x (n_lat bands), polar fans) displaced by a
  band-limited *vector* noise field of amplitude 0.05 so that the surface folds through
  itself.  A purely radial displacement of a star-shaped sphere cannot self-intersect
  (each face stays inside its own cone from the centre), hence the tangential part.
* ``batch_problems``   64 independent two-mesh problems mixing icospheres, tori and
  bump grids with log-uniform sizes, the second mesh of each problem rigidly moved so the
  two overlap.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "icosphere",
    "two_icospheres",
    "grid_mesh",
    "folded_cloth",
    "uv_sphere",
    "vector_noise",
    "noisy_sphere",
    "torus",
    "bump_grid",
    "batch_problems",
    "union",
    "integer_grid_triangles",
    "submesh_near",
]


def _finish(x, tris):
    return np.ascontiguousarray(x, dtype=np.float64), np.ascontiguousarray(tris, dtype=np.int32)


def icosphere(subdivisions: int = 3, radius: float = 1.0):
    """Icosahedron refined by 4-way midpoint subdivision, re-projected to the sphere.

    subdivisions=3 gives 642 vertices / 1280 triangles.  Faces are counter-clockwise seen
    from outside.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [
        (-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
        (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
        (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1),
    ]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    faces = [
        (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
        (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
        (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
        (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
    ]
    for _ in range(subdivisions):
        cache: dict[tuple[int, int], int] = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        new_faces = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    x = np.array(verts) * radius
    return _finish(x, np.array(faces))


def union(meshes):
    """Concatenate meshes into one vertex/triangle array (triangle indices re-based)."""
    xs, ts, off = [], [], 0
    for x, t in meshes:
        xs.append(x)
        ts.append(t + off)
        off += len(x)
    return _finish(np.concatenate(xs), np.concatenate(ts))


def two_icospheres(seed: int = 0, subdivisions: int = 3, offset=(0.5, 0.13, 0.07), jitter=1e-3):
    """Two overlapping radius-1 icospheres as one union mesh (1,284 verts / 2,560 tris)."""
    rng = np.random.default_rng(seed)
    xa, ta = icosphere(subdivisions)
    xb = xa + np.asarray(offset, dtype=np.float64)
    x, tris = union([(xa, ta), (xb, ta)])
    x = x + rng.normal(0.0, jitter, size=x.shape)
    return _finish(x, tris)


def grid_mesh(n: int):
    """n x n vertex grid on [0,1]^2 (z = 0); each quad split along its (i,j)-(i+1,j+1) diagonal.

    Vertex (i, j) has id i*n + j and sits at (i/(n-1), j/(n-1), 0).
    """
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = np.stack([i / (n - 1), j / (n - 1), np.zeros_like(i, dtype=np.float64)], axis=-1).reshape(-1, 3)
    a = (i[:-1, :-1] * n + j[:-1, :-1]).ravel()
    b = a + n          # (i+1, j)
    c = a + n + 1      # (i+1, j+1)
    d = a + 1          # (i, j+1)
    tris = np.stack([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 1).reshape(-1, 3)
    return _finish(x.astype(np.float64), tris)


def _bump_field(rng, n_bumps=8):
    amp = rng.uniform(-1.0, 1.0, n_bumps)
    ctr = rng.uniform(0.0, 1.0, (n_bumps, 2))
    sig = rng.uniform(0.05, 0.2, n_bumps)

    def z(px, py):
        out = np.zeros_like(px)
        for k in range(n_bumps):
            r2 = (px - ctr[k, 0]) ** 2 + (py - ctr[k, 1]) ** 2
            out += amp[k] * np.exp(-r2 / (2.0 * sig[k] ** 2))
        return 0.15 * out

    return z


def folded_cloth(seed: int = 0, n: int = 256):
    """Self-intersecting cloth: bump-field height on a grid, then x > 0.5 folded onto 1 - x.

    The height is evaluated at the unfolded (x, y), so after folding the two layers hold
    different heights over the same footprint and cross along z(x,y) = z(1-x,y).
    n=256 gives 65,536 verts / 130,050 tris.
    """
    rng = np.random.default_rng(seed)
    x, tris = grid_mesh(n)
    z = _bump_field(rng)
    x[:, 2] = z(x[:, 0], x[:, 1])
    fold = x[:, 0] > 0.5
    x[fold, 0] = 1.0 - x[fold, 0]
    return _finish(x, tris)


def uv_sphere(n_lon: int, n_bands: int, radius: float = 1.0):
    """UV sphere with polar triangle fans.

    n_bands latitude bands -> (n_bands - 1) rings of n_lon vertices plus 2 poles, and
    2 * n_lon * (n_bands - 1) triangles.  (1024, 513) gives 524,290 / 1,048,576.
    """
    rings = n_bands - 1
    theta = np.pi * (np.arange(1, rings + 1) / n_bands)        # polar angle of each ring
    phi = 2.0 * np.pi * (np.arange(n_lon) / n_lon)
    st, ct = np.sin(theta)[:, None], np.cos(theta)[:, None]
    ring = np.stack([st * np.cos(phi)[None, :], st * np.sin(phi)[None, :], np.broadcast_to(ct, (rings, n_lon))], -1)
    x = np.concatenate([[[0.0, 0.0, 1.0]], ring.reshape(-1, 3), [[0.0, 0.0, -1.0]]]) * radius
    north, south = 0, 1 + rings * n_lon
    k = np.arange(n_lon)
    kn = (k + 1) % n_lon
    fans_n = np.stack([np.full(n_lon, north), 1 + k, 1 + kn], 1)
    r = np.arange(rings - 1)[:, None]
    a = 1 + r * n_lon + k[None, :]
    b = 1 + r * n_lon + kn[None, :]
    c = a + n_lon
    d = b + n_lon
    band = np.stack([np.stack([a, c, d], -1), np.stack([a, d, b], -1)], -2).reshape(-1, 3)
    last = 1 + (rings - 1) * n_lon
    fans_s = np.stack([last + k, np.full(n_lon, south), last + kn], 1)
    tris = np.concatenate([fans_n, band, fans_s])
    return _finish(x, tris)


def vector_noise(rng, n_modes: int = 64, kmin: float = 16.0, kmax: float = 32.0):
    """Band-limited vector noise N(x) = M^-1/2 sum_m c_m cos(k_m . x + phi_m), c_m ~ N(0, I3)."""
    c = rng.normal(0.0, 1.0, (n_modes, 3))
    w = rng.normal(0.0, 1.0, (n_modes, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    kappa = rng.uniform(kmin, kmax, n_modes)
    kvec = w * kappa[:, None]
    phase = rng.uniform(0.0, 2.0 * np.pi, n_modes)

    def field(x):
        out = np.zeros_like(x)
        for m in range(n_modes):
            out += np.cos(x @ kvec[m] + phase[m])[:, None] * c[m][None, :]
        return out / math.sqrt(n_modes)

    return field


def noisy_sphere(seed: int = 0, n_lon: int = 1024, n_bands: int = 513, amplitude: float = 0.05):
    """UV sphere displaced by amplitude * vector noise (folds through itself for the defaults)."""
    rng = np.random.default_rng(seed)
    x, tris = uv_sphere(n_lon, n_bands)
    x = x + amplitude * vector_noise(rng)(x)
    return _finish(x, tris)


def torus(n_v: int, R: float = 1.0, r: float = 0.4):
    """Torus with n_u = 2 n_v segments around the main ring: 2 n_u n_v triangles."""
    n_u = 2 * n_v
    u = 2.0 * np.pi * np.arange(n_u) / n_u
    v = 2.0 * np.pi * np.arange(n_v) / n_v
    U, V = np.meshgrid(u, v, indexing="ij")
    x = np.stack([(R + r * np.cos(V)) * np.cos(U), (R + r * np.cos(V)) * np.sin(U), r * np.sin(V)], -1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(n_u), np.arange(n_v), indexing="ij")
    a = i * n_v + j
    b = ((i + 1) % n_u) * n_v + j
    c = ((i + 1) % n_u) * n_v + (j + 1) % n_v
    d = i * n_v + (j + 1) % n_v
    tris = np.stack([np.stack([a, b, c], -1), np.stack([a, c, d], -1)], -2).reshape(-1, 3)
    return _finish(x, tris)


def bump_grid(rng, n: int):
    """Unfolded bump-field grid (the cloth height field without the fold)."""
    x, tris = grid_mesh(n)
    z = _bump_field(rng)
    x[:, 2] = z(x[:, 0], x[:, 1])
    return _finish(x, tris)


def _random_rotation(rng):
    q = rng.normal(0.0, 1.0, 4)
    q /= np.linalg.norm(q)
    w, a, b, c = q
    return np.array([
        [1 - 2 * (b * b + c * c), 2 * (a * b - c * w), 2 * (a * c + b * w)],
        [2 * (a * b + c * w), 1 - 2 * (a * a + c * c), 2 * (b * c - a * w)],
        [2 * (a * c - b * w), 2 * (b * c + a * w), 1 - 2 * (a * a + b * b)],
    ])


def _sized_mesh(rng, kind: int, s: float):
    if kind == 0:   # geodesic icosphere: 20 n^2 faces via a n-frequency subdivision of the icosahedron
        n = max(1, int(round(math.sqrt(s / 20.0))))
        x, t = _geodesic_icosphere(n)
    elif kind == 1:
        nv = max(3, int(round(math.sqrt(s / 4.0))))
        x, t = torus(nv)
    else:
        n = max(3, int(round(math.sqrt(s / 2.0))) + 1)
        x, t = bump_grid(rng, n)
    x = x - x.mean(0)
    x = x / np.max(np.linalg.norm(x, axis=1))
    return _finish(x, t)


def _geodesic_icosphere(freq: int):
    """Icosahedron with each face split into freq^2 triangles (class-I geodesic), projected."""
    x0, f0 = icosphere(0)
    verts: list[np.ndarray] = []
    index: dict[tuple, int] = {}

    def vid(p):
        key = tuple(np.round(p, 12))
        if key not in index:
            index[key] = len(verts)
            verts.append(p / np.linalg.norm(p))
        return index[key]

    faces = []
    for a, b, c in f0:
        A, B, C = x0[a], x0[b], x0[c]
        grid = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                p = A + (B - A) * (i / freq) + (C - A) * (j / freq)
                grid[(i, j)] = vid(p)
        for i in range(freq):
            for j in range(freq - i):
                faces.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j + 1 < freq:
                    faces.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    return _finish(np.array(verts), np.array(faces))


def batch_problems(seed: int = 0, n_problems: int = 64, smin: float = 2e3, smax: float = 2e5):
    """64 independent two-mesh problems of log-uniform size (triangles per mesh).

    Returns a list of ``(x, tris, n_tris_first)``: the union mesh of the problem and the
    number of triangles belonging to its first mesh.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_problems):
        meshes = []
        for _m in range(2):
            kind = int(rng.integers(0, 3))
            s = math.exp(rng.uniform(math.log(smin), math.log(smax)))
            meshes.append(_sized_mesh(rng, kind, s))
        (xa, ta), (xb, tb) = meshes
        rot = _random_rotation(rng)
        u = rng.normal(0.0, 1.0, 3)
        u /= np.linalg.norm(u)
        rho = rng.uniform(0.2, 0.8)
        xb = xb @ rot.T + rho * u
        x, t = union([(xa, ta), (xb, tb)])
        out.append((x, t, len(ta)))
    return out


def crumpled_fans(seed: int = 0, n_fans: int = 8, blades: int = 16, height: float = 0.3):
    """An n_fans x n_fans grid of fans: each a centre vertex and a ring of ``blades`` vertices at
    radius 0.5 with random heights N(0, height^2), triangulated around the centre, the ring
    winding twice around it.  Blades of the two windings lie over each other and share only
    the centre vertex: where their heights interleave they cross, giving intersecting pairs
    that share exactly one vertex."""
    rng = np.random.default_rng(seed)
    xs, ts = [], []
    off = 0
    for gx in range(n_fans):
        for gy in range(n_fans):
            c = np.array([gx * 1.2, gy * 1.2, 0.0])
            th = 4 * np.pi * np.arange(blades) / blades
            ring = np.stack([c[0] + 0.5 * np.cos(th), c[1] + 0.5 * np.sin(th), rng.normal(0.0, height, blades)], 1)
            xs.append(np.vstack([c, ring]))
            k = np.arange(blades)
            ts.append(np.stack([np.zeros(blades, np.int64), 1 + k, 1 + (k + 1) % blades], 1) + off)
            off += blades + 1
    return _finish(np.concatenate(xs), np.concatenate(ts))


# integer frames (origin, two spanning vectors) of the planes of ``coplanar_soup``: every point
# origin + u e1 + v e2 with small integers u, v is exactly representable, so triangles on one
# plane are exactly coplanar; the planes lean on different coordinate axes
_SOUP_PLANES = (
    ((0, 0, 0), (1, 0, 0), (0, 1, 0)),     # z = 0
    ((0, 0, -4), (1, 0, 1), (0, 1, 0)),    # x - z = 4
    ((0, -3, 0), (1, 2, 0), (0, 1, 3)),
    ((2, 0, 1), (0, 1, 2), (3, 0, -1)),
)


def coplanar_soup(seed: int = 0, n_tris: int = 4000, grid: int = 64, span: int = 3, planes: int = 4):
    """Separate triangles (three vertices each) on a few exactly representable planes that
    cross each other.  A triangle's (u, v) corners are a base point in [0, grid - span]^2 plus
    integer offsets in [0, span]^2, so triangles on one plane are exactly coplanar and often
    overlap, touch along edges or at vertices, or have no area; triangles on different planes
    cross."""
    rng = np.random.default_rng(seed)
    pl = rng.integers(0, planes, n_tris)
    base = rng.integers(0, grid - span + 1, (n_tris, 1, 2))
    uv = base + rng.integers(0, span + 1, (n_tris, 3, 2))
    frames = np.asarray(_SOUP_PLANES[:planes], np.float64)  # (planes, 3 rows, 3)
    o, e1, e2 = frames[pl, 0], frames[pl, 1], frames[pl, 2]
    x = o[:, None, :] + uv[..., :1] * e1[:, None, :] + uv[..., 1:] * e2[:, None, :]
    return _finish(x.reshape(-1, 3), np.arange(3 * n_tris).reshape(-1, 3))


def concat_problems(problems):
    """One batched mesh from independent problems ``(x, tris, ...)``: the vertices and
    triangles concatenated (triangle indices re-based to global vertex ids) and the offsets
    ``vert_off``, ``tri_off`` (int64, n + 1) of each problem's ranges."""
    xs, ts = [], []
    vert_off, tri_off = [0], [0]
    for prob in problems:
        x, t = prob[0], prob[1]
        xs.append(x)
        ts.append(t + vert_off[-1])
        vert_off.append(vert_off[-1] + len(x))
        tri_off.append(tri_off[-1] + len(t))
    x, t = _finish(np.concatenate(xs), np.concatenate(ts))
    return x, t, np.asarray(vert_off, np.int64), np.asarray(tri_off, np.int64)


def integer_grid_triangles(seed: int, n: int, lo: int = -3, hi: int = 3):
    """n random triangles with integer vertices in {lo..hi}^3, each on its own 3 vertices.

    Dense in exact degeneracies (coplanar, touching, vertex-on-plane, collinear), which is
    what exact predicates must get right.
    """
    rng = np.random.default_rng(seed)
    x = rng.integers(lo, hi + 1, size=(3 * n, 3)).astype(np.float64)
    tris = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    return _finish(x, tris)


def submesh_near(x, tris, point, n_tris: int):
    """The n_tris triangles whose centroids are nearest to ``point`` (ties by index), with
    their vertices re-indexed in order of first appearance."""
    cent = x[tris].mean(axis=1)
    d2 = np.sum((cent - np.asarray(point, dtype=np.float64)) ** 2, axis=1)
    order = np.lexsort((np.arange(len(tris)), d2))[:n_tris]
    sel = tris[np.sort(order)]
    flat = sel.ravel()
    _, first = np.unique(flat, return_index=True)
    old_ids = flat[np.sort(first)]
    remap = np.full(len(x), -1, dtype=np.int64)
    remap[old_ids] = np.arange(len(old_ids))
    return _finish(x[old_ids], remap[sel])
