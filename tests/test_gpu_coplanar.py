"""Coplanar pairs through the C ABI against the oracle: per-pair flags bit-exact (status 4 where
the interiors of two triangles in one plane overlap), with the energy, gradient and Hessian
of the crossing pairs alongside, on integer-grid triangle soups where exact contacts abound."""

import numpy as np
import pytest
import torch

import oracle
import parity_checks as pc
from paper_2606_06511_amd import workloads

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    from paper_2606_06511_amd import ttie

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = ttie.Context(0)
    c.reserve(200_000, 60_000, 1 << 21, max_hits=1 << 18, max_blocks=1 << 21)
    return c


def _dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _sorted_pairs(pairs, n):
    p = pairs[: int(n.item())].cpu().numpy()
    key = p[:, 0].astype(np.int64) << 32 | p[:, 1].astype(np.int64)
    return p[np.argsort(key)]


@pytest.fixture(scope="module")
def soup():
    # 20,000 separate triangles on four crossing planes, small corners on a 64 x 64 integer grid
    x, tris = workloads.coplanar_soup(0, n_tris=20_000)
    pairs = oracle.pairs(x, tris)
    return x, tris, pairs, pc.reference(x, tris, pairs)


@pytest.mark.parametrize("method", [1, 2])
def test_soup_candidates(ctx, soup, method):
    x, tris, ref, _ = soup
    pairs, n = ctx.broadphase(_dev(x, torch.float64), _dev(tris, torch.int32), method)
    ctx.check()
    np.testing.assert_array_equal(_sorted_pairs(pairs, n), ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_soup_flags_and_energy(ctx, soup, precision):
    from paper_2606_06511_amd import ttie

    x, tris, pairs, ref = soup
    assert np.sum(ref["flags"] == ttie.PAIR_COPLANAR) > 10_000
    assert len(ref["hit_pair"]) > 500
    out = ctx.evaluate(_dev(x, torch.float64), _dev(tris, torch.int32), _dev(pairs, torch.int32),
                       precision=precision, flags=True, pair_T=True)
    ctx.check()
    assert np.all(out["pair_T"].cpu().numpy()[ref["flags"] == ttie.PAIR_COPLANAR] == 0.0)
    pc.check_eval_outputs(out, ref, pairs, tris, precision, what="coplanar soup")
    pc.check_hits(ctx.hits(1 << 18), ref, pairs, precision, what="coplanar soup")


@pytest.mark.parametrize("plane", range(4))
def test_same_plane_pairs(ctx, plane):
    """Pairs (2k, 2k+1) of small-grid triangles on one plane: every contact kind appears
    (overlap, shared edge line, vertex contact, no area)."""
    rng = np.random.default_rng(40 + plane)
    n = 4000
    uv = rng.integers(0, 5, (2 * n, 3, 2)).astype(np.float64)
    o, e1, e2 = np.asarray(workloads._SOUP_PLANES[plane], np.float64)
    x = (o + uv[..., :1] * e1 + uv[..., 1:] * e2).reshape(-1, 3)
    tris = np.arange(len(x), dtype=np.int32).reshape(-1, 3)
    pairs = np.arange(len(tris), dtype=np.int32).reshape(-1, 2)
    ref = pc.reference(x, tris, pairs)
    out = ctx.evaluate(_dev(x, torch.float64), _dev(tris, torch.int32), _dev(pairs, torch.int32), flags=True)
    ctx.check()
    got = out["flags"].cpu().numpy()
    np.testing.assert_array_equal(got, ref["flags"])
    assert 0.2 * n < np.sum(got == 4) < 0.8 * n
    assert out["energy"].item() == 0.0


def test_flat_fans_with_vertex_adjacent_pairs(ctx):
    """Fans flattened into the plane z = 0: the two windings' blades coincide and share only
    the centre vertex, so with the vertex-adjacent option they are coplanar overlaps."""
    from paper_2606_06511_amd import ttie

    x, tris = workloads.crumpled_fans(0, n_fans=6, height=0.0)
    pairs = oracle.pairs(x, tris, vertex_adjacent=True)
    ref = pc.reference(x, tris, pairs, vertex_adjacent=True)
    assert np.sum(ref["flags"] == ttie.PAIR_COPLANAR) >= 36 * 8
    xd, td = _dev(x, torch.float64), _dev(tris, torch.int32)
    out = ctx.evaluate(xd, td, _dev(pairs, torch.int32), flags=True, vertex_adjacent=True)
    ctx.check()
    np.testing.assert_array_equal(out["flags"].cpu().numpy(), ref["flags"])
    assert out["energy"].item() == 0.0 == ref["E"]
