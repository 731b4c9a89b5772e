"""Sizes at the tile edges of the library's scans.  The exclusive scan of int32 counts works in
tiles of 2048 entries: in one launch with a look-back below 256 tiles, in three launches (tile
sums, their scan, each tile from its prefix) from 256 tiles on.  The springs pattern scans
N_v + 1 vertex degrees and N_v + 1 row counts, so it is checked at N_v + 1 just below, at and
above tile edges, past 64 tiles (the look-back window) and on both sides of 256 tiles.  The
evaluation's own row ranks scan the touched-vertex bitmap in blocks of 1024 words (32,768
vertices): a small folded cloth spread over N_v vertex slots, the rest unused, is evaluated at
the same sizes.  Candidates, flags, energy, gradient and the BSR matrix against the oracle; the
row pointers bit-exact."""

import numpy as np
import pytest
import torch

import oracle
import parity_checks as pc
from paper_2606_06511_amd import workloads

pytestmark = pytest.mark.gpu

TILE = 2048


@pytest.fixture(scope="module")
def ctx():
    from paper_2606_06511_amd import ttie

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = ttie.Context(0)
    c.reserve(300 * TILE, 4096, 1 << 18, max_hits=1 << 14, max_blocks=1 << 19)
    return c


def spread_cloth(nv, seed):
    """The 40 x 40 folded cloth with its vertices at random slots of [0, nv); the unused
    slots hold points far from it, so they touch nothing."""
    x0, tris0 = workloads.folded_cloth(seed=seed, n=40)
    rng = np.random.default_rng(seed)
    slot = np.sort(rng.choice(nv, size=len(x0), replace=False))
    x = 10.0 + rng.random((nv, 3))
    x[slot] = x0
    return x, slot[tris0].astype(np.int32)


@pytest.mark.parametrize("nv", [TILE - 2, TILE - 1, TILE, 2 * TILE - 1, 64 * TILE - 1, 64 * TILE, 65 * TILE + 5])
def test_scan_tile_edges(ctx, nv):
    from paper_2606_06511_amd import ttie

    x, tris = spread_cloth(nv, seed=nv % 7)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tris).cuda()
    pairs, n = ctx.broadphase(xd, td, ttie.BROAD_LBVH)
    ctx.check()
    got = pairs[: int(n.item())].cpu().numpy()
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    ref_pairs = oracle.pairs(x, tris)
    np.testing.assert_array_equal(got, ref_pairs)
    ref = pc.reference(x, tris, ref_pairs)
    assert len(ref["hit_pair"]) > 0
    out = ctx.evaluate(xd, td, torch.from_numpy(ref_pairs).cuda(), precision=ttie.FP64, flags=True)
    ctx.check()
    pc.check_eval_outputs(out, ref, ref_pairs, tris, ttie.FP64, what=f"n_v = {nv}")


@pytest.mark.parametrize("nv", [TILE - 1, 64 * TILE, 255 * TILE - 1, 255 * TILE, 256 * TILE - 1, 256 * TILE,
                                299 * TILE + 5])
def test_scan_forms_through_the_springs_pattern(ctx, nv):
    """Both scan forms and the switch between them (255 and 256 tiles of N_v + 1 counts): the
    springs pattern of the spread cloth against the oracle's, bit for bit."""
    from oracle import quasistatic as qs

    x, tris = spread_cloth(nv, seed=nv % 5)
    rp, ci = ctx.springs_pattern(torch.from_numpy(tris).cuda(), nv)
    ctx.check()
    edges = qs.spring_edges(tris)
    rp_ref, ci_ref, _ = qs.stiffness_bsr(nv, edges, np.zeros((len(edges), 3, 3)), 0.0)
    np.testing.assert_array_equal(rp.cpu().numpy(), rp_ref)
    np.testing.assert_array_equal(ci.cpu().numpy(), ci_ref)
