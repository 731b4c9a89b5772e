"""Parity at the full sizes of the larger workloads, in the launch configuration the benchmark
times: the 4,194,304-triangle noisy sphere (candidates, flags, energy, gradient, every hit and
the BSR Hessian, mixed and FP64) and the batch of 64 two-mesh problems (5,664,096 triangles:
batched candidates, every problem's energy, the gradient, every hit and the BSR Hessian), all
element by element (tests/parity_checks.py)."""

import numpy as np
import pytest
import torch

import oracle
import parity_checks as pc
from paper_2606_06511_amd import workloads

pytestmark = pytest.mark.gpu


def _sorted(p):
    key = p[:, 0].astype(np.int64) << 32 | p[:, 1].astype(np.int64)
    return p[np.argsort(key)]


@pytest.fixture(scope="module")
def sphere4m():
    x, tris = workloads.noisy_sphere(seed=0, n_lon=2048, n_bands=1025)
    assert len(tris) == 4_194_304
    pairs = oracle.pairs(x, tris)
    return x, tris, pairs, pc.reference(x, tris, pairs, hessian=True)


@pytest.mark.parametrize("precision", [1, 0])
def test_sphere_4m(sphere4m, precision):
    from paper_2606_06511_amd import ttie

    x, tris, ref_pairs, ref = sphere4m
    ctx = ttie.Context(0)
    ctx.reserve(len(x), len(tris), 1 << 25, max_hits=1 << 17, max_blocks=36 << 17)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tris).cuda()
    pairs, n = ctx.broadphase(xd, td, ttie.BROAD_LBVH)
    ctx.check()
    got = pairs[: int(n.item())].cpu().numpy()
    assert len(got) == len(ref_pairs) == 16_296_621
    np.testing.assert_array_equal(_sorted(got), ref_pairs)
    # the evaluation of the list in the broad phase's own (unsorted) order, as the benchmark runs it
    out = ctx.evaluate(xd, td, pairs, n, precision=precision, hessian=True, flags=True)
    ctx.check()
    order = np.lexsort((got[:, 1], got[:, 0]))
    np.testing.assert_array_equal(out["flags"][: len(got)].cpu().numpy()[order], ref["flags"])
    assert int(out["n_hits"].item()) == len(ref["hit_pair"]) == 26_800
    pc.check_eval_outputs(out, ref, ref_pairs, tris, precision, flags=False, what="4M sphere")
    pc.check_hits(ctx.hits(1 << 17), ref, ref_pairs, precision, what="4M sphere")


def test_batch64():
    from paper_2606_06511_amd import ttie

    probs = workloads.batch_problems(seed=0)
    assert len(probs) == 64
    x, tris, vert_off, tri_off = workloads.concat_problems(probs)
    assert len(tris) == 5_664_096
    ctx = ttie.Context(0)
    ctx.reserve(len(x), len(tris), 1 << 22, max_hits=1 << 17, max_blocks=36 << 17)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tris).cuda()
    pairs, n = ctx.batch_broadphase(xd, td, torch.from_numpy(tri_off).cuda())
    out = ctx.batch_evaluate(xd, td, torch.from_numpy(vert_off).cuda(), pairs, n, precision=ttie.MIXED)
    ctx.check()
    got = _sorted(pairs[: int(n.item())].cpu().numpy())
    ref_pairs, refs, hits = [], [], 0
    for p, (xp, tp, _) in enumerate(probs):
        pp = oracle.pairs(xp, tp)
        ref_pairs.append(pp + tri_off[p])
        r = oracle.evaluate(xp, tp, pp, hessian=False)
        refs.append(r)
        hits += len(r["hit_pair"])
    ref_pairs = np.concatenate(ref_pairs)
    np.testing.assert_array_equal(got, ref_pairs)
    assert int(out["n_hits"].item()) == hits
    E = out["energies"].cpu().numpy()
    for p, r in enumerate(refs):
        pc.check_energy(E[p], r, f"problem {p} energy")
    # gradient, every hit and the Hessian against the oracle on the concatenated mesh with the
    # batch's candidates (no pair joins two problems, so that is exactly the batch's answer)
    ref = pc.reference(x, tris, ref_pairs, hessian=True)
    pc.check_eval_outputs(out, ref, ref_pairs, tris, ttie.MIXED, flags=False, what="batch of 64")
    pc.check_hits(ctx.hits(1 << 17), ref, ref_pairs, ttie.MIXED, what="batch of 64")
