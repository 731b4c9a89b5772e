"""Parity at the full sizes of the larger workloads, in the launch configuration the benchmark
times: the 4,194,304-triangle noisy sphere (candidates, flags, energy and gradient, mixed and
FP64) and the batch of 64 two-mesh problems (5,664,096 triangles: batched candidates and the
energy of every problem)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2606_06511_amd import workloads

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _sorted(p):
    key = p[:, 0].astype(np.int64) << 32 | p[:, 1].astype(np.int64)
    return p[np.argsort(key)]


@pytest.fixture(scope="module")
def sphere4m():
    x, tris = workloads.noisy_sphere(seed=0, n_lon=2048, n_bands=1025)
    assert len(tris) == 4_194_304
    pairs = oracle.pairs(x, tris)
    return x, tris, pairs, oracle.evaluate(x, tris, pairs, hessian=False)


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
    assert abs(out["energy"].item() - ref["E"]) <= 1e-10 * ref["E"]
    assert _rel(out["grad"].cpu().numpy(), ref["G"]) <= (1e-10 if precision == 0 else 1e-4)
    assert int(out["n_blocks"].item()) > 0


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
    ref_pairs, E_ref, hits = [], [], 0
    for p, (xp, tp, _) in enumerate(probs):
        pp = oracle.pairs(xp, tp)
        ref_pairs.append(pp + tri_off[p])
        r = oracle.evaluate(xp, tp, pp, hessian=False)
        E_ref.append(r["E"])
        hits += len(r["hit_pair"])
    np.testing.assert_array_equal(got, np.concatenate(ref_pairs))
    assert int(out["n_hits"].item()) == hits
    np.testing.assert_allclose(out["energies"].cpu().numpy(), E_ref, rtol=1e-10)
