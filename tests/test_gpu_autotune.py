"""Launch parameters: range checks, results identical bit for bit under every value, and the
autotuner over them."""

import numpy as np
import pytest
import torch

import oracle
from paper_2606_06511_amd import workloads

pytestmark = pytest.mark.gpu


def _ctx(nv, nt):
    from paper_2606_06511_amd import ttie

    c = ttie.Context(0)
    c.reserve(nv, nt, 1 << 21, max_hits=1 << 14, max_blocks=36 << 14)
    return c


def test_param_range_and_defaults():
    from paper_2606_06511_amd import ttie

    c = _ctx(100, 100)
    assert [c.get_param(p) for p in range(5)] == [4096, 2048, 128, 64, 0]
    c.set_param(ttie.PARAM_TRAV_BUDGET, 32)
    assert c.get_param(ttie.PARAM_TRAV_BUDGET) == 32
    c.set_param(ttie.PARAM_TRAV_BUDGET, 0)
    assert c.get_param(ttie.PARAM_TRAV_BUDGET) == 128
    for p, bad in ((ttie.PARAM_SCREEN_BLOCKS, 1), (ttie.PARAM_ROW_BLOCKS, 1 << 20), (ttie.PARAM_TRAV_BUDGET, 8),
                   (ttie.PARAM_SCREEN_TILE, 32), (ttie.PARAM_SCREEN_TILE, 100), (ttie.PARAM_SCREEN_TILE, 1 << 21)):
        with pytest.raises(ttie.TTIEError):
            c.set_param(p, bad)
    with pytest.raises(ttie.TTIEError):
        c.set_param(7, 100)


@pytest.mark.parametrize("which", ["cloth", "sphere_small"])
def test_results_do_not_depend_on_params(which):
    from paper_2606_06511_amd import ttie

    if which == "cloth":
        x, tris = workloads.folded_cloth(1, n=128)
    else:
        x, tris = workloads.noisy_sphere(1, n_lon=128, n_bands=65)
    c = _ctx(len(x), len(tris))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tris).cuda()
    settings = [{}, {ttie.PARAM_SCREEN_BLOCKS: 64, ttie.PARAM_ROW_BLOCKS: 64, ttie.PARAM_TRAV_BUDGET: 16,
                     ttie.PARAM_HASH_BUDGET: 16},
                {ttie.PARAM_SCREEN_BLOCKS: 65536, ttie.PARAM_ROW_BLOCKS: 65536, ttie.PARAM_TRAV_BUDGET: 1 << 20,
                 ttie.PARAM_HASH_BUDGET: 1 << 20},
                # the screening's tile queue: tiles of one batch, of many, and one tile for all
                {ttie.PARAM_SCREEN_TILE: 64, ttie.PARAM_SCREEN_BLOCKS: 64},
                {ttie.PARAM_SCREEN_TILE: 1024},
                {ttie.PARAM_SCREEN_TILE: 1 << 20, ttie.PARAM_SCREEN_BLOCKS: 65536}]
    ref = None
    for st in settings:
        for p in range(5):
            c.set_param(p, st.get(p, 0))
        res = []
        for method in (ttie.BROAD_LBVH, ttie.BROAD_HASH):
            pairs, n = c.broadphase(xd, td, method)
            c.check()
            p_ = pairs[: int(n.item())].cpu().numpy()
            key = p_[:, 0].astype(np.int64) << 32 | p_[:, 1]
            res.append(p_[np.argsort(key)].tobytes())
        out = c.evaluate(xd, td, pairs, n, precision=ttie.MIXED)
        c.check()
        nb = int(out["n_blocks"].item())
        res += [out["energy"].cpu().numpy().tobytes(), out["grad"].cpu().numpy().tobytes(),
                out["row_ptr"].cpu().numpy().tobytes(), out["col_idx"][:nb].cpu().numpy().tobytes(),
                out["vals"][:nb].cpu().numpy().tobytes()]
        if ref is None:
            ref = res
            assert res[0] == res[1]  # both broad phases give the same set
        assert res == ref, st


@pytest.mark.parametrize("budget", [16, 24])
def test_low_budgets_full_cloth(budget):
    """At low traversal budgets most deferred work is many short searches, which the
    wave-cooperative kernel takes in batches of up to 32 queries per wave (budget 16 defers
    about 24,000 queries on the full cloth: about 24 per wave)."""
    from paper_2606_06511_amd import ttie

    x, tris = workloads.folded_cloth(0)
    c = _ctx(len(x), len(tris))
    c.set_param(ttie.PARAM_TRAV_BUDGET, budget)
    pairs, n = c.broadphase(torch.from_numpy(x).cuda(), torch.from_numpy(tris).cuda(), ttie.BROAD_LBVH)
    c.check()
    got = pairs[: int(n.item())].cpu().numpy()
    np.testing.assert_array_equal(got[np.lexsort((got[:, 1], got[:, 0]))], oracle.pairs(x, tris))


def test_autotune_picks_valid_values():
    from paper_2606_06511_amd import autotune, ttie

    x, tris = workloads.folded_cloth(0, n=96)
    c = _ctx(len(x), len(tris))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tris).cuda()
    pairs = torch.empty((1 << 21, 2), dtype=torch.int32, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = c.evaluate(xd, td, pairs[:1], torch.zeros(1, dtype=torch.int64, device="cuda"), precision=ttie.MIXED)

    def step():
        c.broadphase(xd, td, ttie.BROAD_LBVH, out=(pairs, n))
        c.evaluate(xd, td, pairs, n, precision=ttie.MIXED, out=out)

    best, ms, ms0 = autotune.tune(c, step, reps=3, rounds=1)
    for name, (pid, values) in autotune.SPACE.items():
        assert best[name] in values and c.get_param(pid) == best[name]
    assert ms > 0 and ms0 > 0
    c.check()
