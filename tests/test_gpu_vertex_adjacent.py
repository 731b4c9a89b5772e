"""Pairs sharing exactly one vertex, through the C ABI, against the oracle with the same option.

The paper treats every pair with a shared vertex as adjacent and skips it.  With the option,
a pair sharing one vertex is a candidate and is evaluated; pairs sharing an edge stay
adjacent.  The fans of ``crumpled_fans`` have blades that share only their centre vertex and
cross each other, so the option changes both the candidate set and the energy.
"""

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
    c.reserve(200_000, 200_000, 1 << 21, max_hits=1 << 16, max_blocks=1 << 20)
    return c


@pytest.fixture(scope="module")
def fans():
    # 24 x 24 fans of 16 blades: 9,216 triangles, about 2,400 crossing pairs sharing a vertex
    x, tris = workloads.crumpled_fans(1, n_fans=24)
    return x, tris, oracle.pairs(x, tris, vertex_adjacent=True)


def _dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _sorted_pairs(pairs, n):
    p = pairs[: int(n.item())].cpu().numpy()
    key = p[:, 0].astype(np.int64) << 32 | p[:, 1].astype(np.int64)
    return p[np.argsort(key)]


def _shares_one_vertex(tris, pairs):
    a, b = tris[pairs[:, 0]], tris[pairs[:, 1]]
    return (a[:, :, None] == b[:, None, :]).any(2).sum(1) == 1


@pytest.mark.parametrize("method", ["lbvh", "hash"])
def test_pairs_match_oracle(ctx, fans, method):
    from paper_2606_06511_amd import ttie

    x, tris, ref = fans
    m = {"lbvh": ttie.BROAD_LBVH, "hash": ttie.BROAD_HASH}[method]
    xd, td = _dev(x, torch.float64), _dev(tris, torch.int32)
    pairs, n = ctx.broadphase(xd, td, m, vertex_adjacent=True)
    ctx.check()
    np.testing.assert_array_equal(_sorted_pairs(pairs, n), ref)
    assert _shares_one_vertex(tris, ref).sum() > 0
    # without the option the same call lists exactly the pairs with no shared vertex
    pairs0, n0 = ctx.broadphase(xd, td, m)
    ctx.check()
    np.testing.assert_array_equal(_sorted_pairs(pairs0, n0), ref[~_shares_one_vertex(tris, ref)])


def test_brute_force_pairs(ctx):
    """All pairs with at most one shared vertex (no box test), 8 x 8 fans: 1,024 triangles."""
    from paper_2606_06511_amd import ttie

    x, tris = workloads.crumpled_fans(2, n_fans=8)
    ref = oracle.pairs(x, tris, oracle.BROAD_BRUTE, vertex_adjacent=True)
    xd, td = _dev(x, torch.float64), _dev(tris, torch.int32)
    pairs, n = ctx.broadphase(xd, td, ttie.BROAD_BRUTE, vertex_adjacent=True)
    ctx.check()
    np.testing.assert_array_equal(_sorted_pairs(pairs, n), ref)
    shared = (tris[ref[:, 0]][:, :, None] == tris[ref[:, 1]][:, None, :]).any(2).sum(1)
    assert shared.max() == 1 and (shared == 1).sum() == 64 * (16 * 15 // 2 - 16)


def test_pairs_on_a_grid_mesh(ctx):
    """A cloth grid: every interior vertex is shared by six triangles, so the option adds many
    touching pairs; the lists must still agree pair for pair."""
    from paper_2606_06511_amd import ttie

    x, tris = workloads.folded_cloth(0, n=64)
    ref = oracle.pairs(x, tris, vertex_adjacent=True)
    xd, td = _dev(x, torch.float64), _dev(tris, torch.int32)
    for m in (ttie.BROAD_LBVH, ttie.BROAD_HASH):
        pairs, n = ctx.broadphase(xd, td, m, vertex_adjacent=True)
        ctx.check()
        np.testing.assert_array_equal(_sorted_pairs(pairs, n), ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_eval_matches_oracle(ctx, fans, precision):
    from paper_2606_06511_amd import ttie

    x, tris, pairs = fans
    ref = pc.reference(x, tris, pairs, vertex_adjacent=True)
    assert ref["E"] > 0 and len(ref["hit_pair"]) > 1000
    xd, td, pd = _dev(x, torch.float64), _dev(tris, torch.int32), _dev(pairs, torch.int32)
    out = ctx.evaluate(xd, td, pd, precision=precision, flags=True, pair_T=True, vertex_adjacent=True)
    ctx.check()
    pc.check_eval_outputs(out, ref, pairs, tris, precision, what="fans")
    pc.check_hits(ctx.hits(), ref, pairs, precision, what="fans")
    # every hit of this mesh shares the centre vertex of its fan
    assert _shares_one_vertex(tris, pairs[ref["hit_pair"]]).all()
    # the default evaluation of the same list flags them adjacent: no energy
    out0 = ctx.evaluate(xd, td, pd, precision=precision, flags=True)
    ctx.check()
    ref0 = oracle.evaluate(x, tris, pairs)
    np.testing.assert_array_equal(out0["flags"].cpu().numpy(), ref0["flags"])
    assert out0["energy"].item() == 0.0 and ref0["E"] == 0.0


def test_eval_grid_mesh_touching_pairs(ctx):
    """Grid triangles that share a vertex only touch there: both sides report no hit for them,
    and the energy equals the default one (the folded cloth's crossings share no vertex)."""
    from paper_2606_06511_amd import ttie

    x, tris = workloads.folded_cloth(0, n=64)
    pairs = oracle.pairs(x, tris, vertex_adjacent=True)
    ref = pc.reference(x, tris, pairs, vertex_adjacent=True)
    xd, td, pd = _dev(x, torch.float64), _dev(tris, torch.int32), _dev(pairs, torch.int32)
    out = ctx.evaluate(xd, td, pd, precision=ttie.FP64, flags=True, vertex_adjacent=True)
    ctx.check()
    pc.check_eval_outputs(out, ref, pairs, tris, ttie.FP64, what="grid with touching pairs")


def test_eval_deterministic(ctx, fans):
    """A hit sharing a vertex holds that vertex twice in its row; the assembly still sums in a
    fixed order, so two evaluations agree bit for bit."""
    x, tris, _ = fans
    xd, td = _dev(x, torch.float64), _dev(tris, torch.int32)
    res = []
    for _ in range(2):
        pairs, n = ctx.broadphase(xd, td, vertex_adjacent=True)
        out = ctx.evaluate(xd, td, pairs, n, vertex_adjacent=True)
        ctx.check()
        nb = int(out["n_blocks"].item())
        res.append((out["energy"].cpu().numpy().tobytes(), out["grad"].cpu().numpy().tobytes(),
                    out["vals"][:nb].cpu().numpy().tobytes(), out["col_idx"][:nb].cpu().numpy().tobytes()))
    assert res[0] == res[1]


@pytest.mark.parametrize("precision", [0, 1])
def test_hvp_matches_oracle(ctx, fans, precision):
    from paper_2606_06511_amd import ttie

    x, tris, pairs = fans
    xd, td, pd = _dev(x, torch.float64), _dev(tris, torch.int32), _dev(pairs, torch.int32)
    out = ctx.evaluate(xd, td, pd, precision=precision, vertex_adjacent=True)
    ctx.check()
    rng = np.random.default_rng(3)
    v = rng.normal(size=x.shape)
    v /= np.linalg.norm(v)
    dt = torch.float64 if precision == 0 else torch.float32
    hv = ctx.hvp(xd, td, _dev(v, dt), ttie.HVP_EXACT).cpu().numpy()
    pc.check_vector(hv, oracle.hvp(x, tris, pairs, v, exact=True, vertex_adjacent=True),
                    pc.hvp_row_scales(x, tris, pairs, v, True, vertex_adjacent=True), precision, "exact HVP")
    refp = oracle.hvp(x, tris, pairs, v, exact=False, vertex_adjacent=True)
    scalep = pc.hvp_row_scales(x, tris, pairs, v, False, vertex_adjacent=True)
    hp = ctx.hvp(xd, td, _dev(v, dt), ttie.HVP_PSD).cpu().numpy()
    pc.check_vector(hp, refp, scalep, precision, "PSD HVP")
    y = ctx.bsr_mv(out["row_ptr"], out["col_idx"], out["vals"], _dev(v, dt)).cpu().numpy()
    pc.check_vector(y, refp, scalep, precision, "BSR matvec")


def test_batch_eval_with_option(ctx):
    """Two fan meshes as one batch: per-problem energies equal the oracle's with the option."""
    probs = [workloads.crumpled_fans(s, n_fans=6) for s in (4, 5)]
    x, tris, vert_off, tri_off = workloads.concat_problems(probs)
    ref_pairs, E_ref = [], []
    for p, (xp, tp) in enumerate(probs):
        pp = oracle.pairs(xp, tp, vertex_adjacent=True)
        ref_pairs.append(pp + tri_off[p])
        E_ref.append(oracle.evaluate(xp, tp, pp, vertex_adjacent=True)["E"])
    pairs = np.concatenate(ref_pairs).astype(np.int32)
    out = ctx.batch_evaluate(_dev(x, torch.float64), _dev(tris, torch.int32), _dev(vert_off), _dev(pairs),
                             vertex_adjacent=True)
    ctx.check()
    np.testing.assert_allclose(out["energies"].cpu().numpy(), E_ref, rtol=1e-10)
    assert min(E_ref) > 0


def test_unknown_flags_are_rejected(ctx):
    from paper_2606_06511_amd import ttie

    x, tris = workloads.crumpled_fans(0, n_fans=2)
    xd, td = _dev(x, torch.float64), _dev(tris, torch.int32)
    with pytest.raises(ttie.TTIEError):
        ctx.broadphase(xd, td, ttie.BROAD_LBVH | 0x200)
    pairs = _dev(np.array([[0, 1]], np.int32))
    m = ctx._mesh(xd, td)
    opts = ttie.Options(ttie.FP64, ttie.PSD_PER_PART, ttie.INTERVAL_EQ1, 2)
    out = ctx.evaluate(xd, td, pairs)  # buffers
    import ctypes

    n = _dev(np.array([1], np.int64))
    st = ttie.lib().ttie_eval(ctx.handle, ctypes.byref(m), ttie._ptr(pairs), ttie._ptr(n), 1, ctypes.byref(opts),
                              ttie._ptr(out["energy"]), ttie._ptr(out["grad"]), None, None, None, None, None, 0,
                              None, ttie._ptr(out["n_hits"]), ttie._stream())
    assert st == 1  # invalid argument
