"""Batches of independent problems through the C ABI: the batched broad phase against the
per-problem oracle candidate sets, batched evaluation against the per-problem oracle and
against separate calls, offset validation, and the batched step replayed from a HIP graph."""

import numpy as np
import pytest
import torch

import oracle
import parity_checks as pc
from paper_2606_06511_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    # 12 two-mesh problems (icospheres, tori, bump grids) of 500 to 20,000 triangles per mesh
    probs = workloads.batch_problems(seed=1, n_problems=12, smin=500, smax=2e4)
    x, tris, vert_off, tri_off = workloads.concat_problems(probs)
    ref_pairs, refs = [], []
    for p, (xp, tp, _) in enumerate(probs):
        pp = oracle.pairs(xp, tp)
        ref_pairs.append(pp + tri_off[p])
        refs.append(oracle.evaluate(xp, tp, pp, hessian=True))
    return probs, x, tris, vert_off, tri_off, np.concatenate(ref_pairs), refs


@pytest.fixture(scope="module")
def ctx(batch):
    from paper_2606_06511_amd import ttie

    _, x, tris, _, _, _, _ = batch
    c = ttie.Context(0)
    c.reserve(len(x), len(tris), 1 << 21, max_hits=1 << 16, max_blocks=36 << 16)
    return c


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _expected_bsr(refs, vert_off):
    rp, ci, va = [np.zeros(1, np.int64)], [], []
    for p, r in enumerate(refs):
        rp.append(r["row_ptr"][1:].astype(np.int64) + rp[-1][-1])
        ci.append(r["col_idx"].astype(np.int64) + vert_off[p])
        va.append(r["vals"])
    return np.concatenate(rp), np.concatenate(ci), np.concatenate(va)


def test_batch_pairs_match_per_problem_oracle(batch, ctx):
    _, x, tris, _, tri_off, ref_pairs, _ = batch
    pairs, n = ctx.batch_broadphase(_dev(x), _dev(tris), _dev(tri_off))
    ctx.check()
    got = pairs[: int(n.item())].cpu().numpy()
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    np.testing.assert_array_equal(got, ref_pairs)
    # the same mesh without the batch split does find pairs across problems
    p1, n1 = ctx.broadphase(_dev(x), _dev(tris))
    ctx.check()
    assert int(n1.item()) > len(ref_pairs)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_eval_matches_oracle(batch, ctx, precision):
    """Every output element by element against the oracle on the concatenated mesh with the
    batch's candidates (no pair joins two problems, so that is exactly the batch's answer), and
    every problem's energy against the oracle on that problem alone."""
    _, x, tris, vert_off, tri_off, ref_pairs, refs = batch
    xd, td = _dev(x), _dev(tris)
    pairs, n = ctx.batch_broadphase(xd, td, _dev(tri_off))
    out = ctx.batch_evaluate(xd, td, _dev(vert_off), pairs, n, precision=precision)
    ctx.check()
    E = out["energies"].cpu().numpy()
    assert all(r["E"] > 0 for r in refs)
    for p, r in enumerate(refs):
        pc.check_energy(E[p], r, f"problem {p} energy")  # T is float64 on both paths
    ref = pc.reference(x, tris, ref_pairs)
    pc.check_eval_outputs(out, ref, ref_pairs, tris, precision, flags=False, what="batch")
    pc.check_hits(ctx.hits(), ref, ref_pairs, precision, what="batch")
    # the batch's Hessian is block diagonal: problem by problem, the oracle's own matrices
    rp, ci, va = _expected_bsr(refs, vert_off)
    np.testing.assert_array_equal(ref["row_ptr"], rp)
    np.testing.assert_array_equal(ref["col_idx"], ci)


def test_batch_equals_separate_calls(batch, ctx):
    probs, x, tris, vert_off, tri_off, _, _ = batch
    xd, td = _dev(x), _dev(tris)
    pairs, n = ctx.batch_broadphase(xd, td, _dev(tri_off))
    out = ctx.batch_evaluate(xd, td, _dev(vert_off), pairs, n, precision=1)
    ctx.check()
    G = out["grad"].cpu().numpy()
    nb = int(out["n_blocks"].item())
    rp, ci, va = out["row_ptr"].cpu().numpy(), out["col_idx"][:nb].cpu().numpy(), out["vals"][:nb].cpu().numpy()
    E = out["energies"].cpu().numpy()
    for p, (xp, tp, _) in enumerate(probs):
        xpd, tpd = _dev(xp), _dev(tp)
        pp, npp = ctx.broadphase(xpd, tpd)
        o = ctx.evaluate(xpd, tpd, pp, npp, precision=1)
        ctx.check()
        assert o["energy"].item() == pytest.approx(E[p], rel=1e-12)
        v0, v1 = vert_off[p], vert_off[p + 1]
        # rows are summed in pair-key order in both cases: bit-identical
        assert np.array_equal(o["grad"].cpu().numpy(), G[v0:v1])
        b0, b1 = rp[v0], rp[v1]
        nbp = int(o["n_blocks"].item())
        assert nbp == b1 - b0
        assert np.array_equal(o["col_idx"][:nbp].cpu().numpy() + v0, ci[b0:b1])
        assert np.array_equal(o["vals"][:nbp].cpu().numpy(), va[b0:b1])


def test_batch_offsets_are_validated(batch, ctx):
    _, x, tris, vert_off, tri_off, _, _ = batch
    xd, td = _dev(x), _dev(tris)
    bad_t = tri_off.copy()
    bad_t[-1] -= 1  # does not reach n_tris
    ctx.batch_broadphase(xd, td, _dev(bad_t))
    assert ctx.status() == 1
    bad_t = tri_off.copy()
    bad_t[3], bad_t[4] = bad_t[4], bad_t[3]  # decreasing
    ctx.batch_broadphase(xd, td, _dev(bad_t))
    assert ctx.status() == 1
    pairs, n = ctx.batch_broadphase(xd, td, _dev(tri_off))
    bad_v = vert_off.copy()
    bad_v[0] = 1
    ctx.batch_evaluate(xd, td, _dev(bad_v), pairs, n)
    assert ctx.status() == 1
    ctx.batch_evaluate(xd, td, _dev(vert_off), pairs, n)
    assert ctx.status() == 0


def test_batch_step_in_hip_graph(batch, ctx):
    """The batched step (broad phase + evaluation with the Hessian) captured once and replayed
    three times, with unrelated eager evaluations in between; every replay must reproduce the
    eager result exactly (the step is deterministic)."""
    probs, x, tris, vert_off, tri_off, _, _ = batch
    xd, td, vo, to = _dev(x), _dev(tris), _dev(vert_off), _dev(tri_off)
    ctx.set_timing([])
    cap = 1 << 21
    pairs = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = ctx.batch_evaluate(xd, td, vo, pairs[:1], torch.zeros(1, dtype=torch.int64, device="cuda"), precision=1)

    def step():
        ctx.batch_broadphase(xd, td, to, capacity=cap, out=(pairs, n))
        ctx.batch_evaluate(xd, td, vo, pairs, n, precision=1, out=out)

    def snapshot():
        torch.cuda.synchronize()
        nb = int(out["n_blocks"].item())
        return (int(n.item()), out["energies"].cpu().numpy().copy(), out["grad"].cpu().numpy().copy(),
                out["row_ptr"].cpu().numpy().copy(), out["col_idx"][:nb].cpu().numpy().copy(),
                out["vals"][:nb].cpu().numpy().copy(), int(out["n_hits"].item()))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    ref = snapshot()
    ctx.check()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        step()
    xp, tp, _ = probs[0]
    for rep in range(3):
        out["energies"].zero_()
        out["grad"].zero_()
        g.replay()
        got = snapshot()
        ctx.check()
        assert got[0] == ref[0] and got[6] == ref[6], rep
        for a, b in zip(got[1:6], ref[1:6]):
            assert np.array_equal(a, b), rep
        # eager work on the same context between replays
        pe, ne = ctx.broadphase(_dev(xp), _dev(tp))
        ctx.evaluate(_dev(xp), _dev(tp), pe, ne, precision=1)
        torch.cuda.synchronize()
        ctx.check()
