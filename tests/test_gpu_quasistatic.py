"""Quasi-static coupling through the C ABI against the oracle: the springs' BSR pattern
(bit-exact), the objective (Phi, its gradient and the springs' Hessian), the coupled PCG
against a dense solve, and quasi-static trajectories."""

import numpy as np
import pytest
import torch

import oracle
from oracle import quasistatic as qs
from paper_2606_06511_amd import workloads

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _model(x, tris, **kw):
    from paper_2606_06511_amd.energy import TTIE

    return TTIE(torch.from_numpy(tris), len(x), **kw)


@pytest.mark.parametrize("which", ["cloth", "sphere", "soup"])
def test_springs_pattern(which):
    if which == "cloth":
        x, tris = workloads.folded_cloth(0, n=64)
    elif which == "sphere":
        x, tris = workloads.uv_sphere(64, 33)  # poles of valence 64
    else:
        x, tris = workloads.coplanar_soup(0, n_tris=3000)  # three vertices per triangle
    m = _model(x, tris, max_pairs=1 << 16, max_hits=1 << 12)
    rp, ci = m.ctx.springs_pattern(m.tris, len(x))
    edges = qs.spring_edges(tris)
    rp_ref, ci_ref, _ = qs.stiffness_bsr(len(x), edges, np.zeros((len(edges), 3, 3)), 0.0)
    np.testing.assert_array_equal(rp.cpu().numpy(), rp_ref)
    np.testing.assert_array_equal(ci.cpu().numpy(), ci_ref)


def test_springs_pattern_capacity_and_index_errors():
    from paper_2606_06511_amd import ttie

    x, tris = workloads.grid_mesh(8)
    m = _model(x, tris, max_pairs=1 << 12, max_hits=1 << 10)
    with pytest.raises(ttie.TTIEError):
        m.ctx.springs_pattern(m.tris, len(x), capacity=10)
    bad = tris.copy()
    bad[3, 1] = len(x) + 5
    with pytest.raises(ttie.TTIEError):
        m.ctx.springs_pattern(_dev(bad, torch.int32), len(x))


def test_qs_eval_matches_oracle():
    x, tris = workloads.folded_cloth(0, n=48)
    rng = np.random.default_rng(7)
    rest = x + 0.004 * rng.normal(size=x.shape)   # stretched and compressed edges
    x_prev = x + 0.002 * rng.normal(size=x.shape)
    # one edge of zero length at x
    e0 = qs.spring_edges(tris)[100]
    x = x.copy()
    x[e0[1]] = x[e0[0]]
    k, mm, w = 1.3, 0.7, 2.5e3
    m = _model(x, tris, max_pairs=1 << 18, max_hits=1 << 14)
    xd = _dev(x)
    out_t = m.evaluate(xd, hessian=False)
    o = m.ctx.qs_eval(*m.ctx.springs_pattern(m.tris, len(x)), xd, _dev(rest), _dev(x_prev), k, mm, w,
                      out_t["energy"], out_t["grad"])
    m.ctx.check()
    pl = oracle.pairs(x, tris)
    phi, g, K, r = qs.objective(x, rest, x_prev, tris, qs.spring_edges(tris), pl, k, mm, w)
    assert r["E"] > 0
    assert o["phi"].item() == pytest.approx(phi, rel=1e-12)
    assert _rel(o["grad"].cpu().numpy(), g) <= 1e-12
    assert _rel(o["vals"].cpu().numpy(), K[2]) <= 1e-13
    # without the energy (w = 0)
    o0 = m.ctx.qs_eval(*m.ctx.springs_pattern(m.tris, len(x)), xd, _dev(rest), _dev(x_prev), k, mm, 0.0)
    phi0, g0, _, _ = qs.objective(x, rest, x_prev, tris, qs.spring_edges(tris), pl, k, mm, 0.0, hessian=False)
    assert o0["phi"].item() == pytest.approx(phi0, rel=1e-12)
    assert _rel(o0["grad"].cpu().numpy(), g0) <= 1e-12


def test_pcg_coupled_matches_dense_solve():
    x, tris = workloads.folded_cloth(0, n=24)
    m = _model(x, tris, max_pairs=1 << 16, max_hits=1 << 12)
    xd = _dev(x)
    rp, ci = m.ctx.springs_pattern(m.tris, len(x))
    w = 1e4
    out_t = m.evaluate(xd, hessian=True)
    o = m.ctx.qs_eval(rp, ci, xd, xd, xd, 1.0, 1.0, w, out_t["energy"], out_t["grad"])
    nb = int(out_t["n_blocks"].item())
    H = oracle.bsr_to_dense(out_t["row_ptr"].cpu().numpy(), out_t["col_idx"][:nb].cpu().numpy(),
                            out_t["vals"][:nb].cpu().numpy(), len(x))
    K = oracle.bsr_to_dense(rp.cpu().numpy(), ci.cpu().numpy(), o["vals"].cpu().numpy(), len(x))
    assert np.abs(H).max() > 0
    mu = 0.1
    A = K + w * H + mu * np.eye(3 * len(x))
    b = o["grad"].cpu().numpy().ravel()
    d_ref = np.linalg.solve(A, -b)
    d, info = m.ctx.pcg_coupled(rp, ci, o["vals"], w, o["grad"], scale=-1.0, mu=mu, max_iter=3000, tol=1e-13)
    info = info.cpu().numpy()
    assert _rel(d.cpu().numpy().ravel(), d_ref) <= 1e-9
    assert info[2] == mu and info[3] == pytest.approx(float(d_ref @ -b), rel=1e-9)


def test_evaluation_after_pattern_is_unchanged():
    """The pattern build borrows the evaluation's counters: an evaluation after it must equal
    one before it, bit for bit."""
    x, tris = workloads.folded_cloth(0, n=32)
    m = _model(x, tris, max_pairs=1 << 16, max_hits=1 << 12)
    xd = _dev(x)
    o1 = m.evaluate(xd, hessian=True)
    ref = [o1[k].cpu().numpy().copy() for k in ("energy", "grad", "row_ptr", "n_blocks")]
    m.ctx.springs_pattern(m.tris, len(x))
    o2 = m.evaluate(xd, hessian=True)
    for a, k in zip(ref, ("energy", "grad", "row_ptr", "n_blocks")):
        np.testing.assert_array_equal(o2[k].cpu().numpy(), a)
    assert ref[0][0] > 0


def test_pcg_coupled_needs_fp64_evaluation():
    from paper_2606_06511_amd import ttie

    x, tris = workloads.folded_cloth(0, n=16)
    m = _model(x, tris, max_pairs=1 << 14, max_hits=1 << 10, precision=ttie.MIXED)
    xd = _dev(x)
    rp, ci = m.ctx.springs_pattern(m.tris, len(x))
    m.evaluate(xd, hessian=False)
    vals = torch.zeros((ci.shape[0], 3, 3), dtype=torch.float64, device="cuda")
    b = torch.ones((len(x), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ttie.TTIEError):
        m.ctx.pcg_coupled(rp, ci, vals, 1.0, b)


def test_quasi_static_steps_match_oracle():
    """Newton iterations of the quasi-static objective from the same states on both sides.

    Whole trajectories are not comparable: on this input a perturbation of 1e-15 in x changes
    the oracle's own step lengths after one step (the Armijo decisions and the set of hits
    switch), with truncated and with converged solves alike.  So the states come from a GPU
    run, and from each of them one iteration with a converged solve is compared: objective,
    energy, hits, step length and displacement."""
    from paper_2606_06511_amd.quasistatic import QuasiStatic

    x, tris = workloads.folded_cloth(0, n=24)
    k, mm, w = 1.0, 1.0, 1e4
    m = _model(x, tris, max_pairs=1 << 16, max_hits=1 << 12)
    xd = _dev(x)
    sim = QuasiStatic(m, xd, k, mm, w)
    states = [xd]
    cur, cand = xd, None
    for _ in range(2):
        cur, recs, cand = sim.step(cur, newton_iters=2, pcg_iters=20, cand=cand)
        assert all(r["phi_new"] <= r["phi"] for r in recs)
        states.append(cur)
    for xk in states:
        xk_np = xk.cpu().numpy()
        x1, rg, _ = sim.step(xk, newton_iters=1, pcg_iters=3000, pcg_tol=1e-13)
        x1_ref, ro = qs.qs_step(xk_np, x, tris, k, mm, w, newton_iters=1, pcg_iters=3000, pcg_tol=1e-13)
        a, b = rg[0], ro[0]
        assert a["phi"] == pytest.approx(b["phi"], rel=1e-12)
        assert a["E"] == pytest.approx(b["E"], rel=1e-10)
        assert a["hits"] == b["hits"] > 0
        assert a["alpha"] == b["alpha"]
        assert a["phi_new"] <= a["phi"] and b["phi_new"] <= b["phi"]
        assert _rel(x1.cpu().numpy() - xk_np, x1_ref - xk_np) <= 1e-7


def test_axpy_keeps_positions_in_the_predicate_domain():
    from paper_2606_06511_amd import ttie

    c = ttie.Context(0)
    c.reserve(16, 16, 16)
    x = torch.tensor([[0.0, 1.0, 0.0], [0.0, 0.0, 3.0]], dtype=torch.float64, device="cuda")
    d = torch.tensor([[1e-250, 0.5, 2.0 ** -200], [-(2.0 ** -201), -1e-300, 1.0]], dtype=torch.float64,
                     device="cuda")
    out = c.axpy(x, 1.0, d).cpu().numpy()
    np.testing.assert_array_equal(out, [[0.0, 1.5, 2.0 ** -200], [0.0, 0.0, 4.0]])
