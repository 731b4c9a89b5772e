"""The inexact Newton consumer: device Jacobi-PCG, swept candidates, and the Newton loop on
the 20,000-triangle subset of the 4,194,304-triangle noisy sphere against the oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_2606_06511_amd import workloads

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _model(x, tris, **kw):
    from paper_2606_06511_amd.energy import TTIE

    return TTIE(torch.from_numpy(tris), len(x), **kw)


@pytest.mark.parametrize("precision", [0, 1])
def test_pcg_matches_dense_solve(precision):
    x, tris = workloads.folded_cloth(seed=0, n=40)
    m = _model(x, tris, max_pairs=1 << 16, max_hits=1 << 12, precision=precision)
    xd = torch.from_numpy(x).cuda()
    out = m.evaluate(xd, hessian=True)
    nb = int(out["n_blocks"].item())
    Hd = oracle.bsr_to_dense(out["row_ptr"].cpu().numpy(), out["col_idx"][:nb].cpu().numpy(),
                             out["vals"][:nb].cpu().numpy().astype(np.float64), len(x))
    g = out["grad"].cpu().numpy().astype(np.float64).ravel()
    diag = np.diag(Hd)
    touched = np.repeat(np.diff(out["row_ptr"].cpu().numpy()) > 0, 3)
    mu = 1e-3 * diag[touched].mean()
    d_ref = np.linalg.solve(Hd + mu * np.eye(len(g)), -g)
    d, info = m.ctx.pcg(out["row_ptr"], out["col_idx"], out["vals"], out["grad"], scale=-1.0, mu_rel=1e-3,
                        max_iter=2000, tol=1e-12 if precision == 0 else 1e-6)
    info = info.cpu().numpy()
    assert info[2] == pytest.approx(mu, rel=1e-12 if precision == 0 else 1e-6)
    assert _rel(d.cpu().numpy().ravel(), d_ref) <= (1e-8 if precision == 0 else 1e-3)
    assert info[3] == pytest.approx(float(d_ref @ -g), rel=1e-6 if precision == 0 else 1e-2)
    # a capped solve stops at the iteration limit and reports it
    _, info2 = m.ctx.pcg(out["row_ptr"], out["col_idx"], out["vals"], out["grad"], scale=-1.0, max_iter=3, tol=0.0)
    assert info2.cpu().numpy()[0] == 3


@pytest.mark.parametrize("precision", [0, 1])
def test_matrix_free_pcg_matches_dense_and_bsr(precision):
    x, tris = workloads.folded_cloth(seed=0, n=40)
    m = _model(x, tris, max_pairs=1 << 16, max_hits=1 << 12, precision=precision)
    out = m.evaluate(torch.from_numpy(x).cuda(), hessian=True)
    nb = int(out["n_blocks"].item())
    Hd = oracle.bsr_to_dense(out["row_ptr"].cpu().numpy(), out["col_idx"][:nb].cpu().numpy(),
                             out["vals"][:nb].cpu().numpy().astype(np.float64), len(x))
    g = out["grad"].cpu().numpy().astype(np.float64).ravel()
    touched = np.repeat(np.diff(out["row_ptr"].cpu().numpy()) > 0, 3)
    mu = 1e-3 * np.diag(Hd)[touched].mean()
    d_ref = np.linalg.solve(Hd + mu * np.eye(len(g)), -g)
    tol = 1e-12 if precision == 0 else 1e-6
    d_mf, info_mf = m.ctx.pcg_mf(out["grad"], scale=-1.0, mu_rel=1e-3, max_iter=2000, tol=tol)
    d_bsr, info_bsr = m.ctx.pcg(out["row_ptr"], out["col_idx"], out["vals"], out["grad"], scale=-1.0, mu_rel=1e-3,
                                max_iter=2000, tol=tol)
    i_mf, i_bsr = info_mf.cpu().numpy(), info_bsr.cpu().numpy()
    assert i_mf[2] == pytest.approx(mu, rel=1e-12 if precision == 0 else 1e-6)
    assert i_mf[2] == pytest.approx(i_bsr[2], rel=1e-12 if precision == 0 else 1e-6)
    assert _rel(d_mf.cpu().numpy().ravel(), d_ref) <= (1e-8 if precision == 0 else 1e-3)
    assert _rel(d_mf.cpu().numpy(), d_bsr.cpu().numpy()) <= (1e-8 if precision == 0 else 1e-3)
    # without an evaluation of the same mesh there is no Hessian to use
    from paper_2606_06511_amd import ttie

    with pytest.raises(ttie.TTIEError):
        m.ctx.pcg_mf(out["grad"][:-1].contiguous())


def test_swept_candidates_match_oracle():
    x, tris = workloads.folded_cloth(seed=2, n=96)
    rng = np.random.default_rng(0)
    x_end = x + 0.01 * rng.normal(size=x.shape)
    m = _model(x, tris, max_pairs=1 << 19, max_hits=1 << 12)
    p, n = m.candidates(torch.from_numpy(x).cuda(), torch.from_numpy(x_end).cuda())
    got = p[: int(n.item())].cpu().numpy()
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    ref = oracle.pairs_swept(x, x_end, tris)
    np.testing.assert_array_equal(got, ref)
    assert len(ref) > len(oracle.pairs(x, tris))
    # an undersized pair buffer is reported, not truncated silently
    from paper_2606_06511_amd import ttie

    small = _model(x, tris, max_pairs=1 << 18, max_hits=1 << 12)
    with pytest.raises(ttie.TTIEError):
        small.candidates(torch.from_numpy(x).cuda(), torch.from_numpy(x_end).cuda())


@pytest.fixture(scope="module")
def sphere_subset():
    # the 4,194,304-triangle noisy sphere; the seed point is the centroid of the first
    # intersecting pair in canonical order, and the subset its 20,000 nearest triangles
    x, tris = workloads.noisy_sphere(seed=0, n_lon=2048, n_bands=1025)
    assert len(tris) == 4_194_304
    pairs = oracle.pairs(x, tris)
    res = oracle.evaluate(x, tris, pairs, hessian=False)
    i, j = pairs[res["hit_pair"][0]]
    seed_pt = np.concatenate([x[tris[i]], x[tris[j]]]).mean(0)
    return workloads.submesh_near(x, tris, seed_pt, 20_000)


def test_newton_subset_fp64_against_oracle(sphere_subset):
    from paper_2606_06511_amd.newton import newton

    x, tris = sphere_subset
    assert len(tris) == 20_000
    m = _model(x, tris, max_pairs=1 << 20, max_hits=1 << 16)
    # trajectory parity with 20 PCG iterations per step: at this cap a relative perturbation
    # of 1e-15 in x moves the oracle's own 8-step energies by at most ~1e-8, so the two
    # summation orders must agree to 1e-6 and take the same step lengths
    _, E_ref, al_ref, _ = oracle.newton(x, tris, steps=8, pcg_iters=20)
    _, hist = newton(m, torch.from_numpy(x).cuda(), steps=8, pcg_iters=20)
    E = np.array([h["E"] for h in hist])
    assert E[0] == pytest.approx(E_ref[0], rel=1e-10)
    np.testing.assert_allclose(E, E_ref, rtol=1e-6)
    assert [h["alpha"] for h in hist[:-1]] == list(al_ref)
    # at the default 50 iterations the truncated solve is rounding-sensitive on this input
    # (the oracle alone moves E1 by several percent under the same 1e-15 perturbation):
    # check the properties both runs must have. Armijo: the energy never increases; both
    # remove most of it (the pure TTIE energy can stall where separating one pair deepens
    # another, so exactly 0 is not reached on this subset in 20 steps)
    _, E_ref, _, _ = oracle.newton(x, tris, steps=20)
    _, hist = newton(m, torch.from_numpy(x).cuda(), steps=20)
    E = np.array([h["E"] for h in hist])
    assert E[0] == pytest.approx(E_ref[0], rel=1e-10)
    assert np.all(np.diff(E) <= 0) and np.all(np.diff(E_ref) <= 0)
    assert E[-1] <= 0.3 * E[0] and E_ref[-1] <= 0.3 * E_ref[0]


def test_newton_subset_matrix_free_against_oracle(sphere_subset):
    from paper_2606_06511_amd.newton import newton

    x, tris = sphere_subset
    m = _model(x, tris, max_pairs=1 << 20, max_hits=1 << 16)
    _, E_ref, al_ref, _ = oracle.newton(x, tris, steps=8, pcg_iters=20)
    _, hist = newton(m, torch.from_numpy(x).cuda(), steps=8, pcg_iters=20, matrix_free=True)
    E = np.array([h["E"] for h in hist])
    np.testing.assert_allclose(E, E_ref, rtol=1e-6)
    assert [h["alpha"] for h in hist[:-1]] == list(al_ref)


def test_newton_subset_mixed_against_oracle(sphere_subset):
    """The mixed path (float32 gradient, Hessian and solve) against the float64 oracle: the first
    step element by element -- E0 to 1e-10 (float64 on both paths), the same step length, the
    displacement of every vertex within 1e-3 of the largest one and E1 within 1e-4 (a truncated
    solve of 20 iterations on float32 data) -- then the whole 20-step run by its properties."""
    from paper_2606_06511_amd import ttie
    from paper_2606_06511_amd.newton import newton

    x, tris = sphere_subset
    m = _model(x, tris, max_pairs=1 << 20, max_hits=1 << 16, precision=ttie.MIXED)
    x1_ref, E_ref, al_ref, _ = oracle.newton(x, tris, steps=1, pcg_iters=20)
    x1, hist = newton(m, torch.from_numpy(x).cuda(), steps=1, pcg_iters=20)
    x1 = x1.cpu().numpy()
    assert hist[0]["E"] == pytest.approx(E_ref[0], rel=1e-10)
    assert hist[0]["alpha"] == al_ref[0]
    d, d_ref = x1 - x, x1_ref - x
    assert np.abs(d - d_ref).max() <= 1e-3 * np.abs(d_ref).max()
    assert hist[-1]["E"] == pytest.approx(E_ref[1], rel=1e-4)
    _, hist = newton(m, torch.from_numpy(x).cuda(), steps=20)
    E = np.array([h["E"] for h in hist])
    assert np.all(np.diff(E) <= 0)
    assert E[-1] <= 0.3 * E[0]


def test_pcg_runs_on_the_touched_rows_only():
    """The solve iterates over the rows holding blocks; b must vanish elsewhere (a gradient
    does), and a right-hand side that does not is reported."""
    x, tris = workloads.folded_cloth(seed=0, n=40)
    m = _model(x, tris, max_pairs=1 << 16, max_hits=1 << 12)
    out = m.evaluate(torch.from_numpy(x).cuda(), hessian=True)
    rp = out["row_ptr"].cpu().numpy()
    empty = np.nonzero(np.diff(rp) == 0)[0]
    assert len(empty) > 0
    g = out["grad"].cpu().numpy()
    assert not g[empty].any()
    d, _ = m.ctx.pcg(out["row_ptr"], out["col_idx"], out["vals"], out["grad"], scale=-1.0)
    m.ctx.check()
    assert not d.cpu().numpy()[empty].any()
    b = out["grad"].clone()
    b[int(empty[0]), 1] = 1.0
    m.ctx.pcg(out["row_ptr"], out["col_idx"], out["vals"], b, scale=-1.0)
    assert m.ctx.status() == 1
