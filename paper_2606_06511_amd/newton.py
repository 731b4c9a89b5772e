"""Inexact Newton consumer of the hot path (the abstract's GPU inexact-Newton route).

Per step: evaluate energy, gradient and PSD BSR Hessian at x; solve (H + mu I) d = -g with
the library's device-resident Jacobi-PCG; take candidates with boxes swept from x to x + d
(so every trial point is covered); Armijo backtracking on E along d.  The accepted point lies
on the swept segment, so the next step evaluates over the same swept list instead of running
the broad phase again: its extra pairs have disjoint boxes (T = 0), and the assembly sums the
hits in pair-key order, so the results are bit-identical to those over the exact list.  The
line search evaluates every trial point with the Hessian, and the accepted one (always the last
evaluated) is the next step's evaluation.  The paper gives no parameters: mu = mu_rel * mean diagonal entry, 50 PCG iterations or relative
residual 1e-6, c = 1e-4, halving up to 30 times.  All arithmetic runs in library kernels; this module only
sequences the calls and reads the scalars the line search needs.
"""

from __future__ import annotations

import time

import torch

from .energy import TTIE


def newton(model: TTIE, x: torch.Tensor, steps: int = 20, pcg_iters: int = 50, pcg_tol: float = 1e-6,
           mu_rel: float = 1e-3, armijo_c: float = 1e-4, beta: float = 0.5, max_halvings: int = 30,
           matrix_free: bool = False):
    """Runs up to ``steps`` Newton steps from x (float64 on the GPU).  Returns the final
    positions and a list of per-step records {E, alpha, pcg_iters, pcg_resid, pairs, hits,
    ms}; the last record holds the final energy.  ``matrix_free`` solves with the per-hit
    Hessian records instead of the assembled BSR matrix (same system, no assembly)."""
    ctx = model.ctx
    x = x.detach().clone().contiguous()
    hist = []
    out = None  # the evaluation at x: the first step's, then the accepted trial point's
    for _ in range(steps):
        t0 = time.perf_counter()
        if out is None:
            out = model.evaluate(x, hessian=not matrix_free)
        E = out["energy"].item()
        rec = {"E": E, "pairs": int(model.n_pairs.item()), "hits": int(out["n_hits"].item())}
        if E == 0.0:
            hist.append(rec)
            break
        if matrix_free:
            d, info = ctx.pcg_mf(out["grad"], scale=-1.0, mu_rel=mu_rel, max_iter=pcg_iters, tol=pcg_tol)
        else:
            d, info = ctx.pcg(out["row_ptr"], out["col_idx"], out["vals"], out["grad"], scale=-1.0, mu_rel=mu_rel,
                              max_iter=pcg_iters, tol=pcg_tol)
        inf = info.cpu().tolist()
        gd = -inf[3]  # info[3] = d . (-g)
        pairs, n = model.candidates(x, ctx.axpy(x, 1.0, d))
        alpha = 1.0
        for h in range(max_halvings):
            xt = ctx.axpy(x, alpha, d)
            out = model.evaluate(xt, hessian=not matrix_free, pairs=pairs, n_pairs=n)
            Et = out["energy"].item()
            if Et <= E + armijo_c * alpha * gd or h + 1 == max_halvings:
                break
            alpha *= beta
        x = xt
        torch.cuda.synchronize()
        rec.update(alpha=alpha, pcg_iters=int(inf[0]), pcg_resid=inf[1], mu=inf[2],
                   ms=(time.perf_counter() - t0) * 1e3)
        hist.append(rec)
    out = model.evaluate(x, hessian=False)
    hist.append({"E": out["energy"].item(), "pairs": int(model.n_pairs.item()), "hits": int(out["n_hits"].item())})
    return x, hist
