"""Quasi-static simulation: the energy coupled with a synthetic elastic model (a stand-in for
the unspecified one of the paper's Fig. 2), minimised step by step with inexact Newton.

One step minimises, from the positions x_prev at its start,

    Phi(x) = sum over edges (k/2)(|x_i - x_j| - |r_i - r_j|)^2 + w E(x) + (m/2)|x - x_prev|^2

with ``newton_iters`` Newton iterations: evaluate E and its gradient at x (FP64, candidates
from the broad phase), Phi, grad Phi and the springs' PSD Hessian K (with m I) in
``ttie_qs_eval``; solve (K + w H) d = -grad Phi by Jacobi-PCG with H applied from the hit
records (``ttie_pcg_coupled``); take candidates from boxes swept from x to x + d; backtrack on
Phi (Armijo).  Steps repeat until one starts intersection-free (E = 0).  As in the Newton
loop, an iterate evaluates over the swept candidates of the line search that produced it (a
superset of its own candidates with bit-identical results), so the broad phase runs once per
iteration, and the evaluation of the accepted trial point serves the next iteration.  All arithmetic runs in library kernels; this module sequences the calls and reads
the scalars the line search needs.
"""

from __future__ import annotations

import time

import torch

from . import ttie
from .energy import TTIE


class QuasiStatic:
    """Quasi-static driver for one mesh on one GPU (FP64 throughout)."""

    def __init__(self, model: TTIE, rest: torch.Tensor, k: float, m: float, w: float):
        if model.precision != ttie.FP64:
            raise ValueError("the quasi-static objective needs FP64 evaluations")
        self.model, self.ctx = model, model.ctx
        self.rest = rest.detach().to(model.device, torch.float64).contiguous()
        self.k, self.m, self.w = float(k), float(m), float(w)
        self.row_ptr, self.col_idx = self.ctx.springs_pattern(model.tris, model.n_verts)
        self._out = None

    def objective(self, x, x_prev, out_t, grad=True, vals=True):
        """Phi at x from an evaluation ``out_t`` of the energy at x."""
        out = self.ctx.qs_eval(self.row_ptr, self.col_idx, x, self.rest, x_prev, self.k, self.m, self.w,
                               out_t["energy"], out_t["grad"], grad=grad, vals=vals,
                               out=self._out if (grad and vals) else None)
        if grad and vals:
            self._out = out
        return out

    def step(self, x_prev, newton_iters=4, pcg_iters=50, pcg_tol=1e-6, armijo_c=1e-4, beta=0.5, max_halvings=30,
             cand=None, out_t=None):
        """One quasi-static step from x_prev; returns the new positions, per-iteration records
        and the candidates that cover the new positions.  ``cand`` (pairs, n_pairs) may give
        candidates covering x_prev (e.g. the previous step's); otherwise the broad phase runs.
        ``out_t`` may give the energy's evaluation at x_prev when it is the context's last."""
        model, ctx = self.model, self.ctx
        x_prev = x_prev.detach().contiguous()
        x = x_prev.clone()
        recs = []
        # out_t: the energy's evaluation at x (the accepted trial point's after the first)
        for _ in range(newton_iters):
            t0 = time.perf_counter()
            if out_t is None:
                if cand is None:
                    out_t = model.evaluate(x, hessian=False)
                else:
                    out_t = model.evaluate(x, hessian=False, pairs=cand[0], n_pairs=cand[1])
            o = self.objective(x, x_prev, out_t)
            phi = o["phi"].item()
            d, info = ctx.pcg_coupled(self.row_ptr, self.col_idx, o["vals"], self.w, o["grad"], scale=-1.0, mu=0.0,
                                      max_iter=pcg_iters, tol=pcg_tol)
            inf = info.cpu().tolist()
            gd = -inf[3]  # info[3] = d . (-grad Phi)
            rec = {"phi": phi, "E": out_t["energy"].item(), "hits": int(out_t["n_hits"].item()),
                   "pairs": int(model.n_pairs.item()), "pcg_iters": int(inf[0])}
            pairs, n = model.candidates(x, ctx.axpy(x, 1.0, d))
            alpha = 1.0
            for h in range(max_halvings):
                xt = ctx.axpy(x, alpha, d)
                out_t = model.evaluate(xt, hessian=False, pairs=pairs, n_pairs=n)
                phit = self.objective(xt, x_prev, out_t, grad=False, vals=False)["phi"].item()
                if phit <= phi + armijo_c * alpha * gd:
                    break
                if h + 1 < max_halvings:
                    alpha *= beta
            x = xt
            cand = (pairs, n)
            torch.cuda.synchronize()
            rec.update(alpha=alpha, phi_new=phit, ms=(time.perf_counter() - t0) * 1e3)
            recs.append(rec)
        return x, recs, cand

    def run(self, x0, steps, **kw):
        """Steps from x0 until one starts with E = 0 or ``steps`` ran.  Returns the final
        positions and per-step records {E, hits, newton}."""
        x = x0.detach().clone().contiguous()
        hist = []
        cand = None
        for _ in range(steps):
            if cand is None:
                o = self.model.evaluate(x, hessian=False)
            else:
                o = self.model.evaluate(x, hessian=False, pairs=cand[0], n_pairs=cand[1])
            E = o["energy"].item()
            if E == 0.0:
                hist.append({"E": 0.0, "hits": 0, "newton": []})
                return x, hist
            hits = int(o["n_hits"].item())
            x, recs, cand = self.step(x, cand=cand, out_t=o, **kw)
            hist.append({"E": E, "hits": hits, "newton": recs})
        o = self.model.evaluate(x, hessian=False)
        hist.append({"E": o["energy"].item(), "hits": int(o["n_hits"].item()), "newton": []})
        return x, hist
