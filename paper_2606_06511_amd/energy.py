"""Differentiable TTIE energy on the GPU: an evaluator bound to a mesh topology, and the
PyTorch autograd wrapper whose backward is the library's gradient and whose double backward
is its Hessian-vector product.

Argument marshalling only: every value is computed by ``libttie.so`` kernels.
"""

from __future__ import annotations

import torch

from . import ttie


class TTIE:
    """Evaluator for one triangle topology (``tris``) on one GPU.

    Positions are passed per call (float64, ``(n_verts, 3)``, on the GPU).  The broad phase
    is rerun for every evaluation unless a candidate list is given.  With ``vertex_adjacent``,
    pairs sharing exactly one vertex are listed and evaluated (only pairs sharing an edge are
    skipped as adjacent).
    """

    def __init__(self, tris: torch.Tensor, n_verts: int, *, device: int = 0, max_pairs: int = 1 << 22,
                 max_hits: int = 1 << 18, max_blocks: int | None = None, precision: int = ttie.FP64,
                 psd: int = ttie.PSD_PER_PART, interval: int = ttie.INTERVAL_EQ1, broadphase: int = ttie.BROAD_LBVH,
                 vertex_adjacent: bool = False):
        self.device = torch.device("cuda", device)
        self.tris = tris.to(self.device, torch.int32).contiguous()
        self.n_verts = int(n_verts)
        self.precision, self.psd, self.interval, self.method = precision, psd, interval, broadphase
        self.vertex_adjacent = bool(vertex_adjacent)
        self.ctx = ttie.Context(device)
        self.ctx.reserve(self.n_verts, self.tris.shape[0], max_pairs, max_hits=max_hits,
                         max_blocks=max_blocks if max_blocks is not None else 36 * max_hits)
        self.pairs = torch.empty((max_pairs, 2), dtype=torch.int32, device=self.device)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.generation = 0  # bumped by every evaluation (the hit list lives in the context)
        self._outs = {}

    @property
    def dtype(self):
        return torch.float64 if self.precision == ttie.FP64 else torch.float32

    def candidates(self, x: torch.Tensor, x_end: torch.Tensor | None = None, *, check: bool = True):
        """Candidate pairs at x (or swept from x to x_end) into the evaluator's pair buffer;
        raises when the buffer overflowed (unless ``check`` is False: then the caller checks)."""
        self.ctx.broadphase(x, self.tris, self.method, capacity=self.pairs.shape[0], out=(self.pairs, self.n_pairs),
                            x_end=x_end, vertex_adjacent=self.vertex_adjacent)
        if check:
            self.ctx.check()
        return self.pairs, self.n_pairs

    def evaluate(self, x: torch.Tensor, *, hessian: bool = True, pairs=None, n_pairs=None, flags=False):
        """Energy, gradient and (optionally) the BSR Hessian at x; raises on kernel errors."""
        x = x.detach().contiguous()
        if pairs is None:
            pairs, n_pairs = self.candidates(x, check=False)
        key = (hessian, flags, pairs.shape[0])
        out = self.ctx.evaluate(x, self.tris, pairs, n_pairs, precision=self.precision, psd=self.psd,
                                interval=self.interval, hessian=hessian, flags=flags, out=self._outs.get(key),
                                vertex_adjacent=self.vertex_adjacent)
        self._outs[key] = out
        self.generation += 1
        self.ctx.check()
        return out

    def hvp(self, x: torch.Tensor, v: torch.Tensor, mode: int = ttie.HVP_EXACT):
        """H v at the positions of the last evaluation (which must be x)."""
        return self.ctx.hvp(x.detach().contiguous(), self.tris, v.to(self.dtype).contiguous(), mode)

    def energy(self, x: torch.Tensor) -> torch.Tensor:
        """Differentiable scalar energy (twice differentiable: exact Hessian-vector products)."""
        return _Energy.apply(x, self)


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, model: TTIE):
        out = model.evaluate(x, hessian=False)
        ctx.model = model
        ctx.generation = model.generation
        # the evaluator reuses its output buffers: keep a copy of this gradient
        ctx.save_for_backward(x, out["grad"].clone())
        return out["energy"][0].clone()

    @staticmethod
    def backward(ctx, gE):
        x, G = ctx.saved_tensors
        return _Gradient.apply(x, G, gE, ctx.model, ctx.generation), None


class _Gradient(torch.autograd.Function):
    """x -> dE/dx * gE, whose own backward is the Hessian-vector product."""

    @staticmethod
    def forward(ctx, x, G, gE, model: TTIE, generation: int):
        ctx.model = model
        ctx.generation = generation
        ctx.save_for_backward(x, G, gE)
        return G.to(x.dtype) * gE

    @staticmethod
    def backward(ctx, u):
        x, G, gE = ctx.saved_tensors
        model = ctx.model
        if model.generation != ctx.generation:
            # another evaluation replaced the hit list: rebuild it at x
            model.evaluate(x, hessian=False)
        Hu = model.hvp(x, u).to(x.dtype)
        dx = Hu * gE if ctx.needs_input_grad[0] else None
        dgE = (G.to(u.dtype) * u).sum().reshape(gE.shape) if ctx.needs_input_grad[2] else None
        return dx, None, dgE, None, None
