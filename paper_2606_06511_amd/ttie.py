"""Thin Python binding of ``libttie.so`` (the C ABI declared in ``include/ttie.h``).

Argument marshalling only: PyTorch provides device memory and the stream, every step of
the computation runs in the library's HIP kernels.  There is no CPU fallback: if the
library is missing or no GPU is visible the calls raise.
"""

from __future__ import annotations

import ctypes
import os

import torch  # imported before the library so that it binds to torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttie.so")

TTIE_OK = 0
(TTIE_ERR_INVALID_ARGUMENT, TTIE_ERR_INDEX_OUT_OF_RANGE, TTIE_ERR_NONFINITE_INPUT, TTIE_ERR_CAPACITY, TTIE_ERR_HIP,
 TTIE_ERR_NO_DEVICE, TTIE_ERR_UNSUPPORTED, TTIE_ERR_INTERNAL) = range(1, 9)
STATUS_NAMES = {
    0: "OK", 1: "INVALID_ARGUMENT", 2: "INDEX_OUT_OF_RANGE", 3: "NONFINITE_INPUT", 4: "CAPACITY",
    5: "HIP", 6: "NO_DEVICE", 7: "UNSUPPORTED", 8: "INTERNAL",
}
FP64, MIXED = 0, 1
PSD_PER_PART, PSD_NEAREST, PSD_PAPER_LITERAL, PSD_RAW_EQ4 = 0, 1, 2, 3
INTERVAL_EQ1, INTERVAL_APPENDIX_HALF = 0, 1
BROAD_BRUTE, BROAD_LBVH, BROAD_HASH = 0, 1, 2
BROAD_VERTEX_ADJACENT = 0x100  # OR'ed into a broad-phase method: list pairs sharing one vertex
EVAL_VERTEX_ADJACENT = 1       # Options.flags bit: evaluate pairs sharing one vertex
HVP_EXACT, HVP_PSD = 0, 1
PAIR_NONE, PAIR_HIT, PAIR_ADJACENT, PAIR_DEGENERATE_FRAME, PAIR_COPLANAR = 0, 1, 2, 3, 4
MAX_PROBLEMS = 4096
PARAM_SCREEN_BLOCKS, PARAM_ROW_BLOCKS, PARAM_TRAV_BUDGET, PARAM_HASH_BUDGET, PARAM_SCREEN_TILE = 0, 1, 2, 3, 4

# every function the header declares, with (restype, argtypes)
_vp, _i64, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t


class Limits(ctypes.Structure):
    _fields_ = [("max_verts", _i64), ("max_tris", _i64), ("max_pairs", _i64), ("max_hits", _i64),
                ("max_blocks", _i64)]


class Mesh(ctypes.Structure):
    _fields_ = [("x", _vp), ("n_verts", _i64), ("tris", _vp), ("n_tris", _i64)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("psd_mode", ctypes.c_int32), ("interval", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


SIGNATURES = {
    "ttie_version": (ctypes.c_char_p, []),
    "ttie_last_error": (ctypes.c_char_p, []),
    "ttie_create": (_i32, [_i32, ctypes.POINTER(_vp)]),
    "ttie_destroy": (_i32, [_vp]),
    "ttie_workspace_size": (_i32, [_vp, ctypes.POINTER(Limits), ctypes.POINTER(_sz)]),
    "ttie_set_workspace": (_i32, [_vp, ctypes.POINTER(Limits), _vp, _sz, _vp]),
    "ttie_get_status": (_i32, [_vp, _vp, ctypes.POINTER(_i32)]),
    "ttie_broadphase": (_i32, [_vp, ctypes.POINTER(Mesh), _i32, _vp, _vp, _i64, _vp, _vp]),
    "ttie_eval": (_i32, [_vp, ctypes.POINTER(Mesh), _vp, _vp, _i64, ctypes.POINTER(Options), _vp, _vp, _vp,
                         _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "ttie_eval_static": (_i32, [_vp, ctypes.POINTER(Mesh), _vp, _vp, _i64, _i64, ctypes.POINTER(Options), _vp, _vp,
                                _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "ttie_batch_broadphase": (_i32, [_vp, ctypes.POINTER(Mesh), _i32, _vp, _vp, _vp, _i64, _vp, _vp]),
    "ttie_batch_eval": (_i32, [_vp, ctypes.POINTER(Mesh), _i32, _vp, _vp, _vp, _i64, ctypes.POINTER(Options), _vp,
                               _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "ttie_get_hits": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_i64), _vp]),
    "ttie_bsr_symbolic": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "ttie_bsr_numeric": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "ttie_hvp": (_i32, [_vp, ctypes.POINTER(Mesh), _vp, _vp, _i32, _vp]),
    "ttie_bsr_mv": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "ttie_pcg": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, ctypes.c_double, _i32,
                        ctypes.c_double, _i32, _vp, _vp]),
    "ttie_pcg_mf": (_i32, [_vp, _i64, _vp, ctypes.c_double, _vp, ctypes.c_double, _i32, ctypes.c_double, _vp, _vp]),
    "ttie_axpy": (_i32, [_vp, _i64, ctypes.c_double, _vp, _vp, _vp, _i32, _vp]),
    "ttie_springs_pattern": (_i32, [_vp, ctypes.POINTER(Mesh), _vp, _vp, _i64, _vp, _vp]),
    "ttie_qs_eval": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            _vp, _vp, _vp, _vp, _vp, _vp]),
    "ttie_pcg_coupled": (_i32, [_vp, _i64, _vp, _vp, _vp, ctypes.c_double, _vp, ctypes.c_double, _vp,
                                ctypes.c_double, _i32, ctypes.c_double, _vp, _vp]),
    "ttie_set_param": (_i32, [_vp, _i32, _i64]),
    "ttie_get_param": (_i32, [_vp, _i32, ctypes.POINTER(_i64)]),
    "ttie_set_timing": (_i32, [_vp, ctypes.c_uint32]),
    "ttie_read_timers": (_i32, [_vp, _i32, _vp, _vp]),
}

STAGES = ["bp_boxes", "bp_sort", "bp_build", "bp_traverse", "screen", "screen_exact", "derivs", "assembly", "hvp",
          "pcg", "elastic", "bp_heavy"]

_lib = None


class TTIEError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"ttie: {STATUS_NAMES.get(status, status)}: {msg}")


def lib():
    """Loads libttie.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2606_06511_amd/build_lib.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != TTIE_OK:
        raise TTIEError(st, lib().ttie_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def version() -> str:
    return lib().ttie_version().decode()


class Context:
    """A library context on one GPU plus the workspace tensor it runs in."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _check(lib().ttie_create(device, ctypes.byref(h)))
        self.handle = h
        self.workspace = None
        self.limits = None

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.ttie_destroy(self.handle)
            self.handle = None

    def reserve(self, n_verts, n_tris, max_pairs, max_hits=None, max_blocks=None):
        """Sizes the workspace for meshes up to these sizes (reallocates when they grow)."""
        if max_hits is None:
            max_hits = max(1024, min(max_pairs, 1 << 20))
        if max_blocks is None:
            max_blocks = 36 * max_hits
        want = (int(n_verts), int(n_tris), int(max_pairs), int(max_hits), int(max_blocks))
        if self.limits is not None and all(w <= h for w, h in zip(want, self.limits)):
            return
        lim = Limits(*want)
        nbytes = ctypes.c_size_t()
        _check(lib().ttie_workspace_size(self.handle, ctypes.byref(lim), ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        _check(lib().ttie_set_workspace(self.handle, ctypes.byref(lim), ctypes.c_void_p(aligned), nbytes.value,
                                        _stream()))
        self.limits = want

    @staticmethod
    def _mesh(x, tris):
        assert x.dtype == torch.float64 and x.is_contiguous() and x.shape[-1] == 3
        assert tris.dtype == torch.int32 and tris.is_contiguous() and tris.shape[-1] == 3
        return Mesh(x.data_ptr(), x.shape[0], tris.data_ptr(), tris.shape[0])

    def status(self):
        st = ctypes.c_int(0)
        _check(lib().ttie_get_status(self.handle, _stream(), ctypes.byref(st)))
        return st.value

    def check(self):
        st = self.status()
        if st != TTIE_OK:
            raise TTIEError(st, "reported by a kernel")

    def broadphase(self, x, tris, method=BROAD_LBVH, capacity=None, out=None, x_end=None, vertex_adjacent=False):
        """Candidate pairs: returns (pairs (capacity, 2) int32, n_pairs (1,) int64), both on the GPU.
        With x_end, boxes cover the triangles at x and at x_end (swept candidates).  With
        vertex_adjacent, pairs sharing exactly one vertex are candidates too."""
        if vertex_adjacent:
            method |= BROAD_VERTEX_ADJACENT
        if capacity is None:
            capacity = self.limits[2]
        m = self._mesh(x, tris)
        if out is None:
            pairs = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=self.device)
            n = torch.zeros(1, dtype=torch.int64, device=self.device)
        else:
            pairs, n = out
        if x_end is not None:
            assert x_end.dtype == torch.float64 and x_end.is_contiguous() and x_end.shape == x.shape
        _check(lib().ttie_broadphase(self.handle, ctypes.byref(m), method, _ptr(x_end), _ptr(pairs), capacity, _ptr(n),
                                     _stream()))
        return pairs, n

    def batch_broadphase(self, x, tris, tri_off, capacity=None, out=None, x_end=None):
        """LBVH candidates of a batch of problems (tri_off: (n_problems + 1,) int64 on the GPU);
        no pair joins two problems.  Returns (pairs, n_pairs) like ``broadphase``."""
        if capacity is None:
            capacity = self.limits[2]
        m = self._mesh(x, tris)
        assert tri_off.dtype == torch.int64 and tri_off.is_contiguous() and tri_off.device == self.device
        if out is None:
            pairs = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=self.device)
            n = torch.zeros(1, dtype=torch.int64, device=self.device)
        else:
            pairs, n = out
        if x_end is not None:
            assert x_end.dtype == torch.float64 and x_end.is_contiguous() and x_end.shape == x.shape
        _check(lib().ttie_batch_broadphase(self.handle, ctypes.byref(m), tri_off.shape[0] - 1, _ptr(tri_off),
                                           _ptr(x_end), _ptr(pairs), capacity, _ptr(n), _stream()))
        return pairs, n

    def batch_evaluate(self, x, tris, vert_off, pairs, n_pairs=None, precision=FP64, psd=PSD_PER_PART,
                       interval=INTERVAL_EQ1, hessian=True, flags=False, pair_T=False, out=None,
                       vertex_adjacent=False):
        """``evaluate`` over a batch (vert_off: (n_problems + 1,) int64 on the GPU), adding
        ``energies`` (n_problems,) f64: the energy of every problem."""
        assert vert_off.dtype == torch.int64 and vert_off.is_contiguous() and vert_off.device == self.device
        n_prob = vert_off.shape[0] - 1
        out = self._eval_outputs(x, pairs, precision, hessian, flags, pair_T, out)
        if "energies" not in out:
            out["energies"] = torch.zeros(n_prob, dtype=torch.float64, device=self.device)
        m = self._mesh(x, tris)
        if n_pairs is None:
            n_pairs = torch.tensor([pairs.shape[0]], dtype=torch.int64, device=self.device)
        opts = Options(precision, psd, interval, EVAL_VERTEX_ADJACENT if vertex_adjacent else 0)
        cap = out["col_idx"].shape[0] if hessian else 0
        _check(lib().ttie_batch_eval(self.handle, ctypes.byref(m), n_prob, _ptr(vert_off), _ptr(pairs), _ptr(n_pairs),
                                     pairs.shape[0], ctypes.byref(opts), _ptr(out["energies"]),
                                     _ptr(out["energy"]), _ptr(out["grad"]), _ptr(out.get("flags")),
                                     _ptr(out.get("pair_T")), _ptr(out.get("row_ptr")) if hessian else None,
                                     _ptr(out.get("col_idx")) if hessian else None,
                                     _ptr(out.get("vals")) if hessian else None, cap,
                                     _ptr(out.get("n_blocks")) if hessian else None, _ptr(out["n_hits"]), _stream()))
        return out

    def _eval_outputs(self, x, pairs, precision, hessian, flags, pair_T, out):
        dev = self.device
        dt = torch.float64 if precision == FP64 else torch.float32
        nv = x.shape[0]
        if out is None:
            out = {"energy": torch.zeros(1, dtype=torch.float64, device=dev),
                   "grad": torch.empty((nv, 3), dtype=dt, device=dev),
                   "n_hits": torch.zeros(1, dtype=torch.int64, device=dev)}
            if hessian:
                cap = self.limits[4]
                out.update(row_ptr=torch.empty(nv + 1, dtype=torch.int32, device=dev),
                           col_idx=torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                           vals=torch.empty((max(cap, 1), 3, 3), dtype=dt, device=dev),
                           n_blocks=torch.zeros(1, dtype=torch.int64, device=dev))
            if flags:
                out["flags"] = torch.empty(pairs.shape[0], dtype=torch.uint8, device=dev)
            if pair_T:
                out["pair_T"] = torch.empty(pairs.shape[0], dtype=torch.float64, device=dev)
        return out

    def evaluate(self, x, tris, pairs, n_pairs=None, precision=FP64, psd=PSD_PER_PART, interval=INTERVAL_EQ1,
                 hessian=True, flags=False, pair_T=False, out=None, vertex_adjacent=False):
        """Energy, gradient and (optionally) the BSR Hessian.  Returns a dict of GPU tensors:
        energy (1,) f64, grad (N,3), and when hessian: row_ptr, col_idx, vals, n_blocks;
        n_hits; flags (P,) u8 and pair_T (P,) f64 when asked.  With vertex_adjacent, pairs
        sharing exactly one vertex are evaluated instead of being skipped as adjacent."""
        m = self._mesh(x, tris)
        dev = self.device
        if n_pairs is None:
            n_pairs = torch.tensor([pairs.shape[0]], dtype=torch.int64, device=dev)
        out = self._eval_outputs(x, pairs, precision, hessian, flags, pair_T, out)
        opts = Options(precision, psd, interval, EVAL_VERTEX_ADJACENT if vertex_adjacent else 0)
        cap = out["col_idx"].shape[0] if hessian else 0
        _check(lib().ttie_eval(self.handle, ctypes.byref(m), _ptr(pairs), _ptr(n_pairs), pairs.shape[0],
                               ctypes.byref(opts),
                               _ptr(out["energy"]), _ptr(out["grad"]), _ptr(out.get("flags")),
                               _ptr(out.get("pair_T")), _ptr(out.get("row_ptr")) if hessian else None,
                               _ptr(out.get("col_idx")) if hessian else None,
                               _ptr(out.get("vals")) if hessian else None, cap,
                               _ptr(out.get("n_blocks")) if hessian else None, _ptr(out["n_hits"]), _stream()))
        return out

    def evaluate_static(self, x, tris, pairs, n_pairs=None, max_hits=1 << 14, precision=FP64, psd=PSD_PER_PART,
                        interval=INTERVAL_EQ1, hessian=True, flags=False, pair_T=False, out=None, vertex_adjacent=False,
                        block_capacity=None):
        """``evaluate`` through ttie_eval_static: the library's static device array serves as the
        workspace, so the call itself allocates nothing (the output tensors here are the
        caller's; pass ``out`` to reuse them).  Needs no ``reserve``.  The kernels' status (0 or a
        TTIE_ERR_* code) comes back in ``out["status"]`` (1,) int32."""
        m = self._mesh(x, tris)
        dev = self.device
        if n_pairs is None:
            n_pairs = torch.tensor([pairs.shape[0]], dtype=torch.int64, device=dev)
        if out is None:
            dt = torch.float64 if precision == FP64 else torch.float32
            nv = x.shape[0]
            cap = 36 * max_hits if block_capacity is None else block_capacity
            out = {"energy": torch.zeros(1, dtype=torch.float64, device=dev),
                   "grad": torch.empty((nv, 3), dtype=dt, device=dev),
                   "n_hits": torch.zeros(1, dtype=torch.int64, device=dev),
                   "status": torch.zeros(1, dtype=torch.int32, device=dev)}
            if hessian:
                out.update(row_ptr=torch.empty(nv + 1, dtype=torch.int32, device=dev),
                           col_idx=torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                           vals=torch.empty((max(cap, 1), 3, 3), dtype=dt, device=dev),
                           n_blocks=torch.zeros(1, dtype=torch.int64, device=dev))
            if flags:
                out["flags"] = torch.empty(pairs.shape[0], dtype=torch.uint8, device=dev)
            if pair_T:
                out["pair_T"] = torch.empty(pairs.shape[0], dtype=torch.float64, device=dev)
        opts = Options(precision, psd, interval, EVAL_VERTEX_ADJACENT if vertex_adjacent else 0)
        cap = out["col_idx"].shape[0] if hessian else 0
        _check(lib().ttie_eval_static(self.handle, ctypes.byref(m), _ptr(pairs), _ptr(n_pairs), pairs.shape[0], max_hits,
                                      ctypes.byref(opts), _ptr(out["energy"]), _ptr(out["grad"]),
                                      _ptr(out.get("flags")), _ptr(out.get("pair_T")),
                                      _ptr(out.get("row_ptr")) if hessian else None,
                                      _ptr(out.get("col_idx")) if hessian else None,
                                      _ptr(out.get("vals")) if hessian else None, cap,
                                      _ptr(out.get("n_blocks")) if hessian else None, _ptr(out["n_hits"]),
                                      _ptr(out["status"]), _stream()))
        return out

    def bsr_symbolic(self, n_verts, capacity=None):
        """Pattern of the last evaluation's Hessian: (row_ptr (n_verts + 1,) int32, col_idx
        (capacity,) int32, n_blocks (1,) int64), all on the GPU, no synchronization."""
        dev = self.device
        if capacity is None:
            capacity = self.limits[4]
        row_ptr = torch.empty(n_verts + 1, dtype=torch.int32, device=dev)
        col_idx = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        nb = torch.zeros(1, dtype=torch.int64, device=dev)
        _check(lib().ttie_bsr_symbolic(self.handle, _ptr(row_ptr), _ptr(col_idx), capacity, _ptr(nb), _stream()))
        return row_ptr, col_idx, nb

    def bsr_numeric(self, row_ptr, col_idx, dtype, out=None):
        """Values of the last evaluation's Hessian on the pattern (row_ptr, col_idx): a
        (len(col_idx), 3, 3) tensor of ``dtype`` (the evaluation's precision)."""
        if out is None:
            out = torch.empty((max(col_idx.shape[0], 1), 3, 3), dtype=dtype, device=self.device)
        _check(lib().ttie_bsr_numeric(self.handle, _ptr(row_ptr), _ptr(col_idx), _ptr(out), _stream()))
        return out

    @staticmethod
    def hessian(out, n_verts):
        """The BSR Hessian of an ``evaluate`` result as a ``torch.sparse_bsr_tensor`` of size
        (3 n_verts, 3 n_verts) (reads the block count: synchronizes)."""
        nb = int(out["n_blocks"].item())
        return torch.sparse_bsr_tensor(out["row_ptr"], out["col_idx"][:nb], out["vals"][:nb],
                                       size=(3 * n_verts, 3 * n_verts))

    def hits(self, capacity=None):
        """The last evaluation's hits, sorted by (i, j), as numpy arrays (synchronizes): ij, t (t_c^0,
        t_c^1), T, a, b, g (18 each) and M (the Hessian core: M00, M01, M11)."""
        import numpy as np

        if capacity is None:
            capacity = self.limits[3]
        ij = np.zeros((capacity, 2), np.int32)
        tc = np.zeros((capacity, 2))
        T = np.zeros(capacity)
        a = np.zeros((capacity, 18))
        b = np.zeros((capacity, 18))
        g = np.zeros((capacity, 18))
        M = np.zeros((capacity, 3))
        n = ctypes.c_int64(0)
        _check(lib().ttie_get_hits(self.handle, capacity, ij.ctypes.data_as(_vp), tc.ctypes.data_as(_vp),
                                   T.ctypes.data_as(_vp), a.ctypes.data_as(_vp), b.ctypes.data_as(_vp),
                                   g.ctypes.data_as(_vp), M.ctypes.data_as(_vp), ctypes.byref(n), _stream()))
        k = n.value
        return dict(ij=ij[:k], t=tc[:k], T=T[:k], a=a[:k], b=b[:k], g=g[:k], M=M[:k])

    def hvp(self, x, tris, v, mode=HVP_EXACT, out=None):
        """H v at the last evaluation's positions (v in the evaluation's precision)."""
        m = self._mesh(x, tris)
        if out is None:
            out = torch.empty_like(v)
        _check(lib().ttie_hvp(self.handle, ctypes.byref(m), _ptr(v), _ptr(out), mode, _stream()))
        return out

    def pcg(self, row_ptr, col_idx, vals, b, scale=1.0, mu_rel=1e-3, max_iter=50, tol=1e-6, out=None, info=None):
        """Jacobi-PCG on (H + mu I) x = scale * b on the device; returns (x, info) with info a
        (4,) float64 GPU tensor {iterations, relative residual, mu, x . (scale b)}."""
        precision = FP64 if vals.dtype == torch.float64 else MIXED
        if out is None:
            out = torch.empty_like(b)
        if info is None:
            info = torch.zeros(4, dtype=torch.float64, device=b.device)
        _check(lib().ttie_pcg(self.handle, row_ptr.shape[0] - 1, _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(b),
                              float(scale), _ptr(out), float(mu_rel), int(max_iter), float(tol), precision, _ptr(info),
                              _stream()))
        return out, info

    def pcg_mf(self, b, scale=1.0, mu_rel=1e-3, max_iter=50, tol=1e-6, out=None, info=None):
        """Matrix-free Jacobi-PCG with the PSD Hessian of the last evaluation (no BSR matrix);
        b in that evaluation's precision.  Returns (x, info) like ``pcg``."""
        if out is None:
            out = torch.empty_like(b)
        if info is None:
            info = torch.zeros(4, dtype=torch.float64, device=b.device)
        _check(lib().ttie_pcg_mf(self.handle, b.shape[0], _ptr(b), float(scale), _ptr(out), float(mu_rel),
                                 int(max_iter), float(tol), _ptr(info), _stream()))
        return out, info

    def springs_pattern(self, tris, n_verts, capacity=None):
        """The 3x3-block CSR pattern of the springs' Hessian on the mesh's edge graph: returns
        (row_ptr (n_verts + 1,) int32, col_idx (n_blocks,) int32) on the GPU (synchronizes to size
        col_idx).  Invalidates the last evaluation."""
        dev = self.device
        x_dummy = torch.zeros((n_verts, 3), dtype=torch.float64, device=dev)
        m = self._mesh(x_dummy, tris)
        if capacity is None:
            capacity = 6 * tris.shape[0] + n_verts
        row_ptr = torch.empty(n_verts + 1, dtype=torch.int32, device=dev)
        col_idx = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        nb = torch.zeros(1, dtype=torch.int64, device=dev)
        _check(lib().ttie_springs_pattern(self.handle, ctypes.byref(m), _ptr(row_ptr), _ptr(col_idx), capacity,
                                          _ptr(nb), _stream()))
        self.check()
        return row_ptr, col_idx[: int(nb.item())]

    def qs_eval(self, row_ptr, col_idx, x, rest, x_prev, k, m, w, e_ttie=None, g_ttie=None, grad=True, vals=True,
                out=None):
        """Objective of a quasi-static step (springs + w E + proximal term): returns a dict with
        ``phi`` (1,) f64 and, when asked, ``grad`` (N, 3) and ``vals`` (n_blocks, 3, 3), all f64."""
        dev = self.device
        n = x.shape[0]
        if out is None:
            out = {"phi": torch.zeros(1, dtype=torch.float64, device=dev)}
            if grad:
                out["grad"] = torch.empty((n, 3), dtype=torch.float64, device=dev)
            if vals:
                out["vals"] = torch.empty((col_idx.shape[0], 3, 3), dtype=torch.float64, device=dev)
        _check(lib().ttie_qs_eval(self.handle, n, _ptr(row_ptr), _ptr(col_idx), _ptr(x), _ptr(rest), _ptr(x_prev),
                                  float(k), float(m), float(w), _ptr(e_ttie), _ptr(g_ttie), _ptr(out["phi"]),
                                  _ptr(out.get("grad")) if grad else None, _ptr(out.get("vals")) if vals else None,
                                  _stream()))
        return out

    def pcg_coupled(self, row_ptr, col_idx, vals, w, b, scale=1.0, mu=0.0, max_iter=50, tol=1e-6, out=None, info=None):
        """Jacobi-PCG on (K + w H + mu I) x = scale * b, K in BSR (f64), H the PSD Hessian of the
        last (FP64) evaluation.  Returns (x, info) like ``pcg``."""
        if out is None:
            out = torch.empty_like(b)
        if info is None:
            info = torch.zeros(4, dtype=torch.float64, device=b.device)
        _check(lib().ttie_pcg_coupled(self.handle, b.shape[0], _ptr(row_ptr), _ptr(col_idx), _ptr(vals), float(w),
                                      _ptr(b), float(scale), _ptr(out), float(mu), int(max_iter), float(tol),
                                      _ptr(info), _stream()))
        return out, info

    def axpy(self, x, alpha, d, out=None):
        """out = x + alpha * d (x, out float64 positions; d in either precision)."""
        precision = FP64 if d.dtype == torch.float64 else MIXED
        if out is None:
            out = torch.empty_like(x)
        _check(lib().ttie_axpy(self.handle, x.shape[0], float(alpha), _ptr(x), _ptr(d), _ptr(out), precision, _stream()))
        return out

    def set_param(self, param, value):
        """Sets a launch parameter (PARAM_*); 0 restores its default.  Results do not change."""
        _check(lib().ttie_set_param(self.handle, int(param), int(value)))

    def get_param(self, param):
        v = ctypes.c_int64(0)
        _check(lib().ttie_get_param(self.handle, int(param), ctypes.byref(v)))
        return v.value

    def set_timing(self, stages=None):
        """Enables the stage timers for the named stages (None: all, []: none)."""
        names = STAGES if stages is None else stages
        mask = 0
        for nm in names:
            mask |= 1 << STAGES.index(nm)
        _check(lib().ttie_set_timing(self.handle, mask))

    def read_timers(self):
        """{stage: (launches, total_ms)} since the last read (synchronizes on the events)."""
        import numpy as np

        n = np.zeros(len(STAGES), np.int64)
        ms = np.zeros(len(STAGES))
        _check(lib().ttie_read_timers(self.handle, len(STAGES), n.ctypes.data_as(_vp), ms.ctypes.data_as(_vp)))
        return {s: (int(n[k]), float(ms[k])) for k, s in enumerate(STAGES) if n[k] > 0}

    def bsr_mv(self, row_ptr, col_idx, vals, xin, out=None):
        precision = FP64 if vals.dtype == torch.float64 else MIXED
        if out is None:
            out = torch.empty_like(xin)
        _check(lib().ttie_bsr_mv(self.handle, row_ptr.shape[0] - 1, _ptr(row_ptr), _ptr(col_idx), _ptr(vals),
                                 _ptr(xin), _ptr(out), precision, _stream()))
        return out


# ---- module-level calls (one context per device, sized on demand) -------------------------
_contexts = {}


def _context(device, n_verts, n_tris, n_pairs):
    idx = device.index if device.index is not None else torch.cuda.current_device()
    c = _contexts.get(idx)
    if c is None:
        c = _contexts[idx] = Context(idx)
    c.reserve(max(n_verts, 1), max(n_tris, 1), max(n_pairs, 1), max_hits=max(1024, min(max(n_pairs, 1), 1 << 20)))
    return c


def broadphase(x, tris, method=BROAD_LBVH, max_pairs=None):
    """Candidate pairs of the mesh as an (n_pairs, 2) int32 GPU tensor (reads the count:
    synchronizes).  ``max_pairs`` bounds the list (default 64 per triangle)."""
    if max_pairs is None:
        max_pairs = 64 * max(tris.shape[0], 1)
    c = _context(x.device, x.shape[0], tris.shape[0], max_pairs)
    pairs, n = c.broadphase(x, tris, method, capacity=max_pairs)
    c.check()
    return pairs[: int(n.item())]


def evaluate(x, tris, pairs, precision=FP64, psd=PSD_PER_PART, interval=INTERVAL_EQ1):
    """(E, G, H) over a candidate list: the energy (float64 scalar tensor), the gradient (N, 3)
    and the PSD Hessian as a ``torch.sparse_bsr_tensor`` of size (3N, 3N) with 3 x 3 blocks
    (synchronizes to size H and to check the status word)."""
    c = _context(x.device, x.shape[0], tris.shape[0], pairs.shape[0])
    out = c.evaluate(x, tris, pairs, precision=precision, psd=psd, interval=interval)
    c.check()
    return out["energy"][0], out["grad"], Context.hessian(out, x.shape[0])
