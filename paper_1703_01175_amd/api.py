"""H2Operator: a built H^2 representation on one GPU, driven through the C ABI."""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

from . import _lib

_TIER_BITS = {"fp64": 1, "fp32": 2, "bf16x3": 4}


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(int(s.cuda_stream))


@dataclass
class GmresResult:
    converged: bool
    iterations: int
    matvecs: int
    restarts: int
    outer: int
    rel_residual: float


class H2Operator:
    """Device copy of an h2gen.H2Desc; matvec(x) applies Z (or G) on the GPU."""

    def __init__(self, desc, tiers=("fp64",), max_rhs: int = 1, device: str = "cuda", stream=None):
        import torch
        self.lib = _lib.load()
        self.N = 3 * int(desc.n_vox)
        self.n_vox = int(desc.n_vox)
        hd, keep = _lib.host_desc(desc)
        mask = 0
        for t in tiers:
            mask |= _TIER_BITS[t]
        self.tiers = tuple(tiers)
        opts = _lib.BuildOpts(max_rhs=int(max_rhs), tiers=mask)
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.h2_plan_from_host(C.byref(hd), C.byref(opts), C.byref(nbytes)))
        self.device = torch.device(device)
        self.buf = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = C.c_void_p(0)
        _lib.check(self.lib.h2_build_from_host(C.byref(hd), C.byref(opts), C.c_void_p(self.buf.data_ptr()),
                                               nbytes, _stream_ptr(stream), C.byref(h)))
        del keep
        self.handle = h
        self.max_rhs = int(max_rhs)

    # ------------------------------------------------------------------ product
    def matvec(self, x, op: str = "Z", precision: str = "fp64", out=None, stream=None):
        """y = op(x) for x of shape (N,) or (n_rhs, N) on the device (complex128 for fp64, complex64 otherwise)."""
        import torch
        dt = torch.complex128 if precision == "fp64" else torch.complex64
        if x.dtype != dt or not x.is_cuda or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous {dt} CUDA tensor")
        if x.shape[-1] != self.N:
            raise ValueError(f"x has {x.shape[-1]} unknowns, operator has {self.N}")
        n_rhs = 1 if x.dim() == 1 else int(x.shape[0])
        if out is None:
            out = torch.empty_like(x)
        _lib.check(self.lib.h2_matvec(self.handle, _lib.OP[op], _lib.PRECISION[precision], C.c_void_p(x.data_ptr()),
                                      C.c_void_p(out.data_ptr()), n_rhs, self.N, _stream_ptr(stream)))
        return out

    # ------------------------------------------------------------------ solver
    def gmres(self, b, x=None, tol: float = 1e-6, restart: int = 50, max_matvec: int = 10000,
              precision: str = "fp64", inner_tol: float = 1e-3, max_outer: int = 30, stream=None):
        import torch
        if b.dtype != torch.complex128 or not b.is_cuda or b.shape != (self.N,):
            raise ValueError("b must be a complex128 CUDA tensor of length N")
        if x is None:
            x = torch.empty_like(b)
        opts = _lib.GmresOpts(restart=restart, max_matvec=max_matvec, tol=tol, precision=_lib.PRECISION[precision],
                              inner_tol=inner_tol, max_outer=max_outer)
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.h2_gmres_workspace(self.handle, C.byref(opts), C.byref(nbytes)))
        work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        rep = _lib.GmresReport()
        st = self.lib.h2_gmres_solve(self.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(opts),
                                     C.byref(rep), C.c_void_p(work.data_ptr()), nbytes, _stream_ptr(stream))
        _lib.check(st, allow=(_lib.H2_OK, _lib.H2_NOT_CONVERGED))
        return x, GmresResult(bool(rep.converged), rep.iterations, rep.matvecs, rep.restarts, rep.outer,
                              rep.rel_residual)

    # ------------------------------------------------------------------ misc
    def stats(self) -> dict:
        s = _lib.Stats()
        _lib.check(self.lib.h2_stats(self.handle, C.byref(s)))
        return {f: getattr(s, f) for f, _ in _lib.Stats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.h2_destroy(self.handle)
            self.handle = C.c_void_p(0)
            self.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class H2Group:
    """Several operators (built with the "bf16x3" tier) applied together: every phase of
    the product runs as one launch over all members, replayed from a HIP graph."""

    def __init__(self, ops, stream=None):
        import torch
        self.ops = list(ops)
        self.lib = _lib.load()
        n = len(self.ops)
        arr = (C.c_void_p * n)(*[o.handle.value for o in self.ops])
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.h2_group_plan(arr, n, C.byref(nbytes)))
        self.buf = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.ops[0].device)
        g = C.c_void_p(0)
        _lib.check(self.lib.h2_group_build(arr, n, C.c_void_p(self.buf.data_ptr()), nbytes, _stream_ptr(stream),
                                           C.byref(g)))
        self.handle = g

    def _args(self, xs, ys):
        import torch
        n = len(self.ops)
        if len(xs) != n or len(ys) != n:
            raise ValueError("one input and one output per member")
        xp = (C.c_void_p * n)()
        yp = (C.c_void_p * n)()
        nr = (C.c_int64 * n)()
        ld = (C.c_int64 * n)()
        for i, (o, x, y) in enumerate(zip(self.ops, xs, ys)):
            if x is None:
                nr[i] = 0
                ld[i] = o.N
                continue
            if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous() or x.shape[-1] != o.N:
                raise ValueError("member vectors must be contiguous complex64 CUDA tensors of length N")
            xp[i] = x.data_ptr()
            yp[i] = y.data_ptr()
            nr[i] = 1 if x.dim() == 1 else int(x.shape[0])
            ld[i] = o.N
        return xp, yp, nr, ld

    def matvec(self, xs, op: str = "Z", outs=None, stream=None):
        import torch
        if outs is None:
            outs = [None if x is None else torch.empty_like(x) for x in xs]
        xp, yp, nr, ld = self._args(xs, outs)
        _lib.check(self.lib.h2_group_matvec(self.handle, _lib.OP[op], xp, yp, nr, ld, _stream_ptr(stream)))
        return outs

    def tune(self, xs, op: str = "Z", outs=None, stream=None) -> int:
        import torch
        if outs is None:
            outs = [None if x is None else torch.empty_like(x) for x in xs]
        xp, yp, nr, ld = self._args(xs, outs)
        tile = C.c_int32(0)
        _lib.check(self.lib.h2_group_tune(self.handle, _lib.OP[op], xp, yp, nr, ld, _stream_ptr(stream),
                                          C.byref(tile)))
        return int(tile.value)

    def set(self, tile: int = 0, graph: bool = True):
        _lib.check(self.lib.h2_group_set(self.handle, int(tile), int(graph)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.h2_group_destroy(self.handle)
            self.handle = C.c_void_p(0)
            self.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
