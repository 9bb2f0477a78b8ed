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
    corrections: int = 0
    reorth: int = 0           # Arnoldi steps that took a second Gram-Schmidt pass


class H2Operator:
    """Device copy of an h2gen.H2Desc; matvec(x) applies Z (or G) on the GPU."""

    def __init__(self, desc, tiers=("fp64",), max_rhs: int = 1, device: str = "cuda", stream=None,
                 keep_all_near: bool = False):
        import torch
        self.lib = _lib.load()
        self.N = 3 * int(desc.n_vox)
        self.n_vox = int(desc.n_vox)
        hd, keep = _lib.host_desc(desc)
        mask = 0
        for t in tiers:
            mask |= _TIER_BITS[t]
        self.tiers = tuple(tiers)
        opts = _lib.BuildOpts(max_rhs=int(max_rhs), tiers=mask, flags=1 if keep_all_near else 0)
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
              precision: str = "fp64", inner_tol: float = 1e-3, max_outer: int = 30, precond: str = "none",
              x0=None, stream=None):
        """Solve Z x = b (x0 = 0, or resume from x0); precond "blockdiag"/"mlp" gives flexible GMRES."""
        import torch
        if b.dtype != torch.complex128 or not b.is_cuda or b.shape != (self.N,):
            raise ValueError("b must be a complex128 CUDA tensor of length N")
        if x is None:
            x = torch.empty_like(b)
        use_x0 = 0
        if x0 is not None:
            x.copy_(x0)
            use_x0 = 1
        opts = _lib.GmresOpts(restart=restart, max_matvec=max_matvec, tol=tol, precision=_lib.PRECISION[precision],
                              inner_tol=inner_tol, max_outer=max_outer, precond=_lib.PRECOND[precond], use_x0=use_x0)
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.h2_gmres_workspace(self.handle, C.byref(opts), C.byref(nbytes)))
        work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        rep = _lib.GmresReport()
        st = self.lib.h2_gmres_solve(self.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(opts),
                                     C.byref(rep), C.c_void_p(work.data_ptr()), nbytes, _stream_ptr(stream))
        _lib.check(st, allow=(_lib.H2_OK, _lib.H2_NOT_CONVERGED))
        return x, GmresResult(bool(rep.converged), rep.iterations, rep.matvecs, rep.restarts, rep.outer,
                              rep.rel_residual, rep.corrections, rep.reorth)

    def bicgstab(self, b, x=None, tol: float = 1e-6, max_matvec: int = 10000, stream=None, static: bool = False):
        """Solve Z x = b by FP64 BiCGStab on the device (x0 = 0).  static=True takes the
        entry point that allocates nothing (workspace in the library's device array)."""
        import torch
        if b.dtype != torch.complex128 or not b.is_cuda or b.shape != (self.N,):
            raise ValueError("b must be a complex128 CUDA tensor of length N")
        if x is None:
            x = torch.empty_like(b)
        rep = _lib.GmresReport()
        if static:
            st = self.lib.h2_bicgstab_solve_static(self.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                                   float(tol), int(max_matvec), C.byref(rep), _stream_ptr(stream))
        else:
            nbytes = C.c_size_t(0)
            _lib.check(self.lib.h2_bicgstab_workspace(self.handle, C.byref(nbytes)))
            work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            st = self.lib.h2_bicgstab_solve(self.handle, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                            float(tol), int(max_matvec), C.byref(rep), C.c_void_p(work.data_ptr()),
                                            nbytes, _stream_ptr(stream))
        _lib.check(st, allow=(_lib.H2_OK, _lib.H2_NOT_CONVERGED))
        return x, GmresResult(bool(rep.converged), rep.iterations, rep.matvecs, rep.restarts, rep.outer,
                              rep.rel_residual)

    def gmres_batch(self, B, X=None, tol: float = 1e-6, restart: int = 30, max_matvec: int = 10000,
                    precision: str = "fp64", inner_tol: float = 1e-3, max_outer: int = 30, precond: str = "none",
                    X0=None, stream=None):
        """Solve Z x_c = b_c for the rows of B (n_rhs, N) complex128 in lockstep; every
        product is one multi-column product.  Returns X and one GmresResult per row."""
        import torch
        if B.dtype != torch.complex128 or not B.is_cuda or B.dim() != 2 or B.shape[1] != self.N:
            raise ValueError("B must be a complex128 CUDA tensor of shape (n_rhs, N)")
        B = B.contiguous()
        n = int(B.shape[0])
        if X is None:
            X = torch.empty_like(B)
        use_x0 = 0
        if X0 is not None:
            X.copy_(X0)
            use_x0 = 1
        opts = _lib.GmresOpts(restart=restart, max_matvec=max_matvec, tol=tol, precision=_lib.PRECISION[precision],
                              inner_tol=inner_tol, max_outer=max_outer, precond=_lib.PRECOND[precond], use_x0=use_x0)
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.h2_gmres_batch_workspace(self.handle, n, self.N, C.byref(opts), C.byref(nbytes)))
        work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        reps = (_lib.GmresReport * n)()
        st = self.lib.h2_gmres_solve_batch(self.handle, n, C.c_void_p(B.data_ptr()), C.c_void_p(X.data_ptr()), self.N,
                                           C.byref(opts), reps, C.c_void_p(work.data_ptr()), nbytes,
                                           _stream_ptr(stream))
        _lib.check(st, allow=(_lib.H2_OK, _lib.H2_NOT_CONVERGED))
        return X, [GmresResult(bool(r.converged), r.iterations, r.matvecs, r.restarts, r.outer, r.rel_residual,
                               r.corrections, r.reorth) for r in reps]

    # ------------------------------------------------------------------ per-leaf preconditioners
    def leaf_count(self):
        n, m = C.c_int32(0), C.c_int32(0)
        _lib.check(self.lib.h2_leaf_count(self.handle, C.byref(n), C.byref(m)))
        return int(n.value), int(m.value)

    def set_halo(self, nbr):
        """Neighbour-leaf table (n_leaves, slots) int32, -1 for none; None removes the halo."""
        import numpy as np
        if nbr is None:
            _lib.check(self.lib.h2_leaf_halo(self.handle, None, 0))
            self.halo_slots = 0
            return
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        _lib.check(self.lib.h2_leaf_halo(self.handle, C.c_void_p(nbr.ctypes.data), int(nbr.shape[1])))
        self.halo_slots = int(nbr.shape[1])

    def features(self, r, n_pad: int, stream=None):
        """(n_leaves, 7 n_pad + 6 halo slots) float32 features of a residual r (complex128, length N)."""
        import torch
        nl, _ = self.leaf_count()
        X = torch.empty((nl, 7 * n_pad + 6 * getattr(self, "halo_slots", 0)), dtype=torch.float32, device=self.device)
        scratch = torch.empty(64, dtype=torch.uint8, device=self.device)
        _lib.check(self.lib.h2_leaf_features(self.handle, n_pad, C.c_void_p(r.data_ptr()), C.c_void_p(X.data_ptr()),
                                             C.c_void_p(scratch.data_ptr()), _stream_ptr(stream)))
        return X

    def targets(self, e, r, n_pad: int, stream=None):
        """(n_leaves, 6 n_pad) float32 targets [Re e_t, Im e_t] / s, s from ||r||."""
        import torch
        nl, _ = self.leaf_count()
        T = torch.empty((nl, 6 * n_pad), dtype=torch.float32, device=self.device)
        scratch = torch.empty(64, dtype=torch.uint8, device=self.device)
        _lib.check(self.lib.h2_leaf_targets(self.handle, n_pad, C.c_void_p(e.data_ptr()), C.c_void_p(r.data_ptr()),
                                            C.c_void_p(T.data_ptr()), C.c_void_p(scratch.data_ptr()),
                                            _stream_ptr(stream)))
        return T

    def precond_blockdiag(self, stream=None):
        import torch
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.h2_precond_blockdiag_bytes(self.handle, C.byref(nbytes)))
        self.bd_buf = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        _lib.check(self.lib.h2_precond_blockdiag(self.handle, C.c_void_p(self.bd_buf.data_ptr()), nbytes,
                                                 _stream_ptr(stream)))

    def precond_apply(self, r, which: str = "blockdiag", stream=None):
        """z = P(r) with an attached preconditioner (complex128 device vectors)."""
        import torch
        pc = _lib.PRECOND[which]
        nbytes = C.c_size_t(0)
        _lib.check(self.lib.h2_precond_apply_bytes(self.handle, pc, C.byref(nbytes)))
        work = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=self.device)
        z = torch.empty_like(r)
        _lib.check(self.lib.h2_precond_apply(self.handle, pc, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()),
                                             C.c_void_p(work.data_ptr()), nbytes, _stream_ptr(stream)))
        return z

    def attach_mlp(self, mlp, base: str = "none"):
        """Use `mlp` for precond="mlp"; base "blockdiag" adds its output to the block-diagonal solve."""
        _lib.check(self.lib.h2_precond_mlp(self.handle, C.byref(mlp.dims), mlp.n_pad, C.c_void_p(mlp.params.data_ptr()),
                                           _lib.PRECOND[base]))
        self.mlp = mlp

    # ------------------------------------------------------------------ misc
    def near_tiles(self, on: bool | None = None) -> tuple[bool, bool]:
        """(tiled near field in use, tiles available); on=True/False selects it."""
        cur, avail = C.c_int32(0), C.c_int32(0)
        _lib.check(self.lib.h2_near_tiles(self.handle, -1 if on is None else int(bool(on)),
                                          C.byref(cur), C.byref(avail)))
        return bool(cur.value), bool(avail.value)

    def near_mode(self, symmetric: bool | None = None) -> tuple[bool, bool]:
        """(symmetric mode in use, symmetric mode available); symmetric=True/False selects it."""
        mode, avail = C.c_int32(0), C.c_int32(0)
        _lib.check(self.lib.h2_near_mode(self.handle, -1 if symmetric is None else int(bool(symmetric)),
                                         C.byref(mode), C.byref(avail)))
        return bool(mode.value), bool(avail.value)

    def coupling_mode(self, symmetric: bool | None = None) -> tuple[bool, bool]:
        """(symmetric coupling mode in use, available); symmetric=True/False selects it."""
        mode, avail = C.c_int32(0), C.c_int32(0)
        _lib.check(self.lib.h2_coupling_mode(self.handle, -1 if symmetric is None else int(bool(symmetric)),
                                             C.byref(mode), C.byref(avail)))
        return bool(mode.value), bool(avail.value)

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


def leaf_neighbors(d, shape):
    """Neighbour table of the leaves (cluster order) on a voxel grid of `shape`:
    slot o in {-1, 0, 1}^3 minus the origin (lexicographic) holds the leaf containing
    the voxel one leaf extent away from the leaf's centre voxel, or -1 off the grid."""
    import numpy as np
    nchild = np.asarray(d.nchild)
    leaves = np.nonzero(nchild == 0)[0]
    perm = np.asarray(d.perm)
    begin, end = np.asarray(d.begin)[leaves], np.asarray(d.end)[leaves]
    xyz = np.stack(np.unravel_index(perm, shape), 1)               # tree order
    order = np.argsort(begin)                                      # leaves tile [0, n_vox) in tree order
    lo, hi = np.empty((leaves.size, 3), np.int64), np.empty((leaves.size, 3), np.int64)
    lo[order] = np.minimum.reduceat(xyz, begin[order], axis=0)
    hi[order] = np.maximum.reduceat(xyz, begin[order], axis=0)
    ext = hi - lo + 1
    owner = np.empty(perm.size, np.int64)                           # leaf number of every voxel
    owner[perm[np.concatenate([np.arange(begin[q], end[q]) for q in order])]] = np.repeat(order, (end - begin)[order])
    offs = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)])
    probe = lo[:, None, :] + offs[None, :, :] * ext[:, None, :] + ((ext - 1) // 2)[:, None, :]
    inside = np.all((probe >= 0) & (probe < np.asarray(shape)), axis=2)
    flat = np.ravel_multi_index(tuple(np.clip(probe, 0, np.asarray(shape) - 1).transpose(2, 0, 1)), shape)
    return np.where(inside, owner[flat], -1).astype(np.int32)


class LeafMLP:
    """The per-leaf MLP: parameters and workspaces in device memory, passes in the library."""

    def __init__(self, n_pad: int, hidden: int = 256, seed: int = 0, batch: int = 512, device: str = "cuda",
                 zero_output: bool = False, halo_slots: int = 0):
        """zero_output: start with a zero last layer (output 0), for a correction on top of another map."""
        import numpy as np
        import torch
        self.lib = _lib.load()
        self.n_pad = int(n_pad)
        self.dims = _lib.MlpDims(7 * n_pad + 6 * halo_slots, hidden, 6 * n_pad)
        self.device = torch.device(device)
        pb, wb = C.c_size_t(0), C.c_size_t(0)
        _lib.check(self.lib.h2_mlp_sizes(C.byref(self.dims), batch, C.byref(pb), C.byref(wb)))
        self.params = torch.empty(int(pb.value), dtype=torch.uint8, device=self.device)
        self.batch = batch
        n_in, h, n_out = self.dims.n_in, hidden, 6 * n_pad
        self.nmaster = h * n_in + h + h * h + h + n_out * h + n_out
        # He-normal initial weights drawn here (seeded) and handed to the library
        rng = np.random.default_rng(seed)
        parts = [rng.standard_normal(h * n_in) * np.sqrt(2.0 / n_in), np.zeros(h),
                 rng.standard_normal(h * h) * np.sqrt(2.0 / h), np.zeros(h),
                 rng.standard_normal(n_out * h) * np.sqrt(1.0 / h) * (0.0 if zero_output else 1.0), np.zeros(n_out)]
        self.set_master(np.concatenate(parts).astype(np.float32))

    def _work(self, n):
        import torch
        wb = C.c_size_t(0)
        _lib.check(self.lib.h2_mlp_sizes(C.byref(self.dims), max(int(n), 1), None, C.byref(wb)))
        return torch.empty(int(wb.value), dtype=torch.uint8, device=self.device), wb

    def set_master(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.nmaster
        _lib.check(self.lib.h2_mlp_set(C.byref(self.dims), C.c_void_p(self.params.data_ptr()),
                                       C.c_void_p(w.ctypes.data), None))

    def master(self):
        import numpy as np
        w = np.empty(self.nmaster, np.float32)
        _lib.check(self.lib.h2_mlp_get(C.byref(self.dims), C.c_void_p(self.params.data_ptr()),
                                       C.c_void_p(w.ctypes.data), None))
        return w

    def forward(self, X):
        import torch
        n = X.shape[0]
        Y = torch.empty((n, self.dims.n_out), dtype=torch.float32, device=self.device)
        work, wb = self._work(n)
        _lib.check(self.lib.h2_mlp_forward(C.byref(self.dims), C.c_void_p(self.params.data_ptr()),
                                           C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), n,
                                           C.c_void_p(work.data_ptr()), wb, _stream_ptr()))
        return Y

    def grad(self, X, T):
        import torch
        n = X.shape[0]
        g = torch.empty(self.nmaster, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        work, wb = self._work(n)
        _lib.check(self.lib.h2_mlp_grad(C.byref(self.dims), C.c_void_p(self.params.data_ptr()),
                                        C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), n,
                                        C.c_void_p(g.data_ptr()), C.c_void_p(loss.data_ptr()),
                                        C.c_void_p(work.data_ptr()), wb, _stream_ptr()))
        return g, loss

    def train(self, X, T, epochs: int = 20, batch: int = 256, lr: float = 1e-3, seed: int = 0):
        """Adam over seeded minibatch permutations (drawn here, handed to the library)."""
        import numpy as np
        import torch
        n = X.shape[0]
        rng = np.random.default_rng(seed)
        order = np.concatenate([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
        order_d = torch.from_numpy(order).to(self.device)
        work, wb = self._work(batch)
        losses = np.zeros(epochs, np.float32)
        _lib.check(self.lib.h2_mlp_train(C.byref(self.dims), C.c_void_p(self.params.data_ptr()),
                                         C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), n,
                                         C.c_void_p(order_d.data_ptr()), epochs, batch, float(lr),
                                         C.c_void_p(losses.ctypes.data), C.c_void_p(work.data_ptr()), wb,
                                         _stream_ptr()))
        return losses
