"""ctypes declarations of the C ABI in include/h2vie.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libh2vie.so")

H2_OK, H2_NOT_CONVERGED = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARG", -2: "BAD_DESC", -3: "DEVICE", -4: "OOM",
          -5: "BAD_HANDLE", -6: "NUMERIC"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2}
OP = {"G": 0, "Z": 1}


class H2Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class HostDesc(C.Structure):
    _fields_ = [
        ("n_vox", C.c_int64), ("ncomp", C.c_int32), ("n_clusters", C.c_int32),
        ("perm", C.c_void_p), ("level", C.c_void_p), ("parent", C.c_void_p), ("begin", C.c_void_p),
        ("end", C.c_void_p), ("first_child", C.c_void_p), ("nchild", C.c_void_p), ("rank", C.c_void_p),
        ("basis_off", C.c_void_p), ("basis", C.c_void_p), ("basis_len", C.c_int64),
        ("transfer_off", C.c_void_p), ("transfer", C.c_void_p), ("transfer_len", C.c_int64),
        ("n_far", C.c_int64), ("far_t", C.c_void_p), ("far_s", C.c_void_p), ("far_off", C.c_void_p),
        ("coupling", C.c_void_p), ("coupling_len", C.c_int64),
        ("n_near", C.c_int64), ("near_t", C.c_void_p), ("near_s", C.c_void_p), ("near_off", C.c_void_p),
        ("near_blocks", C.c_void_p), ("near_len", C.c_int64),
        ("chi", C.c_void_p), ("k", C.c_double), ("volume", C.c_double), ("sigma", C.c_double),
    ]


class BuildOpts(C.Structure):
    _fields_ = [("max_rhs", C.c_int32), ("tiers", C.c_int32), ("flags", C.c_int32), ("pad", C.c_int32)]


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_matvec", C.c_int32), ("tol", C.c_double),
                ("precision", C.c_int32), ("inner_tol", C.c_double), ("max_outer", C.c_int32),
                ("precond", C.c_int32), ("use_x0", C.c_int32)]


class MlpDims(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hidden", C.c_int32), ("n_out", C.c_int32)]


PRECOND = {"none": 0, "blockdiag": 1, "mlp": 2, "mlp_restart": 3}


class GmresReport(C.Structure):
    _fields_ = [("converged", C.c_int32), ("iterations", C.c_int32), ("matvecs", C.c_int32),
                ("restarts", C.c_int32), ("outer", C.c_int32), ("rel_residual", C.c_double),
                ("corrections", C.c_int32), ("reorth", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_vox", C.c_int64), ("n_clusters", C.c_int64), ("n_leaves", C.c_int64), ("n_far", C.c_int64),
                ("n_near", C.c_int64), ("depth", C.c_int64), ("near_elems", C.c_int64),
                ("coupling_elems", C.c_int64), ("basis_elems", C.c_int64), ("transfer_elems", C.c_int64),
                ("coef_rows", C.c_int64), ("max_rank", C.c_int32), ("min_leaf_rank", C.c_int32),
                ("dev_bytes", C.c_int64), ("bytes_fp64", C.c_double), ("flops_fp64", C.c_double),
                ("near_stored_elems", C.c_int64), ("near_unique", C.c_int64), ("near_passes", C.c_int64),
                ("coupling_owned_elems", C.c_int64), ("coupling_owned_cols", C.c_int64),
                ("near_tiles", C.c_int64), ("near_tile_steps", C.c_int64)]


_LIB = None


def load() -> C.CDLL:
    """Load the built library; raises if it is missing (there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libh2vie.so not built ({LIB_PATH}); run paper_1703_01175_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    lib.h2_last_error.restype = C.c_char_p
    lib.h2_last_error.argtypes = []
    lib.h2_plan_from_host.restype = C.c_int
    lib.h2_plan_from_host.argtypes = [C.POINTER(HostDesc), C.POINTER(BuildOpts), C.POINTER(sz)]
    lib.h2_build_from_host.restype = C.c_int
    lib.h2_build_from_host.argtypes = [C.POINTER(HostDesc), C.POINTER(BuildOpts), vp, sz, vp, C.POINTER(vp)]
    lib.h2_matvec.restype = C.c_int
    lib.h2_matvec.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_int64, C.c_int64, vp]
    lib.h2_gmres_workspace.restype = C.c_int
    lib.h2_gmres_workspace.argtypes = [vp, C.POINTER(GmresOpts), C.POINTER(sz)]
    lib.h2_gmres_solve.restype = C.c_int
    lib.h2_gmres_solve.argtypes = [vp, vp, vp, C.POINTER(GmresOpts), C.POINTER(GmresReport), vp, sz, vp]
    lib.h2_gmres_batch_workspace.restype = C.c_int
    lib.h2_gmres_batch_workspace.argtypes = [vp, C.c_int64, C.c_int64, C.POINTER(GmresOpts), C.POINTER(sz)]
    lib.h2_gmres_solve_batch.restype = C.c_int
    lib.h2_gmres_solve_batch.argtypes = [vp, C.c_int64, vp, vp, C.c_int64, C.POINTER(GmresOpts),
                                         C.POINTER(GmresReport), vp, sz, vp]
    lib.h2_bicgstab_workspace.restype = C.c_int
    lib.h2_bicgstab_workspace.argtypes = [vp, C.POINTER(sz)]
    lib.h2_bicgstab_solve.restype = C.c_int
    lib.h2_bicgstab_solve.argtypes = [vp, vp, vp, C.c_double, C.c_int32, C.POINTER(GmresReport), vp, sz, vp]
    lib.h2_bicgstab_static_bytes.restype = sz
    lib.h2_bicgstab_static_bytes.argtypes = []
    lib.h2_bicgstab_solve_static.restype = C.c_int
    lib.h2_bicgstab_solve_static.argtypes = [vp, vp, vp, C.c_double, C.c_int32, C.POINTER(GmresReport), vp]
    lib.h2_stats.restype = C.c_int
    lib.h2_stats.argtypes = [vp, C.POINTER(Stats)]
    lib.h2_group_plan.restype = C.c_int
    lib.h2_group_plan.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(sz)]
    lib.h2_group_build.restype = C.c_int
    lib.h2_group_build.argtypes = [C.POINTER(vp), C.c_int32, vp, sz, vp, C.POINTER(vp)]
    lib.h2_group_matvec.restype = C.c_int
    lib.h2_group_matvec.argtypes = [vp, C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64), vp]
    lib.h2_group_tune.restype = C.c_int
    lib.h2_group_tune.argtypes = [vp, C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64), vp, C.POINTER(C.c_int32)]
    lib.h2_group_set.restype = C.c_int
    lib.h2_group_set.argtypes = [vp, C.c_int32, C.c_int32]
    lib.h2_group_destroy.restype = None
    lib.h2_group_destroy.argtypes = [vp]
    lib.h2_profile_enable.restype = C.c_int
    lib.h2_profile_enable.argtypes = [vp, C.c_int]
    lib.h2_profile_read.restype = C.c_int
    lib.h2_profile_read.argtypes = [vp, vp]
    lib.h2_near_mode.restype = C.c_int
    lib.h2_near_mode.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.h2_coupling_mode.restype = C.c_int
    lib.h2_near_tiles.restype = C.c_int
    lib.h2_near_tiles.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.h2_coupling_mode.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    pd = C.POINTER(MlpDims)
    for name, args in [
        ("h2_mlp_sizes", [pd, C.c_int64, C.POINTER(sz), C.POINTER(sz)]),
        ("h2_mlp_set", [pd, vp, vp, vp]),
        ("h2_mlp_get", [pd, vp, vp, vp]),
        ("h2_mlp_forward", [pd, vp, vp, vp, C.c_int64, vp, sz, vp]),
        ("h2_mlp_grad", [pd, vp, vp, vp, C.c_int64, vp, vp, vp, sz, vp]),
        ("h2_mlp_train", [pd, vp, vp, vp, C.c_int64, vp, C.c_int32, C.c_int32, C.c_float, vp, vp, sz, vp]),
        ("h2_leaf_count", [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        ("h2_leaf_features", [vp, C.c_int32, vp, vp, vp, vp]),
        ("h2_leaf_halo", [vp, vp, C.c_int32]),
        ("h2_leaf_targets", [vp, C.c_int32, vp, vp, vp, vp, vp]),
        ("h2_precond_blockdiag_bytes", [vp, C.POINTER(sz)]),
        ("h2_precond_blockdiag", [vp, vp, sz, vp]),
        ("h2_precond_mlp", [vp, pd, C.c_int32, vp, C.c_int32]),
        ("h2_precond_apply_bytes", [vp, C.c_int32, C.POINTER(sz)]),
        ("h2_precond_apply", [vp, C.c_int32, vp, vp, vp, sz, vp]),
    ]:
        f = getattr(lib, name)
        f.restype = C.c_int
        f.argtypes = args
    lib.h2_destroy.restype = None
    lib.h2_destroy.argtypes = [vp]
    _LIB = lib
    return lib


def check(status: int, allow=(H2_OK,)) -> int:
    if status in allow:
        return status
    raise H2Error(status, load().h2_last_error().decode())


_DTYPES = dict(perm=np.int64, level=np.int32, parent=np.int32, begin=np.int64, end=np.int64,
               first_child=np.int32, nchild=np.int32, rank=np.int32, basis_off=np.int64, basis=np.complex128,
               transfer_off=np.int64, transfer=np.complex128, far_t=np.int32, far_s=np.int32, far_off=np.int64,
               coupling=np.complex128, near_t=np.int32, near_s=np.int32, near_off=np.int64,
               near=np.complex128, chi=np.complex128)


def host_desc(d):
    """HostDesc for an h2gen.H2Desc; returns (struct, arrays to keep alive)."""
    keep = {}
    for name, dt in _DTYPES.items():
        a = np.ascontiguousarray(getattr(d, name), dtype=dt)
        if a.size == 0:
            a = np.zeros(1, dtype=dt)
        keep[name] = a
    p = {k: v.ctypes.data for k, v in keep.items()}
    hd = HostDesc(n_vox=int(d.n_vox), ncomp=int(d.ncomp), n_clusters=int(d.level.shape[0]),
                  perm=p["perm"], level=p["level"], parent=p["parent"], begin=p["begin"], end=p["end"],
                  first_child=p["first_child"], nchild=p["nchild"], rank=p["rank"],
                  basis_off=p["basis_off"], basis=p["basis"], basis_len=int(np.asarray(d.basis).size),
                  transfer_off=p["transfer_off"], transfer=p["transfer"],
                  transfer_len=int(np.asarray(d.transfer).size),
                  n_far=int(np.asarray(d.far_t).size), far_t=p["far_t"], far_s=p["far_s"], far_off=p["far_off"],
                  coupling=p["coupling"], coupling_len=int(np.asarray(d.coupling).size),
                  n_near=int(np.asarray(d.near_t).size), near_t=p["near_t"], near_s=p["near_s"],
                  near_off=p["near_off"], near_blocks=p["near"], near_len=int(np.asarray(d.near).size),
                  chi=p["chi"], k=float(d.k), volume=float(d.volume), sigma=float(d.sigma))
    return hd, keep
