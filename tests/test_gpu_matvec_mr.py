"""Multi-RHS FP64 / FP32 product (passes of four right-hand sides) through the C ABI:
every column must equal the single-vector product and the oracle's."""
import numpy as np
import pytest

import h2gen
from conftest import built
from oracle import matvec as om

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


_OPS = {}


def operator(name):
    from paper_1703_01175_amd import H2Operator
    if name not in _OPS:
        g, d = built(name)
        _OPS[name] = (g, d, H2Operator(d, tiers=("fp64", "fp32"), max_rhs=8))
    return _OPS[name]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["cube12", "box9", "rod", "cube16", "cube8"])
@pytest.mark.parametrize("n_rhs", [2, 5, 9])
@pytest.mark.parametrize("op", ["Z", "G"])
def test_multi_rhs_fp64_matches_single_and_oracle(torch, name, n_rhs, op):
    print(f"[gpu] multi-RHS fp64 {name} n_rhs={n_rhs} op={op}", flush=True)
    g, d, H = operator(name)
    X = h2gen.random_vector(3 * g.n_vox, 40 + n_rhs, ncols=n_rhs)     # (n_rhs, N)
    Y = H.matvec(torch.from_numpy(X).cuda(), op=op).cpu().numpy()
    for c in range(n_rhs):
        y1 = H.matvec(torch.from_numpy(np.ascontiguousarray(X[c])).cuda(), op=op).cpu().numpy()
        assert _rel(Y[c], y1) <= 1e-13
    for c in (0, n_rhs - 1):
        assert _rel(Y[c], om.h2_matvec(d, X[c], op)) <= 1e-12


def test_multi_rhs_fp32_matches_single(torch):
    g, d, H = operator("cube16")
    X = h2gen.random_vector(3 * g.n_vox, 50, ncols=6).astype(np.complex64)
    Y = H.matvec(torch.from_numpy(X).cuda(), precision="fp32").cpu().numpy()
    for c in range(6):
        y1 = H.matvec(torch.from_numpy(np.ascontiguousarray(X[c])).cuda(), precision="fp32").cpu().numpy()
        assert _rel(Y[c], y1) <= 1e-6
        assert _rel(Y[c], om.h2_matvec(d, X[c].astype(np.complex128))) <= 1e-5


def test_multi_rhs_leading_dimension(torch):
    """Columns with ld > N: only the first N entries of each column are read or written."""
    import ctypes as C
    from paper_1703_01175_amd import _lib
    g, d, H = operator("cube12")
    N = 3 * g.n_vox
    ld = N + 40
    n = 3
    X = h2gen.random_vector(N, 60, ncols=n)
    xb = torch.zeros((n, ld), dtype=torch.complex128, device="cuda")
    xb[:, :N] = torch.from_numpy(X).cuda()
    yb = torch.full((n, ld), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    _lib.check(H.lib.h2_matvec(H.handle, _lib.OP["Z"], _lib.PRECISION["fp64"], C.c_void_p(xb.data_ptr()),
                               C.c_void_p(yb.data_ptr()), n, ld, None))
    torch.cuda.synchronize()
    Y = yb.cpu().numpy()
    assert np.all(Y[:, N:] == 7.0)
    for c in range(n):
        assert _rel(Y[c, :N], om.h2_matvec(d, X[c])) <= 1e-12
