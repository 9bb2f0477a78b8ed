"""GPU GMRES / GMRES-IR through the C ABI, judged by the oracle's FP64 residual."""
import numpy as np
import pytest

import h2gen
from conftest import built
from oracle import krylov
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
        _OPS[name] = (g, d, H2Operator(d, tiers=("fp64", "fp32")))
    return _OPS[name]


def _true_res(d, x, b):
    return float(np.linalg.norm(b - om.h2_matvec(d, x)) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["cube12", "rod", "cube16"])
def test_gmres_fp64_converges(torch, name):
    print(f"[gpu] gmres fp64 {name}", flush=True)
    g, d, H = operator(name)
    b = h2gen.plane_wave(g, 2)[0]
    x, rep = H.gmres(torch.from_numpy(b).cuda(), tol=1e-6)
    x = x.cpu().numpy()
    assert rep.converged and rep.rel_residual <= 1e-6
    assert _true_res(d, x, b) <= 1.0001e-6


@pytest.mark.parametrize("name", ["rod", "cube12", "rod_sym"])
def test_gmres_iterations_match_oracle(torch, name):
    # the oracle's Arnoldi takes the device's selective second pass (DGKS): the same
    # iteration count and the same number of second passes
    g, d, H = operator(name)
    Z = om.densify(d)
    b = h2gen.random_vector(3 * g.n_vox, 8)
    for restart in (50, 4):
        x, rep = H.gmres(torch.from_numpy(b).cuda(), tol=1e-8, restart=restart)
        xo, ro = krylov.gmres(lambda v: Z @ v, b, tol=1e-8, restart=restart)
        print(f"[gpu] gmres {name} m={restart}: device {rep.iterations} its {rep.reorth} reorth, "
              f"oracle {ro.iterations} its {ro.reorth} reorth", flush=True)
        assert rep.iterations == ro.iterations and rep.reorth == ro.reorth
        assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-6 * np.linalg.norm(xo)


def test_gmres_ir_fp32(torch):
    g, d, H = operator("cube12")
    b = h2gen.plane_wave(g, 4)[0]
    x, rep = H.gmres(torch.from_numpy(b).cuda(), tol=1e-6, precision="fp32", inner_tol=1e-3)
    assert rep.converged and rep.outer >= 1
    assert _true_res(d, x.cpu().numpy(), b) <= 1.0001e-6


def test_gmres_ir_bf16x3_single_rhs(torch):
    """BF16x3 products (matrix cores, one column) inside the refinement of a single solve."""
    from paper_1703_01175_amd import H2Operator
    g, d = built("cube12")
    H = H2Operator(d, tiers=("fp64", "bf16x3"), max_rhs=1)
    b = h2gen.plane_wave(g, 5)[0]
    x, rep = H.gmres(torch.from_numpy(b).cuda(), tol=1e-9, precision="bf16x3", inner_tol=1e-3)
    assert rep.converged and rep.outer >= 2
    assert _true_res(d, x.cpu().numpy(), b) <= 1.0001e-9
    H.close()
    # without the tier the request is refused
    _, _, H64 = operator("cube12")
    with pytest.raises(Exception):
        H64.gmres(torch.from_numpy(b).cuda(), precision="bf16x3")


def test_gmres_zero_rhs(torch):
    g, d, H = operator("rod")
    b = torch.zeros(3 * g.n_vox, dtype=torch.complex128, device="cuda")
    x, rep = H.gmres(b)
    assert rep.converged and rep.iterations == 0 and float(x.abs().max()) == 0.0


def test_gmres_nan_rhs(torch):
    from paper_1703_01175_amd import H2Error
    g, d, H = operator("rod")
    b = torch.from_numpy(h2gen.random_vector(3 * g.n_vox, 1)).cuda()
    b[5] = float("nan")
    with pytest.raises(H2Error) as e:
        H.gmres(b)
    assert e.value.status == -6


def test_gmres_budget_exhausted(torch):
    g, d, H = operator("cube12")
    b = h2gen.random_vector(3 * g.n_vox, 3)
    x, rep = H.gmres(torch.from_numpy(b).cuda(), tol=1e-12, restart=3, max_matvec=7)
    assert not rep.converged and rep.matvecs <= 8
    assert rep.rel_residual == pytest.approx(_true_res(d, x.cpu().numpy(), b), rel=1e-6)
