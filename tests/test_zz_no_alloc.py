"""The BiCGStab entry point that allocates nothing (workspace in the library's
device array) against the allocating one, through the C ABI: two calls in a row
on one device, the second on a smaller system, each bit for bit equal to the
allocating solve and judged by the oracle's FP64 residual."""
import numpy as np
import pytest

import h2gen
from conftest import built
from oracle import matvec as om

pytestmark = pytest.mark.gpu


def test_static_bicgstab_matches_allocating_solve_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1703_01175_amd import H2Operator, _lib
    lib = _lib.load()
    assert lib.h2_bicgstab_static_bytes() == 128 << 20
    for name, seed in (("cube12", 21), ("cube8", 22)):          # the second system is smaller
        print(f"[gpu] static bicgstab {name}", flush=True)
        g, d = built(name)
        H = H2Operator(d, tiers=("fp64",))
        b = torch.from_numpy(h2gen.plane_wave(g, seed)[0]).cuda()
        x_ref, rep_ref = H.bicgstab(b, tol=1e-8)
        x_st, rep_st = H.bicgstab(b, tol=1e-8, static=True)
        torch.cuda.synchronize()
        assert rep_st.converged and rep_ref.converged
        assert (rep_st.iterations, rep_st.matvecs) == (rep_ref.iterations, rep_ref.matvecs)
        assert rep_st.rel_residual == rep_ref.rel_residual
        assert torch.equal(x_st, x_ref)
        bn = b.cpu().numpy()
        res = np.linalg.norm(bn - om.h2_matvec(d, x_st.cpu().numpy())) / np.linalg.norm(bn)
        assert res <= 1.0001e-8
        H.close()
