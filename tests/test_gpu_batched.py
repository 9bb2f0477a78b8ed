"""GPU batched BF16x3 tier (matrix cores): products for many right-hand sides and
groups of geometries, against the FP64 oracle and the oracle's tier emulation."""
import numpy as np
import pytest

import h2gen
from conftest import built
from oracle import matvec as om
from oracle import precision as oprec

pytestmark = pytest.mark.gpu

CASES = ["cube12", "rod", "slab", "cube13", "box9", "cube16", "cube8"]


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
        _OPS[name] = (g, d, H2Operator(d, tiers=("fp64", "bf16x3"), max_rhs=6))
    return _OPS[name]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("nrhs", [1, 5])
def test_bf16x3_product(torch, name, nrhs):
    print(f"[gpu] bf16x3 {name} n_rhs {nrhs}", flush=True)
    g, d, H = operator(name)
    X = h2gen.random_vector(3 * g.n_vox, 31, ncols=nrhs)             # (nrhs, N)
    Y = H.matvec(torch.from_numpy(X.astype(np.complex64)).cuda(), precision="bf16x3").cpu().numpy()
    for r in range(nrhs):
        yo = om.h2_matvec(d, X[r])
        emu = oprec.h2_matvec_tier(d, X[r], "bf16x3")
        e, ee = _rel(Y[r], yo), _rel(emu, yo)
        dev = _rel(Y[r], emu)      # device against the emulation of its own arithmetic
        print(f"[gpu] bf16x3 {name} col {r}: error {e:.3e}, emulated {ee:.3e}, device-emulation {dev:.3e}",
              flush=True)
        assert e <= 1e-4 and e <= 2.0 * ee, (r, e, ee)
        assert dev <= 0.5 * ee, (r, dev, ee)


def test_bf16x3_op_g(torch):
    g, d, H = operator("cube16")
    x = h2gen.random_vector(3 * g.n_vox, 3)
    y = H.matvec(torch.from_numpy(x.astype(np.complex64)).cuda(), op="G", precision="bf16x3").cpu().numpy()
    assert _rel(y, om.h2_matvec(d, x, "G")) <= 1e-4


def test_group_matches_members_and_replays(torch):
    from paper_1703_01175_amd import H2Group
    names = ["rod", "cube13", "box9", "cube12"]
    members = [operator(n) for n in names]
    grp = H2Group([m[2] for m in members])
    xs, ref = [], []
    for i, (g, d, H) in enumerate(members):
        nr = [1, 2, 3, 1][i]
        X = h2gen.random_vector(3 * g.n_vox, 40 + i, ncols=nr).astype(np.complex64)
        xs.append(torch.from_numpy(X).cuda())
        ref.append(H.matvec(xs[-1], precision="bf16x3").cpu().numpy())
    outs = None
    for rep in range(3):                   # graph captured on the first call, replayed after
        outs = grp.matvec(xs, outs=outs)
        torch.cuda.synchronize()
        _ = (xs[0] * 2).sum().item()       # eager work between replays
        for i in range(len(members)):
            assert np.array_equal(outs[i].cpu().numpy(), ref[i]), (rep, names[i])
    # a member skipped (n_rhs = 0) leaves the others unchanged
    outs2 = grp.matvec([xs[0], None, xs[2], None])
    assert np.array_equal(outs2[0].cpu().numpy(), ref[0]) and np.array_equal(outs2[2].cpu().numpy(), ref[2])
    for i, (g, d, H) in enumerate(members):
        X = xs[i].cpu().numpy().reshape(-1, 3 * g.n_vox)
        for r in range(X.shape[0]):
            assert _rel(outs[i].cpu().numpy().reshape(-1, 3 * g.n_vox)[r], om.h2_matvec(d, X[r].astype(np.complex128))) <= 1e-4
    grp.close()


def test_group_tune_and_no_graph(torch):
    from paper_1703_01175_amd import H2Group
    g, d, H = operator("slab")
    grp = H2Group([H])
    X = torch.from_numpy(h2gen.random_vector(3 * g.n_vox, 9, ncols=4).astype(np.complex64)).cuda()
    tile = grp.tune([X])
    assert tile in (32, 64, 128)
    y1 = grp.matvec([X])[0].cpu().numpy()
    grp.set(tile=32, graph=False)
    y2 = grp.matvec([X])[0].cpu().numpy()
    yo = om.h2_matvec(d, X.cpu().numpy()[1].astype(np.complex128))
    assert _rel(y1[1], yo) <= 1e-4 and _rel(y2[1], yo) <= 1e-4
    grp.close()
