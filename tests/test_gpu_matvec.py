"""GPU parity of the H^2 product through the C ABI against the CPU oracle."""
import os

import numpy as np
import pytest

import h2gen
from conftest import built
from oracle import matvec as om
from oracle import precision as oprec

pytestmark = pytest.mark.gpu

CASES = ["cube8", "cube12", "cube12_e3", "rod", "slab", "cube13", "box9", "cube16"]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


_OPS = {}


def operator(name, tiers=("fp64", "fp32")):
    from paper_1703_01175_amd import H2Operator
    key = (name, tiers)
    if key not in _OPS:
        g, d = built(name)
        _OPS[key] = (g, d, H2Operator(d, tiers=tiers, max_rhs=4))
    return _OPS[key]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("op", ["Z", "G"])
def test_fp64_product_matches_oracle(torch, name, op):
    print(f"[gpu] fp64 product {name} op {op}", flush=True)
    g, d, H = operator(name)
    x = h2gen.random_vector(3 * g.n_vox, 17)
    y = H.matvec(torch.from_numpy(x).cuda(), op=op).cpu().numpy()
    yo = om.h2_matvec(d, x, op)
    assert _rel(y, yo) <= 1e-12
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()


def test_multiple_rhs(torch):
    g, d, H = operator("slab")
    X = h2gen.random_vector(3 * g.n_vox, 5, ncols=3)          # (3, N): column major N x 3
    Y = H.matvec(torch.from_numpy(X).cuda()).cpu().numpy()
    Yo = om.h2_matvec(d, X.T.copy()).T
    assert _rel(Y, Yo) <= 1e-12


def test_plane_wave_product(torch):
    g, d, H = operator("cube12")
    b = h2gen.plane_wave(g, 3)[0]
    y = H.matvec(torch.from_numpy(b).cuda()).cpu().numpy()
    assert _rel(y, om.h2_matvec(d, b)) <= 1e-12


@pytest.mark.parametrize("name", ["cube12", "rod", "cube16"])
def test_fp32_tier_error(torch, name):
    g, d, H = operator(name)
    x = h2gen.random_vector(3 * g.n_vox, 23)
    yo = om.h2_matvec(d, x)
    y32 = H.matvec(torch.from_numpy(x.astype(np.complex64)).cuda(), precision="fp32").cpu().numpy()
    emu = oprec.h2_matvec_tier(d, x, "fp32")
    e_gpu, e_emu = _rel(y32, yo), _rel(emu, yo)
    dev = _rel(y32, emu)
    print(f"[gpu] fp32 tier {name}: gpu {e_gpu:.2e} emulated {e_emu:.2e} device-emulation {dev:.2e}", flush=True)
    assert e_gpu <= 1e-5 and e_gpu <= 2.0 * e_emu
    assert dev <= 2.0 * e_emu


def test_build_rejects_small_buffer(torch):
    import ctypes as C
    from paper_1703_01175_amd import _lib
    g, d = built("rod")
    lib = _lib.load()
    hd, keep = _lib.host_desc(d)
    opts = _lib.BuildOpts(1, 1)
    n = C.c_size_t(0)
    assert lib.h2_plan_from_host(C.byref(hd), C.byref(opts), C.byref(n)) == 0
    buf = torch.empty(n.value // 2, dtype=torch.uint8, device="cuda")
    h = C.c_void_p(0)
    st = lib.h2_build_from_host(C.byref(hd), C.byref(opts), C.c_void_p(buf.data_ptr()), n.value // 2,
                                None, C.byref(h))
    assert st == -4 and not h.value


def test_destroyed_handle_and_bad_args(torch):
    from paper_1703_01175_amd import H2Operator
    g, d = built("rod")
    H = H2Operator(d)                                   # FP64 tier only
    x = torch.from_numpy(h2gen.random_vector(3 * g.n_vox, 1)).cuda()
    y = torch.empty_like(x)
    lib = H.lib
    assert lib.h2_matvec(H.handle, 1, 1, x.data_ptr(), y.data_ptr(), 1, H.N, None) == -1   # tier not built
    assert lib.h2_matvec(H.handle, 1, 0, x.data_ptr(), x.data_ptr(), 1, H.N, None) == -1   # x, y overlap
    assert lib.h2_matvec(H.handle, 1, 0, x.data_ptr(), y.data_ptr(), 1, H.N - 1, None) == -1  # ld < N
    assert lib.h2_matvec(H.handle, 7, 0, x.data_ptr(), y.data_ptr(), 1, H.N, None) == -1   # unknown op
    assert lib.h2_matvec(H.handle, 1, 0, x.data_ptr() + 8, y.data_ptr(), 1, H.N, None) == -1  # misaligned
    handle = H.handle
    H.close()
    assert lib.h2_matvec(handle, 1, 0, x.data_ptr(), y.data_ptr(), 1, H.N, None) == -5


def test_profile_counts_kernel_families(torch):
    import ctypes as C
    from paper_1703_01175_amd import _lib
    g, d, H = operator("cube16")
    lib = H.lib
    assert lib.h2_profile_enable(H.handle, 1) == 0
    x = torch.from_numpy(h2gen.random_vector(3 * g.n_vox, 2)).cuda()
    for _ in range(3):
        H.matvec(x)
    buf = (C.c_byte * 128)()
    assert lib.h2_profile_read(H.handle, buf) == 0
    ms = np.frombuffer(bytes(buf)[:64], np.float64)
    launches = np.frombuffer(bytes(buf)[64:], np.int64)
    # with several near passes over stored-once blocks, the early passes run (and are
    # timed) on the side stream: two near intervals per product
    # (so does the tiled near field, whose block products run there before the finish)
    per = 2 if ((H.stats()["near_passes"] > 1 or H.near_tiles()[0]) and not H.near_mode()[0]) else 1
    assert launches[5] == 3 * per and launches[0] == 3 and ms[5] > 0
    assert lib.h2_profile_enable(H.handle, 0) == 0


@pytest.mark.parametrize("name", ["cube12", "rod", "slab", "cube13", "box9"])
def test_symmetric_near_mode_matches_full_mode_and_oracle(torch, name):
    """The near blocks of G are transposes of each other bit for bit, so the
    symmetric near mode is available; both modes match the oracle, in FP64 and
    FP32, and agree with each other to rounding."""
    print(f"[gpu] near modes {name}", flush=True)
    g, d, H = operator(name)
    stored_once = H.stats()["near_stored_elems"] < H.stats()["near_elems"]
    assert H.near_mode() == (not stored_once, True)     # the default: symmetric unless blocks are cached
    assert H.near_mode(True) == (True, True)
    x = h2gen.random_vector(3 * g.n_vox, 23)
    xs = torch.from_numpy(x).cuda()
    ys = H.matvec(xs).cpu().numpy()
    yf32s = H.matvec(torch.from_numpy(x.astype(np.complex64)).cuda(), precision="fp32").cpu().numpy()
    assert H.near_mode(False) == (False, True)
    yf = H.matvec(xs).cpu().numpy()
    yf32f = H.matvec(torch.from_numpy(x.astype(np.complex64)).cuda(), precision="fp32").cpu().numpy()
    H.near_mode(not stored_once)
    yo = om.h2_matvec(d, x)
    assert _rel(ys, yo) <= 1e-12 and _rel(yf, yo) <= 1e-12
    assert _rel(ys, yf) <= 1e-13
    assert _rel(yf32s, yo) <= 1e-5 and _rel(yf32f, yo) <= 1e-5


def test_asymmetric_near_blocks_use_the_full_mode(torch):
    """One off-diagonal near entry changed: the symmetric mode is not offered and
    the product follows the changed description."""
    import dataclasses
    from paper_1703_01175_amd import H2Operator
    from paper_1703_01175_amd._lib import H2Error
    g, d = built("cube12")
    i = int(np.nonzero(d.near_t != d.near_s)[0][0])
    near = d.near.copy()
    near[d.near_off[i] + 1] *= 1.5
    d2 = dataclasses.replace(d, near=near)
    H = H2Operator(d2, tiers=("fp64",))
    assert H.near_mode() == (False, False)
    with pytest.raises(H2Error):
        H.near_mode(True)
    x = h2gen.random_vector(3 * g.n_vox, 29)
    y = H.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y, om.h2_matvec(d2, x)) <= 1e-12
    H.close()


@pytest.mark.parametrize("name", ["cube12", "slab", "cube16"])
def test_identical_near_blocks_stored_once_give_identical_products(torch, name):
    """Storing identical near blocks once (and reading them through the caches)
    changes no arithmetic beyond the order of the near sums (the full mode runs the
    leaf's blocks in passes over a share of the distinct blocks each): the
    symmetric mode and BF16x3 products equal, bit for bit, those of an operator
    built with every near block kept; the full mode, FP32 and several right-hand
    sides per pass agree to rounding; both match the oracle."""
    from paper_1703_01175_amd import H2Operator
    print(f"[gpu] stored-once near blocks {name}", flush=True)
    g, d = built(name)
    tiers = ("fp64", "fp32", "bf16x3")
    A = H2Operator(d, tiers=tiers, max_rhs=4)
    B = H2Operator(d, tiers=tiers, max_rhs=4, keep_all_near=True)
    sa, sb = A.stats(), B.stats()
    assert sa["near_unique"] < sa["n_near"] and 2 * sa["near_stored_elems"] <= sa["near_elems"]
    assert sb["near_unique"] == sb["n_near"] and sb["near_stored_elems"] == sb["near_elems"]
    x = h2gen.random_vector(3 * g.n_vox, 31)
    X = h2gen.random_vector(3 * g.n_vox, 32, ncols=4)
    x32 = torch.from_numpy(x.astype(np.complex64)).cuda()
    for sym in (True, False):
        A.near_mode(sym)
        B.near_mode(sym)
        ya = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        yb = B.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        assert np.array_equal(ya, yb) if sym else _rel(ya, yb) <= 1e-14, sym
        assert _rel(ya, om.h2_matvec(d, x)) <= 1e-12
        fa = A.matvec(x32, precision="fp32").cpu().numpy()
        fb = B.matvec(x32, precision="fp32").cpu().numpy()
        assert np.array_equal(fa, fb) if sym else _rel(fa, fb) <= 1e-6, sym
    Ya = A.matvec(torch.from_numpy(X).cuda()).cpu().numpy()
    Yb = B.matvec(torch.from_numpy(X).cuda()).cpu().numpy()
    assert _rel(Ya, Yb) <= 1e-14
    X32 = torch.from_numpy(X.astype(np.complex64)).cuda()
    Za = A.matvec(X32, precision="bf16x3").cpu().numpy()
    Zb = B.matvec(X32, precision="bf16x3").cpu().numpy()
    assert np.array_equal(Za, Zb)
    assert _rel(Za[2], om.h2_matvec(d, X[2])) <= 1e-4
    A.close()
    B.close()


def test_overlapped_near_passes_over_several_rhs(torch):
    """cube16 stores its near blocks once and runs them in several passes, the early
    ones on the side stream beside the couplings.  A handle built for one right-hand
    side takes several in turn (the loop reuses U and the pass row sums for each):
    every column matches the oracle."""
    from paper_1703_01175_amd import H2Operator
    g, d = built("cube16")
    H = H2Operator(d, tiers=("fp64",), max_rhs=1)
    assert H.stats()["near_passes"] > 1 and not H.near_mode()[0]
    X = h2gen.random_vector(3 * g.n_vox, 41, ncols=3)               # (3, N)
    lib = H.lib
    Xd = torch.from_numpy(X).cuda()
    import ctypes as C
    from paper_1703_01175_amd import _lib
    for tiles in (False, True):          # the passes, then the tiled near field
        assert H.near_tiles(tiles) == (tiles, True)
        Yd = torch.empty_like(Xd)
        _lib.check(lib.h2_matvec(H.handle, 1, 0, C.c_void_p(Xd.data_ptr()), C.c_void_p(Yd.data_ptr()), 3, H.N, None))
        Y = Yd.cpu().numpy()
        for c in range(3):
            assert _rel(Y[c], om.h2_matvec(d, X[c])) <= 1e-12, (tiles, c)
    H.close()


@pytest.mark.parametrize("name", CASES)
def test_tiled_near_field_matches_per_leaf_kernel_and_oracle(torch, name):
    """Near blocks stored once: the full-mode product applies each stored block to the
    sources of 16 target leaves at once on the matrix cores (tiles of 16 leaves
    consecutive in tree order; FP64 and FP32 tiers).  It covers leaves of 27 voxels (cube12: columns past a
    block's width, rows past its height), tiles with empty slots (cube8: 8 leaves) and
    every geometry here; FP64 products match the per-leaf kernel to rounding and the
    oracle, for Z and G, and FP32 ones stay within the tier's bound.  Without stored-once blocks there are no tiles."""
    from paper_1703_01175_amd._lib import H2Error
    print(f"[gpu] tiled near field {name}", flush=True)
    g, d, H = operator(name)
    st = H.stats()
    stored_once = st["near_stored_elems"] < st["near_elems"]
    n_leaves = int(st["n_leaves"])
    if not stored_once:
        assert H.near_tiles() == (False, False) and st["near_tiles"] == 0
        with pytest.raises(H2Error):
            H.near_tiles(True)
        return
    assert st["near_tiles"] == (n_leaves + 15) // 16
    assert st["near_tile_steps"] >= st["n_near"] / 16
    sym0 = H.near_mode()[0]
    H.near_mode(False)
    assert H.near_tiles() == (True, True)
    x = h2gen.random_vector(3 * g.n_vox, 43)
    xs = torch.from_numpy(x).cuda()
    for op in ("Z", "G"):
        yt = H.matvec(xs, op=op).cpu().numpy()
        assert H.near_tiles(False) == (False, True)
        yl = H.matvec(xs, op=op).cpu().numpy()
        assert H.near_tiles(True) == (True, True)
        yo = om.h2_matvec(d, x, op)
        assert _rel(yt, yl) <= 1e-13, op
        assert _rel(yt, yo) <= 1e-12, op
        assert np.abs(yt - yo).max() <= 1e-12 * np.abs(yo).max(), op
    # the FP32 tier: tiles on the FP32 matrix cores, within the tier's bound
    x32 = torch.from_numpy(x.astype(np.complex64)).cuda()
    yt32 = H.matvec(x32, precision="fp32").cpu().numpy()
    H.near_tiles(False)
    yl32 = H.matvec(x32, precision="fp32").cpu().numpy()
    H.near_tiles(True)
    yo = om.h2_matvec(d, x)
    e_emu = _rel(oprec.h2_matvec_tier(d, x, "fp32"), yo)
    e_t, e_l = _rel(yt32, yo), _rel(yl32, yo)
    print(f"[gpu] fp32 {name}: tiles {e_t:.2e} per-leaf {e_l:.2e} emulated {e_emu:.2e}", flush=True)
    assert e_t <= 1e-5 and e_t <= 2.0 * e_emu
    assert _rel(yt32, yl32) <= 2.0 * e_emu
    H.near_mode(sym0)


SYM_CASES = ["cube12_sym", "rod_sym", "slab_sym", "cube13_sym", "box9_sym", "cube16_sym"]


@pytest.mark.parametrize("name", SYM_CASES)
def test_symmetric_coupling_mode_matches_full_mode_and_oracle(torch, name):
    """Couplings symmetrised in the description (S_st = S_ts^T bit for bit): the
    symmetric coupling mode (each unordered pair streamed once) is available; in both
    coupling modes and both near modes the FP64 product matches the
    oracle on the same description (op Z and G), the modes agree to rounding, and
    the FP32 tier stays within its bound."""
    print(f"[gpu] coupling modes {name}", flush=True)
    g, d, H = operator(name)
    st = H.stats()
    assert H.coupling_mode() == (False, True)          # available; handles start in the full mode
    assert 0.45 * st["coupling_elems"] <= st["coupling_owned_elems"] <= 0.55 * st["coupling_elems"]
    x = h2gen.random_vector(3 * g.n_vox, 43)
    xd = torch.from_numpy(x).cuda()
    x32 = torch.from_numpy(x.astype(np.complex64)).cuda()
    near0 = H.near_mode()[0]
    for op in ("Z", "G"):
        yo = om.h2_matvec(d, x, op)
        out = {}
        for near_sym in (True, False):
            H.near_mode(near_sym)
            for coup_sym in (True, False):
                H.coupling_mode(coup_sym)
                y = H.matvec(xd, op=op).cpu().numpy()
                assert _rel(y, yo) <= 1e-12, (op, near_sym, coup_sym)
                assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
                out[(near_sym, coup_sym)] = y
                if op == "Z":
                    y32 = H.matvec(x32, precision="fp32").cpu().numpy()
                    assert _rel(y32, yo) <= 1e-5, (near_sym, coup_sym)
        for k in out:
            assert _rel(out[k], out[(True, True)]) <= 1e-13, k
    H.near_mode(near0)
    H.coupling_mode(False)


def test_unsymmetric_couplings_use_the_full_mode(torch):
    """The generator's couplings from eq. (18) are not exact transposes: no symmetric
    coupling mode, and asking for it fails."""
    from paper_1703_01175_amd._lib import H2Error
    g, d, H = operator("rod")
    assert H.coupling_mode() == (False, False)
    assert H.stats()["coupling_owned_elems"] == 0
    with pytest.raises(H2Error):
        H.coupling_mode(True)


def test_symmetric_coupling_mode_one_changed_entry(torch):
    """One coupling entry of a symmetrised description changed: the mode is not offered."""
    import dataclasses
    from paper_1703_01175_amd import H2Operator
    g, d = built("rod_sym")
    c = d.coupling.copy()
    c[int(d.far_off[5]) + 1] *= 1.0 + 1e-15
    d2 = dataclasses.replace(d, coupling=c)
    H = H2Operator(d2, tiers=("fp64",))
    assert H.coupling_mode() == (False, False)
    x = h2gen.random_vector(3 * g.n_vox, 47)
    y = H.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y, om.h2_matvec(d2, x)) <= 1e-12
    H.close()


@pytest.mark.parametrize("name", ["rod_sym", "cube16_sym", "slab_sym"])
def test_symmetric_coupling_storage_other_products(torch, name):
    """With symmetric couplings each grouped block row is stored with its owned
    blocks first; the products that stream every block (several right-hand sides in
    FP64 and FP32, the BF16x3 tier packed from the stored blocks) read the same
    storage and match the oracle."""
    from paper_1703_01175_amd import H2Operator
    print(f"[gpu] symmetric coupling storage {name}", flush=True)
    g, d = built(name)
    H = H2Operator(d, tiers=("fp64", "fp32", "bf16x3"), max_rhs=5)
    assert H.coupling_mode(True) == (True, True)
    X = h2gen.random_vector(3 * g.n_vox, 57, ncols=5)
    Y = H.matvec(torch.from_numpy(X).cuda()).cpu().numpy()
    Y32 = H.matvec(torch.from_numpy(X.astype(np.complex64)).cuda(), precision="fp32").cpu().numpy()
    Yb = H.matvec(torch.from_numpy(X.astype(np.complex64)).cuda(), precision="bf16x3").cpu().numpy()
    for c in range(5):
        yo = om.h2_matvec(d, X[c])
        assert _rel(Y[c], yo) <= 1e-12
        assert _rel(Y32[c], yo) <= 1e-5
        assert _rel(Yb[c], yo) <= 1e-4
    H.close()
