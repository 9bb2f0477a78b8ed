"""The C-ABI library on the CPU: it loads, exports every declared symbol, and its
host-side validation turns corrupted descriptions into the documented status."""
import copy
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1703_01175_amd import _lib
from paper_1703_01175_amd.build import LIB

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "h2vie.h")


def _lib_or_build():
    if not os.path.exists(LIB):
        from paper_1703_01175_amd.build import build
        build()
    return _lib.load()


def test_exports_every_declared_symbol():
    lib = _lib_or_build()
    names = set(re.findall(r"\b(h2_[a-z_0-9]+)\s*\(", open(HEADER).read()))
    assert names, "no declarations found"
    for n in sorted(names):
        assert hasattr(lib, n), n


def _plan(d, max_rhs=1, tiers=1, flags=0):
    lib = _lib_or_build()
    hd, keep = _lib.host_desc(d)
    opts = _lib.BuildOpts(max_rhs=max_rhs, tiers=tiers, flags=flags)
    n = C.c_size_t(0)
    st = lib.h2_plan_from_host(C.byref(hd), C.byref(opts), C.byref(n))
    return st, n.value


@pytest.fixture(scope="module")
def desc():
    from conftest import built
    return built("rod")[1]


def test_plan_ok(desc):
    st, n = _plan(desc, flags=1)
    assert st == 0 and n > desc.near.nbytes + desc.coupling.nbytes
    st2, n2 = _plan(desc, tiers=3, flags=1)
    assert st2 == 0 and n2 > n
    st3, n3 = _plan(desc)
    assert st3 == 0 and n3 < n


def test_plan_reserves_partials_only_for_symmetric_near_blocks(desc):
    """The plan checks G_st = G_ts^T bit for bit on the host: the symmetric near
    mode's partial slots (one 64 x 3 complex slot per unordered leaf pair) are
    reserved for the generated description and not once one entry is changed."""
    st, n = _plan(desc, flags=1)
    i = int(np.nonzero(desc.near_t != desc.near_s)[0][0])
    e = copy.copy(desc)
    e.near = desc.near.copy()
    e.near[desc.near_off[i] + 1] *= 1.5
    st2, n2 = _plan(e, flags=1)
    pairs = int((desc.near_t != desc.near_s).sum()) // 2
    assert st == 0 and st2 == 0
    assert n - n2 >= pairs * 64 * 3 * 16 + 16 * desc.n_vox * 3


def _unique_near(d):
    """Distinct near blocks (size and bytes), counted by brute force."""
    size = d.end - d.begin
    seen = {}
    for i in range(len(d.near_t)):
        n = int(size[d.near_t[i]] * size[d.near_s[i]])
        seen.setdefault((n, d.near[d.near_off[i]:d.near_off[i] + n].tobytes()), n)
    return len(seen), sum(seen.values())


def test_plan_stores_identical_near_blocks_once():
    """cube12: 2680 near pairs over 117 distinct blocks.  The plan holds each
    distinct block once (the device buffer shrinks by the entries saved), unless
    asked to keep every block; an unknown flag is rejected."""
    from conftest import built
    d = built("cube12")[1]
    n_unique, stored = _unique_near(d)
    assert n_unique == 117
    st, n = _plan(d)
    st2, n2 = _plan(d, flags=1)
    assert st == 0 and st2 == 0
    # (the stored-once plan adds the near-field tiles: steps of 16 source slots, and
    # the row sums of the side-stream launch)
    assert n2 - n >= 16 * (d.near.size - stored) - 48 * d.n_vox - (1 << 18)
    assert _plan(d, flags=2)[0] == -1


def test_plan_keeps_near_blocks_when_few_repeat():
    """box9 repeats too few blocks for storing them once to halve the storage: the
    plan is the same with and without the flag."""
    from conftest import built
    d = built("box9")[1]
    n_unique, stored = _unique_near(d)
    assert 2 * stored > d.near.size
    assert _plan(d)[1] == _plan(d, flags=1)[1]


def _corrupt(desc, field, fn):
    e = copy.copy(desc)
    setattr(e, field, fn(np.array(getattr(desc, field))))
    return e


def _set(i, v):
    def f(a):
        a[i] = v
        return a
    return f


CORRUPTIONS = [
    ("perm", _set(0, 1), -2),                     # duplicate index
    ("rank", lambda a: np.where(a > 0, 100, a), -2),   # rank larger than the leaf
    ("basis_off", lambda a: np.where(a >= 0, a + 10 ** 9, a), -2),
    ("far_off", lambda a: a + 1, -2),               # blocks not back to back / past the end
    ("near_t", lambda a: a[::-1].copy(), -2),       # not sorted
    ("near_s", _set(0, 0), -2),                     # root is not a leaf
    ("near_off", _set(-1, 10 ** 12), -2),
    ("end", _set(1, 0), -2),                        # empty / inverted range
    ("parent", _set(2, 5), -2),
    ("far_s", _set(0, 10 ** 6), -2),
]


@pytest.mark.parametrize("field,fn,status", CORRUPTIONS, ids=[c[0] for c in CORRUPTIONS])
def test_corrupted_descriptions_rejected(desc, field, fn, status):
    st, _ = _plan(_corrupt(desc, field, fn))
    assert st == status
    assert _lib.load().h2_last_error().decode()


def test_bad_scalars_and_options(desc):
    e = copy.copy(desc)
    e.k = float("nan")
    assert _plan(e)[0] == -2
    e = copy.copy(desc)
    e.ncomp = 2
    assert _plan(e)[0] == -2
    assert _plan(desc, max_rhs=0)[0] == -1
    assert _plan(desc, tiers=8)[0] == -1
    lib = _lib_or_build()
    n = C.c_size_t(0)
    opts = _lib.BuildOpts(1, 1)
    assert lib.h2_plan_from_host(None, C.byref(opts), C.byref(n)) == -1


def test_bad_handles_without_gpu():
    lib = _lib_or_build()
    fake = C.c_void_p(0x1000)
    assert lib.h2_matvec(None, 1, 0, None, None, 1, 1, None) == -5
    assert lib.h2_matvec(fake, 1, 0, None, None, 1, 1, None) == -5
    s = _lib.Stats()
    assert lib.h2_stats(fake, C.byref(s)) == -5
    n = C.c_size_t(0)
    o = _lib.GmresOpts(50, 100, 1e-6, 0, 1e-3, 10)
    assert lib.h2_gmres_workspace(fake, C.byref(o), C.byref(n)) == -5
    rep = _lib.GmresReport()
    assert lib.h2_gmres_solve(None, None, None, C.byref(o), C.byref(rep), None, 0, None) == -5
    lib.h2_destroy(None)
    lib.h2_destroy(fake)    # unknown pointers are ignored
    assert lib.h2_profile_enable(fake, 1) == -5


def test_plan_reserves_coupling_partials_only_for_symmetric_couplings():
    """A description with symmetrised couplings (S_st = S_ts^T bit for bit, checked
    by the plan) gets the symmetric coupling mode's buffers: one 3-complex partial
    per owned column (each unordered admissible pair owned by one of its clusters,
    about half of every cluster's pairs) plus the receive lists.  The
    generator's own couplings (eq. (18), not exact transposes) get none."""
    from conftest import built
    d0 = built("rod")[1]
    d = built("rod_sym")[1]
    st0, n0 = _plan(d0, flags=1)
    st, n = _plan(d, flags=1)
    assert st0 == 0 and st == 0
    own = 0
    for t, s in zip(d.far_t, d.far_s):
        t, s = int(t), int(s)
        owner = t if (t < s) == ((t + s) % 2 == 0) else s
        if owner == t:
            own += int(d.rank[s])
    total_cols = int(d.rank[d.far_s].sum())
    assert 0.4 * total_cols <= own <= 0.6 * total_cols
    assert n - n0 >= own * 3 * 16
