"""Pins of the oracle H^2 product (P8) and of the construction (P4-P6).

The oracle product is compared with brute-force dense products written
independently in oracle/kernel.py; planted mistakes in the oracle must be
caught by the same comparisons.
"""
import numpy as np
import pytest

import h2gen
from conftest import built
from oracle import matvec as om
from oracle.kernel import dense_G, dense_Z_matvec

CASES = ["cube12", "cube12_e3", "rod", "slab", "cube13", "box9", "cube16"]


def _err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", CASES)
def test_h2_product_vs_dense(name):
    """Relative error of the represented G below the truncation epsilon, and of Z well below it."""
    g, d = built(name)
    eps = d.meta["eps"]
    x = h2gen.random_vector(3 * g.n_vox, 1)
    for op, bound in (("G", eps), ("Z", eps)):
        y = om.h2_matvec(d, x, op)
        yd = dense_Z_matvec(g.shape, g.h, g.k, g.chi, g.sigma, x, op)
        assert _err(y, yd) < bound, (name, op, _err(y, yd))


def test_all_near_equals_dense():
    g, d = built("cube8")
    assert d.n_far == 0
    x = h2gen.random_vector(3 * g.n_vox, 5)
    for op in ("G", "Z"):
        y = om.h2_matvec(d, x, op)
        yd = dense_Z_matvec(g.shape, g.h, g.k, g.chi, g.sigma, x, op)
        assert _err(y, yd) < 1e-13


def test_multiple_columns_match_single():
    g, d = built("cube12")
    X = h2gen.random_vector(3 * g.n_vox, 9, ncols=3).T.copy()
    Y = om.h2_matvec(d, X, "Z")
    for j in range(3):
        assert np.allclose(Y[:, j], om.h2_matvec(d, X[:, j].copy(), "Z"), rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", ["cube12", "rod", "cube13"])
def test_complex_symmetry(name):
    """G = G^T (the kernel depends on |r - r'| only); the H^2 product keeps it to ~eps."""
    g, d = built(name)
    x = h2gen.random_vector(3 * g.n_vox, 2)
    y = h2gen.random_vector(3 * g.n_vox, 3)
    Hy = om.h2_matvec(d, y, "G")
    Hx = om.h2_matvec(d, x, "G")
    asym = abs(x @ Hy - y @ Hx)
    assert asym <= d.meta["eps"] * np.linalg.norm(x) * np.linalg.norm(Hy)


@pytest.mark.parametrize("name", ["rod", "slab", "cube16", "box9"])
def test_symmetrized_couplings(name):
    """Couplings averaged with the transposes of their mirror blocks (S_st := S_ts^T):
    every stored pair is an exact transpose, the represented G is then symmetric to
    rounding (P8 with symmetric storage), and the representation keeps its accuracy
    against the dense G."""
    g, d0 = built(name)
    _, d = built(name + "_sym")
    assert d.meta.get("symmetric_couplings") and not d0.meta.get("symmetric_couplings")
    rev = {(int(t), int(s)): i for i, (t, s) in enumerate(zip(d.far_t, d.far_s))}
    for i, (t, s) in enumerate(zip(d.far_t, d.far_s)):
        j = rev[(int(s), int(t))]
        assert np.array_equal(om._coupling(d, i), om._coupling(d, j).T)
        if t < s:
            mean = 0.5 * (om._coupling(d0, i) + om._coupling(d0, j).T)
            assert np.array_equal(om._coupling(d, i), mean)
    x = h2gen.random_vector(3 * g.n_vox, 2)
    y = h2gen.random_vector(3 * g.n_vox, 3)
    Hx, Hy = om.h2_matvec(d, x, "G"), om.h2_matvec(d, y, "G")
    assert abs(x @ Hy - y @ Hx) <= 1e-14 * np.linalg.norm(x) * np.linalg.norm(Hy)
    H0x = om.h2_matvec(d0, x, "G")
    eps = d.meta["eps"]
    yd = dense_Z_matvec(g.shape, g.h, g.k, g.chi, g.sigma, x, "G")
    assert _err(Hx, yd) < eps and _err(Hx, H0x) < eps


def test_epsilon_tightens_error():
    g = h2gen.cube(12, 0.5, 4.0)
    from h2gen.construct import build_h2
    x = h2gen.random_vector(3 * g.n_vox, 4)
    yd = dense_Z_matvec(g.shape, g.h, g.k, g.chi, g.sigma, x, "G")
    errs = []
    for eps in (1e-2, 1e-4, 1e-8):
        d = build_h2(g, eps=eps)
        errs.append(_err(om.h2_matvec(d, x, "G"), yd))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-8


# ---------------------------------------------------------------- construction pins

_FB = {}


def _full_basis(d, c):
    """V_c formed explicitly from the leaf bases and transfers (eq. (9))."""
    key = (id(d), int(c))
    if key in _FB:
        return _FB[key]
    if d.nchild[c] == 0:
        V = om._basis(d, c)
    else:
        parts = [(_full_basis(d, ch) @ om._transfer(d, ch))
                 for ch in range(d.first_child[c], d.first_child[c] + d.nchild[c]) if d.rank[ch] > 0]
        V = np.concatenate(parts, axis=0)
    _FB[key] = V
    return V


@pytest.mark.parametrize("name", ["rod", "slab", "cube16", "box9"])
def test_bases_orthonormal_and_nested(name):
    """V^H V = I for leaf bases and for the nested bases of eq. (9)."""
    g, d = built(name)
    for c in range(d.n_clusters):
        k = int(d.rank[c])
        if k == 0:
            continue
        V = _full_basis(d, c)
        assert V.shape == (int(d.end[c] - d.begin[c]), k)
        assert np.abs(V.conj().T @ V - np.eye(k)).max() < 1e-12


def _tree_order_G(g, d):
    G = dense_G(g.shape, g.h, g.k)
    return G[np.ix_(d.perm, d.perm)]


@pytest.mark.parametrize("name", ["cube12", "rod", "slab"])
def test_couplings_match_projected_dense_blocks(name):
    """S_ts ~= V_t^H G^(t,s) conj(V_s) (eq. (18)) to the accuracy of the grouped row."""
    g, d = built(name)
    G = _tree_order_G(g, d)
    eps = d.meta["eps"]
    for t in np.unique(d.far_t):
        idx = np.nonzero(d.far_t == t)[0]
        Vt = _full_basis(d, t)
        rows = slice(d.begin[t], d.end[t])
        grp = np.concatenate([G[rows, d.begin[d.far_s[i]]:d.end[d.far_s[i]]] for i in idx], axis=1)
        scale = np.linalg.norm(grp, 2)
        for i in idx:
            s = d.far_s[i]
            Vs = _full_basis(d, s)
            Sx = Vt.conj().T @ G[rows, d.begin[s]:d.end[s]] @ Vs.conj()
            assert np.linalg.norm(om._coupling(d, i) - Sx, 2) <= 3 * eps * scale


@pytest.mark.parametrize("name", ["cube12", "rod", "slab", "box9"])
def test_bases_capture_row_blocks(name):
    """||(I - V V^H) G_(t)|| <= ~eps ||G_(t)|| for the admissible row block of t at and above its level."""
    g, d = built(name)
    G = _tree_order_G(g, d)
    eps = d.meta["eps"]
    anc = {}
    for c in range(d.n_clusters):
        chain, p = [c], int(d.parent[c])
        while p >= 0:
            chain.append(p)
            p = int(d.parent[p])
        anc[c] = chain
    for c in range(d.n_clusters):
        if d.rank[c] == 0:
            continue
        cols = []
        for j in anc[c]:
            for i in np.nonzero(d.far_t == j)[0]:
                s = d.far_s[i]
                cols.append(np.arange(d.begin[s], d.end[s]))
        if not cols:
            continue
        Gt = G[d.begin[c]:d.end[c]][:, np.concatenate(cols)]
        V = _full_basis(d, c)
        resid = Gt - V @ (V.conj().T @ Gt)
        assert np.linalg.norm(resid, 2) <= 4 * eps * np.linalg.norm(Gt, 2)


def test_aca_and_rsvd_against_dense():
    """Stage I (eqs. (5)-(7)): ACA error ~eps_A and r-SVD rank = exact SVD rank at eps."""
    from h2gen.aca import aca_partial, rsvd_truncate
    from h2gen.partition import build_partition
    from h2gen.tree import build_tree
    g = h2gen.cube(16, 1.0, 4.0)
    tree = build_tree(g.shape, 64)
    part = build_partition(tree)
    c = tree.coords.astype(float) * g.h
    rng = np.random.default_rng(0)
    ts = rng.choice(np.unique(part.far_t), 12, replace=False)
    for t in ts:
        cols = np.concatenate([np.arange(tree.begin[s], tree.end[s]) for s in part.far_s[part.far_t == t]])
        rows = np.arange(tree.begin[t], tree.end[t])
        diff = c[rows][:, None, :] - c[cols][None, :, :]
        from oracle.kernel import green
        Gt = green(np.sqrt((diff * diff).sum(-1)), g.k)
        U, V = aca_partial(lambda i: Gt[i], lambda j: Gt[:, j], Gt.shape[0], Gt.shape[1], 1e-5)
        assert np.linalg.norm(Gt - U @ V.T) <= 5e-5 * np.linalg.norm(Gt)
        A, B, K = rsvd_truncate(U, V, 1e-3)
        sv = np.linalg.svd(Gt, compute_uv=False)
        kex = int((sv > 1e-3 * sv[0]).sum())
        assert abs(A.shape[1] - kex) <= 1
        assert np.linalg.norm(Gt - A @ B.T, 2) <= 1.2e-3 * sv[0]
        assert np.allclose(K, B.T @ B.conj(), atol=1e-12)


# ---------------------------------------------------------------- planted mistakes

def _planted(monkeypatch, what):
    orig_basis, orig_transfer, orig_coupling, orig_near = om._basis, om._transfer, om._coupling, om._near
    if what == "conj_basis":
        monkeypatch.setattr(om, "_basis", lambda d, c: orig_basis(d, c).conj())
    elif what == "conj_transfer":
        monkeypatch.setattr(om, "_transfer", lambda d, c: orig_transfer(d, c).conj())
    elif what == "transposed_coupling":
        def tc(d, i):
            S = orig_coupling(d, i)
            return S.T if S.shape[0] == S.shape[1] else S[:, ::-1]
        monkeypatch.setattr(om, "_coupling", tc)
    elif what == "dropped_near":
        monkeypatch.setattr(om, "_near", lambda d, i: orig_near(d, i) * (0.0 if i == 7 else 1.0))
    elif what == "near_transposed":
        monkeypatch.setattr(om, "_near", lambda d, i: orig_near(d, i).T if d.near_t[i] != d.near_s[i] else orig_near(d, i))


@pytest.mark.parametrize("what", ["conj_basis", "conj_transfer", "transposed_coupling", "dropped_near"])
def test_planted_mistakes_are_caught(monkeypatch, what):
    name = "rod" if what == "conj_transfer" else "cube12"
    g, d = built(name)
    x = h2gen.random_vector(3 * g.n_vox, 1)
    yd = dense_Z_matvec(g.shape, g.h, g.k, g.chi, g.sigma, x, "G")
    _planted(monkeypatch, what)
    assert _err(om.h2_matvec(d, x, "G"), yd) > 10 * d.meta["eps"]


def test_planted_epilogue_sign_is_caught(monkeypatch):
    g, d = built("cube12")
    x = h2gen.random_vector(3 * g.n_vox, 1)
    zd = dense_Z_matvec(g.shape, g.h, g.k, g.chi, g.sigma, x, "Z")
    monkeypatch.setattr(d, "sigma", -d.sigma)
    assert _err(om.h2_matvec(d, x, "Z"), zd) > 10 * d.meta["eps"]
