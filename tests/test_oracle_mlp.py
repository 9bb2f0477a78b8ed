"""Pins of the MLP-preconditioner reference (P11) and of the block-diagonal apply."""
import numpy as np
import pytest
import torch

from oracle import mlp
from oracle.precision import bf16_round


def _small(seed=0, n_pad=4, hidden=16):
    n_in, h, n_out = mlp.dims(n_pad, hidden)
    p = mlp.init_params(n_in, h, n_out, seed)
    rng = np.random.default_rng(seed + 1)
    for k in p:
        if k.startswith("b"):
            p[k] = (0.1 * rng.standard_normal(p[k].shape)).astype(np.float32)
    X = rng.standard_normal((9, n_in))
    T = rng.standard_normal((9, n_out))
    return p, X, T


def test_forward_matches_torch_functional():
    p, X, T = _small()
    q = mlp.rounded(p)
    tt = {k: torch.from_numpy(v) for k, v in q.items()}
    x = torch.from_numpy(X)
    h = torch.relu(torch.nn.functional.linear(x, tt["W1"], tt["b1"]))
    h = torch.relu(torch.nn.functional.linear(h, tt["W2"], tt["b2"]))
    y = torch.nn.functional.linear(h, tt["W3"], tt["b3"]).numpy()
    assert np.allclose(mlp.forward(q, X), y, rtol=1e-13, atol=1e-13)


def test_gradients_vs_central_differences():
    p, X, T = _small(3)
    q = mlp.rounded(p)
    L, g = mlp.loss_and_grads(q, X, T)
    rng = np.random.default_rng(7)
    for k in q:
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in q[k].shape)
            h = 1e-6
            qp = {kk: vv.copy() for kk, vv in q.items()}
            qm = {kk: vv.copy() for kk, vv in q.items()}
            qp[k][idx] += h
            qm[k][idx] -= h
            fd = (mlp.loss_and_grads(qp, X, T)[0] - mlp.loss_and_grads(qm, X, T)[0]) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_gradients_vs_torch_autograd():
    p, X, T = _small(5)
    q = mlp.rounded(p)
    L, g = mlp.loss_and_grads(q, X, T)
    tt = {k: torch.tensor(v, requires_grad=True) for k, v in q.items()}
    x = torch.from_numpy(X)
    h = torch.relu(x @ tt["W1"].T + tt["b1"])
    h = torch.relu(h @ tt["W2"].T + tt["b2"])
    y = h @ tt["W3"].T + tt["b3"]
    loss = 0.5 * ((y - torch.from_numpy(T)) ** 2).sum() / X.shape[0]
    loss.backward()
    assert abs(float(loss) - L) <= 1e-12 * abs(L)
    for k in q:
        assert np.allclose(g[k], tt[k].grad.numpy(), rtol=1e-12, atol=1e-14)


def test_adam_matches_torch():
    p, X, T = _small(8)
    master = {k: v.copy() for k, v in p.items()}
    m = {k: np.zeros_like(v, dtype=np.float64) for k, v in p.items()}
    v = {k: np.zeros_like(vv, dtype=np.float64) for k, vv in p.items()}
    tp = {k: torch.tensor(val.astype(np.float64), requires_grad=True) for k, val in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    rng = np.random.default_rng(2)
    for step in range(1, 4):
        g = {k: rng.standard_normal(val.shape) for k, val in p.items()}
        mlp.adam_step(master, m, v, g, step, 1e-3)
        for k in tp:
            tp[k].grad = torch.from_numpy(g[k])
        opt.step()
    for k in p:
        assert np.allclose(master[k], tp[k].detach().numpy(), rtol=1e-6, atol=1e-7)


def test_weights_pass_through_bf16():
    p, X, T = _small(1)
    q = mlp.rounded(p)
    for k in ("W1", "W2", "W3"):
        assert np.array_equal(q[k], bf16_round(p[k]).astype(np.float64))


def test_blockdiag_apply_matches_dense_leaf_solves():
    from conftest import built
    from oracle.kernel import dense_G
    import h2gen
    g, d = built("cube12")
    r = h2gen.random_vector(3 * g.n_vox, 4)
    z = mlp.blockdiag_apply(d, r)
    G = dense_G(g.shape, g.h, g.k)
    alpha = g.sigma * g.k ** 2 * g.volume
    R = r.reshape(-1, 3)
    Z = z.reshape(-1, 3)
    for t in np.nonzero(d.nchild == 0)[0][:6]:
        vox = d.perm[d.begin[t]:d.end[t]]
        M = np.eye(vox.size) + alpha * G[np.ix_(vox, vox)] * g.chi[vox][None, :]
        assert np.allclose(M @ Z[vox], R[vox], rtol=0, atol=1e-12 * np.abs(R).max())


def test_features_and_apply_layout():
    from conftest import built
    import h2gen
    g, d = built("rod")
    r = h2gen.random_vector(3 * g.n_vox, 6)
    X, leaves, s = mlp.leaf_features(d, r, 64)
    assert X.shape == (leaves.size, 7 * 64)
    assert abs(s - np.linalg.norm(r) / np.sqrt(r.size)) < 1e-15
    # the residual block of the features is the targets of r itself, and scattering
    # targets of any e (scaled by the same s) gives e back
    T = mlp.leaf_targets(d, r, r, 64)
    assert np.array_equal(X[:, :6 * 64], T)
    assert np.allclose(mlp.scatter(d, T, s, 64, r.size), r, rtol=0, atol=1e-14)
    e = h2gen.random_vector(3 * g.n_vox, 7)
    assert np.allclose(mlp.scatter(d, mlp.leaf_targets(d, e, r, 64), s, 64, r.size), e, rtol=0, atol=1e-14)
    # the chi block holds Re chi of the leaf's voxels, zero padded
    q = 0
    vox = d.perm[d.begin[leaves[q]]:d.end[leaves[q]]]
    assert np.array_equal(X[q, 6 * 64:6 * 64 + vox.size], g.chi[vox].real)
    assert not X[q, 6 * 64 + vox.size:].any()


def test_halo_table_on_a_uniform_leaf_grid():
    """On the 12^3 cube every leaf is a 3^3 block on a 4^3 grid of leaves: the table is
    the 26-neighbourhood of that grid, -1 exactly where it leaves the grid."""
    from conftest import built
    g, d = built("cube12")
    tab = mlp.halo_table(d, g.shape)
    leaves = np.nonzero(d.nchild == 0)[0]
    cell = []
    for t in leaves:
        xyz = np.stack(np.unravel_index(d.perm[d.begin[t]:d.end[t]], g.shape), 1)
        assert (xyz.max(0) - xyz.min(0) + 1 == 3).all() and d.end[t] - d.begin[t] == 27
        cell.append(tuple(xyz.min(0) // 3))
    where = {c: q for q, c in enumerate(cell)}
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]
    for q, c in enumerate(cell):
        for j, o in enumerate(offs):
            nb = tuple(c[a] + o[a] for a in range(3))
            assert tab[q, j] == where.get(nb, -1)
    # symmetric: o and -o are reverse slots
    for q in range(len(cell)):
        for j in range(26):
            if tab[q, j] >= 0:
                assert tab[tab[q, j], 25 - j] == q


def test_halo_features_are_neighbour_means():
    from conftest import built
    import h2gen
    g, d = built("box9")                       # uneven leaves
    tab = mlp.halo_table(d, g.shape)
    r = h2gen.random_vector(3 * g.n_vox, 9)
    X0, leaves, s = mlp.leaf_features(d, r, 64)
    X, _, _ = mlp.leaf_features(d, r, 64, tab)
    assert np.array_equal(X[:, :7 * 64], X0)
    R = r.reshape(-1, 3) / s
    for q in range(0, leaves.size, 5):
        for j in range(26):
            nb = tab[q, j]
            blk = X[q, 7 * 64 + 6 * j:7 * 64 + 6 * j + 6]
            if nb < 0:
                assert not blk.any()
            else:
                vox = d.perm[d.begin[leaves[nb]]:d.end[leaves[nb]]]
                m = R[vox].sum(0) / vox.size
                assert np.allclose(blk, np.concatenate([m.real, m.imag]), rtol=0, atol=1e-14)
