"""H^2 matrix-vector product, plain loops (test infrastructure).

Follows Sec. IV.B of the paper on the stored representation (eq. (8)):
G^{t,s} ~= V^t S^{t,s} (V^s)^T for admissible blocks, full blocks otherwise.

1. forward transformation  x^s := (V^s)^T x|_s for every cluster s, using the
   nested bases of eq. (9): at a leaf (V^s)^T x|_s, above it
   x^p = sum_c (T^c)^T x^c (plain transpose, not conjugate);
2. coupling multiplication y^t := sum_{s in R^t} S^{t,s} x^s;
3. backward transformation y_i := sum_{t containing i} (V^t y^t)_i, i.e.
   y^c += T^c y^p top down and y|_t += V^t y^t at the leaves;
4. inadmissible blocks: y|_t += G^{t,s} x|_s in full.

The operator on the caller's vector (unknown 3i+c) is
Z x = x + sigma k^2 V (G (x) I_3)(chi . x); op "G" returns (G (x) I_3) x.
Arrays are read from an H2Desc (column-major blocks at element offsets).
"""

from __future__ import annotations

import numpy as np


def _basis(d, c):
    n = int(d.end[c] - d.begin[c])
    k = int(d.rank[c])
    o = int(d.basis_off[c])
    return d.basis[o:o + n * k].reshape(k, n).T


def _transfer(d, c):
    kc = int(d.rank[c])
    kp = int(d.rank[int(d.parent[c])])
    o = int(d.transfer_off[c])
    return d.transfer[o:o + kc * kp].reshape(kp, kc).T


def _coupling(d, i):
    kt = int(d.rank[int(d.far_t[i])])
    ks = int(d.rank[int(d.far_s[i])])
    o = int(d.far_off[i])
    return d.coupling[o:o + kt * ks].reshape(ks, kt).T


def _near(d, i):
    t, s = int(d.near_t[i]), int(d.near_s[i])
    nt = int(d.end[t] - d.begin[t])
    ns = int(d.end[s] - d.begin[s])
    o = int(d.near_off[i])
    return d.near[o:o + nt * ns].reshape(ns, nt).T


def h2_apply_tree(d, u: np.ndarray) -> np.ndarray:
    """y = G u for u in tree order, shape (n_vox, ncol)."""
    ncl = int(d.level.shape[0])
    depth = int(d.level.max())
    xh = [None] * ncl
    yh = [None] * ncl
    # 1. forward transformation, leaves then levels bottom up
    for lev in range(depth, -1, -1):
        for c in np.nonzero(d.level == lev)[0]:
            if d.rank[c] == 0:
                continue
            if d.nchild[c] == 0:
                xh[c] = _basis(d, c).T @ u[d.begin[c]:d.end[c]]
            else:
                acc = np.zeros((int(d.rank[c]), u.shape[1]), np.complex128)
                for ch in range(d.first_child[c], d.first_child[c] + d.nchild[c]):
                    if d.rank[ch] > 0:
                        acc += _transfer(d, ch).T @ xh[ch]
                xh[c] = acc
    # 2. coupling multiplication
    for c in range(ncl):
        if d.rank[c] > 0:
            yh[c] = np.zeros((int(d.rank[c]), u.shape[1]), np.complex128)
    for i in range(d.far_t.shape[0]):
        t, s = int(d.far_t[i]), int(d.far_s[i])
        yh[t] += _coupling(d, i) @ xh[s]
    # 3. backward transformation, top down
    y = np.zeros_like(u)
    for lev in range(0, depth + 1):
        for c in np.nonzero(d.level == lev)[0]:
            if d.rank[c] == 0:
                continue
            p = int(d.parent[c])
            if p >= 0 and d.rank[p] > 0:
                yh[c] += _transfer(d, c) @ yh[p]
            if d.nchild[c] == 0:
                y[d.begin[c]:d.end[c]] += _basis(d, c) @ yh[c]
    # 4. inadmissible blocks in full
    for i in range(d.near_t.shape[0]):
        t, s = int(d.near_t[i]), int(d.near_s[i])
        y[d.begin[t]:d.end[t]] += _near(d, i) @ u[d.begin[s]:d.end[s]]
    return y


def h2_matvec(d, x: np.ndarray, op: str = "Z") -> np.ndarray:
    """Apply op in {"Z", "G"} to x of shape (3*n_vox,) or (3*n_vox, nrhs), caller ordering."""
    n = int(d.n_vox)
    X = np.ascontiguousarray(x, dtype=np.complex128).reshape(n, -1)
    U = X if op == "G" else d.chi[:, None] * X
    u_tree = U[d.perm]
    y_tree = h2_apply_tree(d, u_tree)
    Y = np.empty_like(y_tree)
    Y[d.perm] = y_tree
    if op == "G":
        return Y.reshape(x.shape)
    return (X + d.sigma * d.k * d.k * d.volume * Y).reshape(x.shape)


def densify(d, op: str = "Z") -> np.ndarray:
    """Dense matrix of the represented operator on the 3*n_vox unknowns (tiny inputs only)."""
    n = int(d.n_vox)
    N = 3 * n
    cols = []
    E = np.eye(N, dtype=np.complex128)
    for j in range(0, N, 256):
        cols.append(h2_matvec(d, E[:, j:j + 256], op))
    return np.concatenate(cols, axis=1)
