"""Per-leaf MLP preconditioner, FP64 reference (test infrastructure).

The network is not from the paper, which has none; it is the learned
preconditioner added around the method.  One MLP with weights shared by every
leaf cluster maps a leaf's residual to a leaf correction:

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3,

with x = [Re r_t / s, Im r_t / s, Re chi_t] (components voxel-major, zero
padded to n_pad voxels), y = [Re z_t, Im z_t] / s, and s = ||r|| / sqrt(N).
Training minimises L = (0.5 / n) sum_i ||y_i - t_i||^2 with Adam on FP32
master weights; the forward and backward passes use the master weights
rounded to bfloat16 (the gradient is applied to the master copy).
"""

from __future__ import annotations

import numpy as np

from .precision import bf16_round


def dims(n_pad: int, hidden: int = 256):
    return 7 * n_pad, hidden, 6 * n_pad


def init_params(n_in: int, hidden: int, n_out: int, seed: int):
    """He-normal weights (fan-in), zero biases; float32 master copies."""
    rng = np.random.default_rng(seed)
    W1 = (rng.standard_normal((hidden, n_in)) * np.sqrt(2.0 / n_in)).astype(np.float32)
    W2 = (rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)).astype(np.float32)
    W3 = (rng.standard_normal((n_out, hidden)) * np.sqrt(1.0 / hidden)).astype(np.float32)
    return dict(W1=W1, b1=np.zeros(hidden, np.float32), W2=W2, b2=np.zeros(hidden, np.float32),
                W3=W3, b3=np.zeros(n_out, np.float32))


def rounded(p):
    """Weights as used in the passes: bf16-rounded matrices, float32 biases, all as float64."""
    return {k: (bf16_round(v).astype(np.float64) if k.startswith("W") else v.astype(np.float64)) for k, v in p.items()}


def forward(p, X: np.ndarray, keep: bool = False):
    """X (n, n_in) -> Y (n, n_out); p already rounded (float64)."""
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    Y = h2 @ p["W3"].T + p["b3"]
    if keep:
        return Y, (X, a1, h1, a2, h2)
    return Y


def loss_and_grads(p, X: np.ndarray, T: np.ndarray):
    """L = 0.5/n sum ||Y - T||^2 and its gradients with respect to every parameter."""
    n = X.shape[0]
    Y, (X_, a1, h1, a2, h2) = forward(p, X, keep=True)
    R = Y - T
    L = 0.5 * float((R * R).sum()) / n
    dY = R / n
    g = {}
    g["W3"] = dY.T @ h2
    g["b3"] = dY.sum(0)
    dh2 = (dY @ p["W3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ p["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ X_
    g["b1"] = dh1.sum(0)
    return L, g


def adam_step(master, m, v, g, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update of the float32 master weights (in place)."""
    for k in master:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        master[k] = (master[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)


def halo_table(d, shape):
    """Neighbour leaves on the voxel grid: for leaf q and offset o in {-1, 0, 1}^3
    (lexicographic, origin skipped), the leaf that holds the voxel at the leaf's
    centre voxel (lower middle) plus o times the leaf's extent; -1 off the grid."""
    leaves = [int(t) for t in np.nonzero(np.asarray(d.nchild) == 0)[0]]
    perm = np.asarray(d.perm)
    leaf_of = {}
    boxes = []
    for q, t in enumerate(leaves):
        pts = [np.unravel_index(int(v), shape) for v in perm[d.begin[t]:d.end[t]]]
        for p in pts:
            leaf_of[tuple(int(c) for c in p)] = q
        lo = [min(p[a] for p in pts) for a in range(3)]
        hi = [max(p[a] for p in pts) for a in range(3)]
        boxes.append((lo, hi))
    offsets = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]
    table = np.full((len(leaves), len(offsets)), -1, np.int64)
    for q, (lo, hi) in enumerate(boxes):
        for j, o in enumerate(offsets):
            probe = tuple(lo[a] + (hi[a] - lo[a]) // 2 + o[a] * (hi[a] - lo[a] + 1) for a in range(3))
            if all(0 <= probe[a] < shape[a] for a in range(3)):
                table[q, j] = leaf_of[probe]
    return table


def leaf_features(d, r: np.ndarray, n_pad: int, halo=None):
    """Features of every leaf for a residual r (caller order, length 3 n_vox); returns (X, leaves, s).
    With a neighbour table, 6 values per slot follow: the neighbour's mean [Re r_c, Im r_c] / s."""
    N = r.shape[0]
    s = float(np.linalg.norm(r)) / np.sqrt(N)
    s = s if s > 0 else 1.0
    leaves = np.nonzero(np.asarray(d.nchild) == 0)[0]
    slots = 0 if halo is None else halo.shape[1]
    X = np.zeros((leaves.size, 7 * n_pad + 6 * slots))
    R = r.reshape(-1, 3)
    means = np.zeros((leaves.size, 6))
    for q, t in enumerate(leaves):
        vox = np.asarray(d.perm)[d.begin[t]:d.end[t]]
        n = vox.size
        rt = R[vox] / s                                   # (n, 3)
        X[q, :3 * n] = rt.real.reshape(-1)
        X[q, 3 * n_pad:3 * n_pad + 3 * n] = rt.imag.reshape(-1)
        X[q, 6 * n_pad:6 * n_pad + n] = np.asarray(d.chi)[vox].real
        means[q, :3] = rt.real.mean(0)
        means[q, 3:] = rt.imag.mean(0)
    for q in range(leaves.size):
        for j in range(slots):
            nb = int(halo[q, j])
            if nb >= 0:
                X[q, 7 * n_pad + 6 * j:7 * n_pad + 6 * j + 6] = means[nb]
    return X, leaves, s


def leaf_targets(d, e: np.ndarray, r: np.ndarray, n_pad: int):
    """Targets [Re e_t, Im e_t] / s of every leaf (s from the residual r, as in the features)."""
    N = r.shape[0]
    s = float(np.linalg.norm(r)) / np.sqrt(N)
    s = s if s > 0 else 1.0
    leaves = np.nonzero(np.asarray(d.nchild) == 0)[0]
    T = np.zeros((leaves.size, 6 * n_pad))
    E = e.reshape(-1, 3)
    for q, t in enumerate(leaves):
        vox = np.asarray(d.perm)[d.begin[t]:d.end[t]]
        n = vox.size
        et = E[vox] / s
        T[q, :3 * n] = et.real.reshape(-1)
        T[q, 3 * n_pad:3 * n_pad + 3 * n] = et.imag.reshape(-1)
    return T


def scatter(d, Y: np.ndarray, s: float, n_pad: int, N: int) -> np.ndarray:
    """Assemble per-leaf outputs (Re, Im blocks of 3 n_pad) times s into a vector in caller order."""
    leaves = np.nonzero(np.asarray(d.nchild) == 0)[0]
    z = np.zeros((N // 3, 3), np.complex128)
    for q, t in enumerate(leaves):
        vox = np.asarray(d.perm)[d.begin[t]:d.end[t]]
        n = vox.size
        re = Y[q, :3 * n].reshape(n, 3)
        im = Y[q, 3 * n_pad:3 * n_pad + 3 * n].reshape(n, 3)
        z[vox] = (re + 1j * im) * s
    return z.reshape(-1)


def apply(d, p, r: np.ndarray, n_pad: int, on_blockdiag: bool = False, halo=None) -> np.ndarray:
    """z = MLP correction of every leaf, assembled in caller order; with on_blockdiag
    the correction is added to the block-diagonal solve of r."""
    X, leaves, s = leaf_features(d, r, n_pad, halo)
    z = scatter(d, forward(p, X), s, n_pad, r.shape[0])
    return z + blockdiag_apply(d, r) if on_blockdiag else z


def blockdiag_apply(d, r: np.ndarray) -> np.ndarray:
    """z_t = (Z_tt)^-1 r_t per leaf, Z_tt = I + sigma k^2 V G_tt diag(chi_t) on each component."""
    alpha = d.sigma * d.k * d.k * d.volume
    z = np.zeros_like(r).reshape(-1, 3)
    R = r.reshape(-1, 3)
    for i in range(d.near_t.shape[0]):
        t, s_ = int(d.near_t[i]), int(d.near_s[i])
        if t != s_:
            continue
        n = int(d.end[t] - d.begin[t])
        o = int(d.near_off[i])
        G = np.asarray(d.near[o:o + n * n]).reshape(n, n).T
        vox = np.asarray(d.perm)[d.begin[t]:d.end[t]]
        M = np.eye(n) + alpha * G * np.asarray(d.chi)[vox][None, :]
        z[vox] = np.linalg.solve(M, R[vox])
    return z.reshape(-1)
