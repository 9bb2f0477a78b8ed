"""Green's function, self term and brute-force dense products (test infrastructure).

The scalar operator is the D-field VIE of eq. (1) reduced to a voxel
collocation with the scalar kernel g(r) = exp(-j k0 r) / (4 pi r):

    Z x = x + sigma * k^2 * V * (G (x) I_3) (chi . x),   chi = eps_r - 1,

where G_ij = g(r_ij) between voxel centres and V*G_ii is the integral of g over
the sphere with the voxel's volume.  The contrast sits on the source side, as
kappa(r') inside the integral of eq. (1).
"""

from __future__ import annotations

import numpy as np


def green(r: np.ndarray, k: float) -> np.ndarray:
    """g(r) = exp(-j k r) / (4 pi r) (eq. (1)); r > 0."""
    r = np.asarray(r, dtype=np.float64)
    return np.exp(-1j * k * r) / (4.0 * np.pi * r)


def sphere_radius(volume: float) -> float:
    return (3.0 * volume / (4.0 * np.pi)) ** (1.0 / 3.0)


def self_integral(volume: float, k: float) -> complex:
    """Integral of g over a ball of volume V centred on the source point.

    In spherical coordinates this is int_0^a r exp(-jkr) dr, whose antiderivative
    is (1 + jkr) exp(-jkr) / k^2.
    """
    a = sphere_radius(volume)
    return complex(((1.0 + 1j * k * a) * np.exp(-1j * k * a) - 1.0) / (k * k))


def grid_coords(shape) -> np.ndarray:
    """Integer voxel coordinates in C order of shape."""
    nx, ny, nz = shape
    out = np.empty((nx * ny * nz, 3), np.int64)
    n = 0
    for i in range(nx):
        for j in range(ny):
            for l in range(nz):
                out[n] = (i, j, l)
                n += 1
    return out


def dense_G(shape, h: float, k: float, rows=None) -> np.ndarray:
    """Dense G (rows x n_vox) in the caller's voxel order (C order of `shape`)."""
    c = grid_coords(shape).astype(np.float64) * h
    ri = c if rows is None else c[rows]
    diff = ri[:, None, :] - c[None, :, :]
    r = np.sqrt((diff * diff).sum(-1))
    with np.errstate(divide="ignore", invalid="ignore"):
        G = green(r, k)
    V = h ** 3
    sval = self_integral(V, k) / V
    G[r == 0.0] = sval
    return G


def dense_G_matvec(shape, h: float, k: float, u: np.ndarray, chunk: int = 512) -> np.ndarray:
    """y = (G (x) I) u for u of shape (n_vox, ncol), chunked over rows."""
    n = int(np.prod(shape))
    y = np.empty((n, u.shape[1]), np.complex128)
    for lo in range(0, n, chunk):
        rows = np.arange(lo, min(n, lo + chunk))
        y[rows] = dense_G(shape, h, k, rows) @ u
    return y


def dense_Z_matvec(shape, h: float, k: float, chi: np.ndarray, sigma: float, x: np.ndarray,
                   op: str = "Z") -> np.ndarray:
    """Brute-force product with x of shape (3*n_vox,) or (3*n_vox, nrhs), unknown 3i+c.

    op "G": (G (x) I_3) x;  op "Z": x + sigma k^2 V (G (x) I_3)(chi . x).
    """
    n = int(np.prod(shape))
    X = np.ascontiguousarray(x).reshape(n, -1)
    if op == "G":
        return dense_G_matvec(shape, h, k, X).reshape(x.shape)
    Y = dense_G_matvec(shape, h, k, chi[:, None] * X)
    return (X + sigma * k * k * h ** 3 * Y).reshape(x.shape)
