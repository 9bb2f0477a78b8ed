"""Seeded right-hand sides and test vectors.

* random_vector: x ~ CN(0, 1) = (N(0,1) + j N(0,1)) / sqrt(2), PCG64 from the seed.
* plane_wave: incidence d uniform on the sphere (cos(theta) ~ U[-1,1],
  phi ~ U[0, 2 pi)), polarisation p = cos(psi) e_theta + sin(psi) e_phi with
  psi ~ U[0, 2 pi), sampled at voxel centres: b[3i+c] = p_c exp(-j k d.r_i)
  (exp(+j omega t) convention, as in g of eq. (1)).
* paper_excitation: the fixed incidence of Sec. V.B-D, travelling along -y and
  polarised along z: b[3i+c] = delta_{c,z} exp(+j k y_i).
"""

from __future__ import annotations

import numpy as np

from .geometry import Geometry


def random_vector(n: int, seed: int, ncols: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    shape = (n,) if ncols is None else (ncols, n)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    return x.astype(np.complex128)


def plane_wave_params(seed: int, count: int = 1):
    rng = np.random.default_rng(seed)
    cth = rng.uniform(-1.0, 1.0, size=count)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=count)
    psi = rng.uniform(0.0, 2.0 * np.pi, size=count)
    sth = np.sqrt(1.0 - cth * cth)
    d = np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)
    e_th = np.stack([cth * np.cos(phi), cth * np.sin(phi), -sth], axis=1)
    e_ph = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=1)
    p = np.cos(psi)[:, None] * e_th + np.sin(psi)[:, None] * e_ph
    return d, p


def plane_wave(geom: Geometry, seed: int, count: int = 1) -> np.ndarray:
    """(count, 3*n_vox) complex128 plane waves in the caller's (C-order voxel) ordering."""
    d, p = plane_wave_params(seed, count)
    r = geom.centres()
    phase = np.exp(-1j * geom.k * (r @ d.T))          # (n_vox, count)
    b = phase.T[:, :, None] * p[:, None, :]           # (count, n_vox, 3)
    return b.reshape(count, -1).astype(np.complex128)


def plane_wave_dir(geom: Geometry, d, p) -> np.ndarray:
    """(3*n_vox,) plane wave travelling along the unit vector d with polarisation p."""
    d = np.asarray(d, np.float64)
    p = np.asarray(p, np.complex128)
    phase = np.exp(-1j * geom.k * (geom.centres() @ d))
    return (phase[:, None] * p[None, :]).reshape(-1).astype(np.complex128)


def paper_excitation(geom: Geometry) -> np.ndarray:
    """Sec. V.B-D: incidence along -y, polarised along z."""
    return plane_wave_dir(geom, (0.0, -1.0, 0.0), (0.0, 0.0, 1.0))

