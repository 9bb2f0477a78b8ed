"""Voxelised dielectric bodies (seeded, synthetic).

A body is a box of nx*ny*nz equal cubic voxels of edge h, wavelength 1
(k = 2*pi), with a relative permittivity per voxel.  The scalar operator the
hot path applies is

    Z x = x + sigma * k^2 * V * (G (x) I_3) (chi . x),   chi = eps_r - 1,

with G_ij = exp(-j k r_ij) / (4 pi r_ij) between voxel centres (the free-space
Green's function g of eq. (1)) and the diagonal G_ii set so that V*G_ii equals
the integral of g over the sphere of volume V centred on the voxel.  The
contrast multiplies the source side (kappa(r') sits inside the integral of
eq. (1)), so G itself stays complex symmetric.

Distances are computed from integer voxel offsets, r_ij = h*sqrt(dx^2+dy^2+dz^2),
so r_ij and r_ji are bitwise equal and G is exactly symmetric and
translation invariant on the grid.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclass
class Geometry:
    shape: tuple            # (nx, ny, nz) voxels
    h: float                # voxel edge in wavelengths
    eps_r: np.ndarray       # (n_vox,) complex128, C-order over (nx, ny, nz)
    k: float = TWO_PI       # wavenumber (wavelength 1)
    sigma: float = 1.0      # sign of the scattering term
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_vox(self) -> int:
        return int(np.prod(self.shape))

    @property
    def volume(self) -> float:
        return self.h ** 3

    @property
    def chi(self) -> np.ndarray:
        return (self.eps_r - 1.0).astype(np.complex128)

    def coords(self) -> np.ndarray:
        """Integer voxel coordinates (n_vox, 3) in C order of `shape`."""
        nx, ny, nz = self.shape
        ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        return np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.int64)

    def centres(self) -> np.ndarray:
        return (self.coords().astype(np.float64) + 0.5) * self.h

    def self_term(self) -> complex:
        """G_ii: (1/V) * integral of g over the equal-volume sphere.

        With a = (3V/(4 pi))^(1/3):  int_0^a r e^{-jkr} dr = ((1+jka) e^{-jka} - 1)/k^2.
        """
        a = (3.0 * self.volume / (4.0 * np.pi)) ** (1.0 / 3.0)
        k = self.k
        integral = ((1.0 + 1j * k * a) * np.exp(-1j * k * a) - 1.0) / (k * k)
        return complex(integral / self.volume)

    def green_table(self) -> np.ndarray:
        """G as a function of the squared integer offset d2 (index 0 = self term).

        The generator evaluates every block through this table; it holds the
        same value the closed form gives for each distance on the grid.
        """
        nx, ny, nz = self.shape
        dmax = (nx - 1) ** 2 + (ny - 1) ** 2 + (nz - 1) ** 2
        d2 = np.arange(dmax + 1, dtype=np.float64)
        r = self.h * np.sqrt(d2)
        tab = np.empty(dmax + 1, dtype=np.complex128)
        with np.errstate(divide="ignore", invalid="ignore"):
            tab[1:] = np.exp(-1j * self.k * r[1:]) / (4.0 * np.pi * r[1:])
        tab[0] = self.self_term()
        return tab


def cube(n: int, side_wavelengths: float, eps=4.0, seed: int | None = None,
         sigma: float = 1.0, name: str = "") -> Geometry:
    """n^3 cube of side `side_wavelengths`; eps is a constant or (lo, hi) drawn per voxel."""
    h = side_wavelengths / n
    nv = n ** 3
    if isinstance(eps, tuple):
        rng = np.random.default_rng(seed)
        e = rng.uniform(eps[0], eps[1], size=nv)
    else:
        e = np.full(nv, float(eps))
    return Geometry((n, n, n), h, e.astype(np.complex128), sigma=sigma,
                    name=name or f"cube{n}", meta={"eps": eps, "seed": seed})


def box(shape, h: float, eps=4.0, seed: int | None = None, sigma: float = 1.0,
        name: str = "") -> Geometry:
    """General nx*ny*nz box with voxel edge h (rods and slabs of the scaling tests)."""
    nv = int(np.prod(shape))
    if isinstance(eps, tuple):
        rng = np.random.default_rng(seed)
        e = rng.uniform(eps[0], eps[1], size=nv)
    else:
        e = np.full(nv, float(eps))
    return Geometry(tuple(int(s) for s in shape), h, e.astype(np.complex128), sigma=sigma,
                    name=name or "box%dx%dx%d" % tuple(shape), meta={"eps": eps, "seed": seed})


def slab(shape=(96, 96, 48), thickness_wavelengths=2.0, n_layers=6, eps_range=(1.0, 10.0),
         seed: int = 5, sigma: float = 1.0) -> Geometry:
    """Layered slab: n_layers-1 distinct seeded cut planes along z, eps_r ~ U(eps_range) per layer."""
    nx, ny, nz = shape
    h = thickness_wavelengths / nz
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.choice(np.arange(1, nz), size=n_layers - 1, replace=False))
    layer_eps = rng.uniform(eps_range[0], eps_range[1], size=n_layers)
    layer_of_z = np.searchsorted(cuts, np.arange(nz), side="right")
    ez = layer_eps[layer_of_z]
    e = np.broadcast_to(ez[None, None, :], (nx, ny, nz)).reshape(-1)
    return Geometry((nx, ny, nz), h, e.astype(np.complex128), sigma=sigma,
                    name="slab%dx%dx%d" % shape,
                    meta={"cuts": cuts.tolist(), "layer_eps": layer_eps.tolist(), "seed": seed})


def uneven_cubes(count=32, edge_range=(8, 48), eps_range=(1.5, 8.0), h=1.0 / 16.0,
                 seed: int = 4, sigma: float = 1.0):
    """`count` independent cubes with edges ~ U{edge_range} and eps_r ~ U(eps_range) per voxel."""
    rng = np.random.default_rng(seed)
    edges = rng.integers(edge_range[0], edge_range[1] + 1, size=count)
    out = []
    for i, n in enumerate(edges):
        n = int(n)
        e = rng.uniform(eps_range[0], eps_range[1], size=n ** 3)
        out.append(Geometry((n, n, n), h, e.astype(np.complex128), sigma=sigma,
                            name=f"ucube{i}_{n}", meta={"seed": seed, "index": i}))
    return out


# ---------------------------------------------------------------- the paper's Sec. V bodies
# Voxel versions of the three scaling workloads of Sec. V.B-D: relative permittivity
# 2.54 throughout, voxel edge lambda/20 by default.  The paper discretises the bodies
# with SWG functions; here they are voxelised on the same grid as every other body.

PAPER_EPS = 2.54


def paper_rod(length_wavelengths: float, h: float = 1.0 / 20.0) -> Geometry:
    """Sec. V.B: a rod of cross-section lambda/10 x lambda/10 (2 x 2 voxels at h = lambda/20)
    and the given length along x."""
    side = max(1, int(round(0.1 / h)))
    n = max(1, int(round(length_wavelengths / h)))
    return box((n, side, side), h, eps=PAPER_EPS, name=f"rod{length_wavelengths:g}L")


def paper_slab(side_wavelengths: float, h: float = 1.0 / 20.0) -> Geometry:
    """Sec. V.C: a slab lambda/10 thick (2 voxels at h = lambda/20), square in x and y."""
    t = max(1, int(round(0.1 / h)))
    n = max(1, int(round(side_wavelengths / h)))
    return box((n, n, t), h, eps=PAPER_EPS, name=f"slab{side_wavelengths:g}L")


def paper_cube_array(count: int, cube_voxels: int = 6, h: float = 1.0 / 20.0) -> Geometry:
    """Sec. V.D: count^3 dielectric cubes of edge 0.3 lambda (cube_voxels at h = lambda/20),
    neighbours 0.3 lambda apart.  The body is the array's bounding box with eps_r = 1
    (chi = 0) in the gaps: the gap voxels carry no source and their unknowns are the
    field there, so the cubes' unknowns solve the same equations as with the cubes
    alone."""
    m = count * cube_voxels + (count - 1) * cube_voxels
    on = (np.arange(m) // cube_voxels) % 2 == 0          # cube, gap, cube, ... along each axis
    mask = on[:, None, None] & on[None, :, None] & on[None, None, :]
    e = np.where(mask.reshape(-1), PAPER_EPS, 1.0)
    return Geometry((m, m, m), h, e.astype(np.complex128), name=f"cubearray{count}",
                    meta={"count": count, "cube_voxels": cube_voxels})

