"""Voxel versions of the paper's scaling workloads (Sec. V.B-D): the rod, the slab and
the array of cubes, eps_r = 2.54, with the fixed incidence (along -y, polarised along
z).  Host checks: the bodies and the excitation as the section states them, the
representation against the brute-force product, and the two properties Fig. 7 reports
for the rod (rank and iteration count independent of the length)."""
import numpy as np
import pytest

import h2gen
from h2gen.construct import build_h2
from oracle import krylov as ok
from oracle import matvec as om
from oracle.kernel import dense_Z_matvec


def test_bodies_as_stated():
    r = h2gen.paper_rod(8)                        # lambda/10 x lambda/10 cross-section at h = lambda/20
    assert r.shape == (160, 2, 2) and np.isclose(r.h * 2, 0.1) and np.isclose(r.h * 160, 8.0)
    s = h2gen.paper_slab(2)                       # lambda/10 thick
    assert s.shape == (40, 40, 2) and np.isclose(s.h * 2, 0.1)
    for g in (r, s):
        assert np.all(g.eps_r == 2.54)
    a = h2gen.paper_cube_array(3)                 # cubes of 0.3 lambda, 0.3 lambda apart
    assert a.shape == (30, 30, 30) and np.isclose(6 * a.h, 0.3)
    eps = a.eps_r.reshape(a.shape).real
    assert np.count_nonzero(eps == 2.54) == 27 * 6 ** 3
    assert np.count_nonzero(eps == 1.0) == 30 ** 3 - 27 * 6 ** 3
    # one cube is a solid 6^3 block, the next one starts 6 voxels further on
    assert np.all(eps[0:6, 0:6, 0:6] == 2.54) and np.all(eps[6:12, :, :] == 1.0)
    assert np.all(eps[12:18, 12:18, 24:30] == 2.54)
    # chi = 0 in the gaps: those columns of Z - I vanish
    assert np.all(a.chi[eps.reshape(-1) == 1.0] == 0)


def test_excitation_direction_and_polarisation():
    g = h2gen.paper_rod(2)
    b = h2gen.paper_excitation(g).reshape(-1, 3)
    assert np.all(b[:, :2] == 0)                  # z-polarised
    y = g.centres()[:, 1]
    assert np.allclose(b[:, 2], np.exp(1j * g.k * y))   # exp(+j k y): travelling along -y
    assert np.allclose(np.abs(b[:, 2]), 1.0)


@pytest.mark.parametrize("make,eps,bound", [
    (lambda: h2gen.paper_rod(8), 1e-3, 1e-4),
    (lambda: h2gen.paper_slab(2), 1e-3, 3e-4),
    (lambda: h2gen.paper_cube_array(2, 4), 1e-3, 3e-4),
])
def test_representation_against_brute_force(make, eps, bound):
    g = make()
    d = build_h2(g, eps=eps)
    x = h2gen.random_vector(3 * g.n_vox, 5)
    yd = dense_Z_matvec(g.shape, g.h, g.k, g.chi, g.sigma, x)
    e = np.linalg.norm(om.h2_matvec(d, x) - yd) / np.linalg.norm(yd)
    assert e < bound


def test_rod_rank_and_iterations_do_not_grow_with_length():
    """Fig. 7: on the rod the accuracy-determined rank and the BiCGStab iteration count
    at 1e-3 stay constant as the rod gets longer."""
    ranks, its = [], []
    for L in (8, 32, 128):
        g = h2gen.paper_rod(L)
        d = build_h2(g, eps=1e-3)
        ranks.append(int(d.rank.max()))
        _, rep = ok.bicgstab(lambda v: om.h2_matvec(d, v), h2gen.paper_excitation(g), tol=1e-3)
        assert rep.converged
        its.append(rep.iterations)
    assert max(ranks) == min(ranks)
    assert max(its) <= its[0]


def test_cube_array_gaps_do_not_change_the_cubes_equations():
    """The array of cubes is solved on its bounding box with chi = 0 in the gaps: the gap
    columns of Z are identity columns, and the cube voxels' part of the box solution
    solves the system restricted to the cube voxels alone."""
    from oracle.kernel import dense_G
    g = h2gen.paper_cube_array(2, cube_voxels=2)            # 6^3 box, 8 cubes of 2^3 voxels
    n = g.n_vox
    G = dense_G(g.shape, g.h, g.k)
    Zs = np.eye(n) + g.sigma * g.k ** 2 * g.volume * G * g.chi[None, :]   # scalar Z, one component
    gap = g.chi == 0
    assert gap.sum() == 6 ** 3 - 8 * 2 ** 3
    assert np.array_equal(Zs[:, gap], np.eye(n)[:, gap])
    b = h2gen.paper_excitation(g).reshape(n, 3)[:, 2]
    x = np.linalg.solve(Zs, b)
    cubes = ~gap
    xc = np.linalg.solve(Zs[np.ix_(cubes, cubes)], b[cubes])
    assert np.linalg.norm(x[cubes] - xc) <= 1e-12 * np.linalg.norm(xc)
