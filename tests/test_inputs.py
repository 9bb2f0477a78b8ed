"""Pins of the seeded input generators (P2): the plane-wave right-hand side and
the random test vectors, against what a plane wave and a CN(0, 1) draw are."""
import numpy as np

import h2gen
from h2gen.rhs import plane_wave_params


def test_plane_wave_is_transverse_unit_and_seeded():
    d, p = plane_wave_params(7, count=400)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    assert np.allclose(np.linalg.norm(p, axis=1), 1.0, atol=1e-15)
    assert np.abs(np.sum(d * p, axis=1)).max() <= 1e-15           # p . d = 0
    d2, p2 = plane_wave_params(7, count=400)
    assert np.array_equal(d, d2) and np.array_equal(p, p2)        # reproducible from the seed
    d3, _ = plane_wave_params(8, count=400)
    assert not np.array_equal(d, d3)


def test_plane_wave_directions_uniform_on_the_sphere():
    d, p = plane_wave_params(11, count=200000)
    # uniform on the sphere: mean 0, second moments 1/3 each, no cross moments
    assert np.abs(d.mean(axis=0)).max() < 0.01
    assert np.allclose((d * d).mean(axis=0), 1.0 / 3.0, atol=0.005)
    assert abs(np.mean(d[:, 0] * d[:, 1])) < 0.005
    # polarisation angle uniform in the transverse plane: p averages to 0 as well
    assert np.abs(p.mean(axis=0)).max() < 0.01


def test_plane_wave_samples_exp_minus_jkdr():
    g = h2gen.cube(6, 0.5, 4.0)
    b = h2gen.plane_wave(g, 3, count=2)
    d, p = plane_wave_params(3, count=2)
    r = g.centres()
    for w in range(2):
        bw = b[w].reshape(g.n_vox, 3)
        # |b_{3i+c}| = |p_c| at every voxel
        assert np.allclose(np.abs(bw), np.abs(p[w])[None, :], atol=1e-14)
        # b_i = p exp(-j k d . r_i): the ratio between two voxels is the phase of their offset
        i, j = 5, 170
        ratio = bw[i] / bw[j]
        mask = np.abs(p[w]) > 1e-3
        expect = np.exp(-1j * g.k * d[w] @ (r[i] - r[j]))
        assert np.allclose(ratio[mask], expect, atol=1e-12)
        # it satisfies the Helmholtz relation of a plane wave: a step h along axis a multiplies
        # by exp(-j k h d_a)
        bb = bw.reshape(6, 6, 6, 3)
        assert np.allclose(bb[1:] / bb[:-1], np.exp(-1j * g.k * g.h * d[w, 0]), atol=1e-12)


def test_random_vector_is_standard_complex_normal():
    x = h2gen.random_vector(400000, 3)
    assert abs(x.mean()) < 0.005
    assert abs(np.mean(np.abs(x) ** 2) - 1.0) < 0.01               # E|x|^2 = 1
    assert abs(np.mean(x * x)) < 0.005                              # circular: E x^2 = 0
    assert np.array_equal(x, h2gen.random_vector(400000, 3))
