"""The seeded synthetic systems have the advertised shape (counts, neutrality, geometry)."""
import math

import numpy as np
import pytest

import workloads as W


def test_config1_alternating():
    w = W.config(1)
    assert w.n == 1000 and w.mesh == (16, 16, 16) and w.order == 5
    assert np.all(w.q[::2] == 1) and np.all(w.q[1::2] == -1)
    assert np.all((w.pos >= 0) & (w.pos < 20.0))


def test_config2_water_geometry_and_density():
    w = W.config(2)
    assert w.n == 32001
    assert abs(w.q.sum()) < 1e-9
    L = 68.0
    o_pos, h1, h2 = w.pos[0::3], w.pos[1::3], w.pos[2::3]

    def mic(d):  # minimum image
        return d - L * np.round(d / L)

    d1, d2 = mic(h1 - o_pos), mic(h2 - o_pos)
    np.testing.assert_allclose(np.linalg.norm(d1, axis=1), 1.0, atol=1e-9)
    np.testing.assert_allclose(np.linalg.norm(d2, axis=1), 1.0, atol=1e-9)
    cosang = np.sum(d1 * d2, axis=1)
    np.testing.assert_allclose(np.degrees(np.arccos(cosang)), 109.47, atol=1e-6)
    # liquid water: about 0.0334 molecules per cubic angstrom
    dens = (w.n // 3) / L ** 3
    assert 0.03 < dens < 0.04


def test_config3_exactly_neutral_pm1():
    w = W.config(3)
    assert w.n == 524288 and w.mesh == (128,) * 3
    assert np.sum(w.q == 1) == np.sum(w.q == -1) == 262144
    assert W.config(3, order=7).order == 7


def test_config4_gaussian_neutral():
    w = W.config(4)
    assert w.n == 65536
    assert abs(w.q.sum()) < 1e-9
    assert 0.45 < w.q.std() < 0.55


@pytest.mark.slow
def test_config5_size():
    w = W.config(5)
    assert w.n == 4194304 and w.mesh == (256,) * 3 and w.order == 7
    assert w.q[-1] == 0.0
    assert abs(w.q.sum()) < 1e-6


def test_seeded_reproducible():
    a, b = W.config(1), W.config(1)
    np.testing.assert_array_equal(a.pos, b.pos)
    p1, q1 = W.random_system(10, (3, 4, 5), seed=1)
    p2, q2 = W.random_system(10, (3, 4, 5), seed=1)
    np.testing.assert_array_equal(p1, p2)


def test_nacl_lattice():
    pos, q, L = W.nacl_lattice(8, 2.5)
    assert len(q) == 512 and L == 20.0 and q.sum() == 0


def test_interfacial_slab():
    w = W.interfacial()
    assert w.n == 524288 and w.q.sum() == 0 and np.all(np.abs(w.q) == 1)
    assert np.all(w.pos[:, 2] < 85.0) and np.all(w.pos >= 0)
    # x and y still span the whole box
    assert w.pos[:, 0].max() > 169.0 and w.pos[:, 1].max() > 169.0
