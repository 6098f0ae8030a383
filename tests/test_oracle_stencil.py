"""Pins of the oracle's particle map and stencil coefficients (Section 3.1).

The paper says only that the coefficients are a product of three polynomials
whose order equals the stencil size.  Read as the order-P cardinal B-spline,
they must satisfy textbook identities that these tests check against closed
forms and an independent definition of the spline (the truncated-power sum),
never against the oracle's own recursion.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as o

FRACS = [0.0, 1e-9, 0.125, 0.3, 0.5, 0.61, 0.875, 0.999999]


def truncated_power_bspline(n, x):
    """M_n(x) = 1/(n-1)! sum_k (-1)^k C(n,k) (x-k)_+^(n-1): the spline as an n-fold box convolution."""
    total = 0.0
    for k in range(n + 1):
        if x - k > 0:
            total += (-1) ** k * math.comb(n, k) * (x - k) ** (n - 1)
    return total / math.factorial(n - 1)


@pytest.mark.parametrize("f", FRACS)
def test_order2_is_linear_interpolation(f):
    w, dw = o.weights(2, f)
    np.testing.assert_allclose(w, [1 - f, f], atol=1e-15)
    np.testing.assert_allclose(dw, [-1.0, 1.0], atol=1e-15)


@pytest.mark.parametrize("f", FRACS)
def test_order3_closed_form(f):
    # P = 3: the nearest grid point is s + 1 and delta = u - (s + 1) = f - 1/2.
    d = f - 0.5
    w, _ = o.weights(3, f)
    np.testing.assert_allclose(w, [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], atol=1e-15)


@pytest.mark.parametrize("f", FRACS)
def test_order4_closed_form(f):
    # cubic B-spline pieces (4 - 6 t^2 + 3 |t|^3)/6 and (2 - |t|)^3 / 6
    w, _ = o.weights(4, f)
    exp = [(1 - f) ** 3 / 6, (4 - 6 * f * f + 3 * f ** 3) / 6,
           (1 + 3 * f + 3 * f * f - 3 * f ** 3) / 6, f ** 3 / 6]
    np.testing.assert_allclose(w, exp, atol=1e-15)


@pytest.mark.parametrize("P", range(2, 8))
@pytest.mark.parametrize("f", FRACS)
def test_weights_match_truncated_power_definition(P, f):
    w, _ = o.weights(P, f)
    exp = [truncated_power_bspline(P, f + P - 1 - j) for j in range(P)]
    np.testing.assert_allclose(w, exp, atol=2e-13)


@pytest.mark.parametrize("P", range(2, 8))
@pytest.mark.parametrize("f", FRACS)
def test_moments(P, f):
    """Partition of unity, exact first moment, second central moment P/12 for P >= 3."""
    w, dw = o.weights(P, f)
    # offsets of the stencil points from the charge, in mesh units: j - (f + P/2 - 1)
    x = np.arange(P) - (f + 0.5 * P - 1.0)
    assert abs(w.sum() - 1.0) < 1e-14
    assert abs(np.dot(w, x)) < 1e-14
    if P >= 3:
        assert abs(np.dot(w, x * x) - P / 12.0) < 1e-13
    # derivative coefficients: d/du of the moments above
    assert abs(dw.sum()) < 1e-14
    assert abs(np.dot(dw, np.arange(P)) - 1.0) < 1e-13


@pytest.mark.parametrize("P", range(2, 8))
@pytest.mark.parametrize("f", [0.1, 0.37, 0.5, 0.8])
def test_reflection_symmetry(P, f):
    w, dw = o.weights(P, f)
    wr, dwr = o.weights(P, 1.0 - f)
    np.testing.assert_allclose(w, wr[::-1], atol=1e-15)
    np.testing.assert_allclose(dw, -dwr[::-1], atol=1e-14)


@pytest.mark.parametrize("P", range(2, 8))
@pytest.mark.parametrize("f", [0.1, 0.37, 0.5, 0.8])
def test_derivative_coefficients_by_finite_difference(P, f):
    eps = 1e-6
    _, dw = o.weights(P, f)
    wp, _ = o.weights(P, f + eps)
    wm, _ = o.weights(P, f - eps)
    np.testing.assert_allclose(dw, (wp - wm) / (2 * eps), atol=1e-8)


@pytest.mark.parametrize("P", range(2, 8))
def test_edge_weight_vanishes_at_fraction_zero(P):
    # the spline is continuous and zero at the end of its support: the stencil
    # point s + P - 1 gets weight M_P(0) = 0 when f = 0 (tie-break harmlessness)
    w, _ = o.weights(P, 0.0)
    assert abs(w[P - 1]) < 1e-15
    w1, _ = o.weights(P, 1.0)
    assert abs(w1[0]) < 1e-15
    np.testing.assert_allclose(w1[1:], w[:-1], atol=1e-14)


@pytest.mark.parametrize("P", range(2, 8))
def test_stencil_start_centres_on_nearest_point(P):
    K = 16
    box = o.Box((0, 0, 0), (K * 1.0, K * 1.0, K * 1.0), (K, K, K), P)
    rng = np.random.default_rng(7)
    u = rng.uniform(0, K, size=(200, 3))
    s, f = o.particle_map(u, box)
    if P % 2:
        expect = np.floor(u + 0.5) - (P - 1) // 2
    else:
        expect = np.floor(u) - (P // 2 - 1)
    np.testing.assert_array_equal(s, expect.astype(np.int64))
    assert np.all((f >= 0) & (f < 1))
    np.testing.assert_allclose(s + f, u + 1 - 0.5 * P, atol=1e-12)


def test_particle_map_wraps_periodic_images():
    box = o.Box((-3.0, 1.0, 2.5), (11.0, 13.0, 7.0), (8, 10, 6), 5)
    rng = np.random.default_rng(3)
    pos = box.lo + rng.uniform(0, 1, size=(64, 3)) * box.len
    s0, f0 = o.particle_map(pos, box)
    for shift in (-3, -1, 1, 2):
        s1, f1 = o.particle_map(pos + shift * box.len, box)
        np.testing.assert_array_equal(np.mod(s1, box.mesh), np.mod(s0, box.mesh))
        np.testing.assert_allclose(f1, f0, atol=1e-9)
    # exactly on the upper face is the same point as the lower face
    edge = np.array([box.lo + box.len])
    s_e, f_e = o.particle_map(edge, box)
    s_l, f_l = o.particle_map(np.array([box.lo]), box)
    np.testing.assert_array_equal(np.mod(s_e, box.mesh), np.mod(s_l, box.mesh))
    np.testing.assert_allclose(f_e, f_l, atol=1e-12)


def test_cells_touched_ratio_matches_paper():
    # Section 2.3: a 7^3 stencil touches about 2.7x the cells of a 5^3 stencil
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "stencil_cells.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    assert 7 ** 3 / 5 ** 3 == pytest.approx(vals["ratio_7_to_5"], abs=1e-3)
    assert round(7 ** 3 / 5 ** 3, 1) == vals["paper_rounded"]
