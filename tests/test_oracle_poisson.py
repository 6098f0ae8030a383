"""Pins of the oracle's Poisson step (Equation 2; Section 2.1 step 2).

The FFT normalisation, the 4 pi, the Ewald screening factor and the sign are
checked against the continuum solution of the screened Poisson equation for a
single Fourier mode; the two energy forms against each other (Parseval); the
influence function against its small-k limit and its symmetry.
"""
import math

import numpy as np
import pytest

from oracle import oracle as o
from workloads import random_system


def mode_error(K, P, diff, n=(1, 2, 0), length=(30.0, 36.0, 24.0), g=0.3, C=2.5):
    """Max relative deviation of the mesh solution of rho = A h^3 cos(k.r) from the continuum.

    A charge density A cos(k.r) (charge per volume) has the long-range Ewald
    potential Phi = C A 4 pi exp(-k^2/4g^2)/k^2 cos(k.r) and field
    E = -grad Phi = C A 4 pi exp(-k^2/4g^2)/k^2 k sin(k.r).
    """
    # the mode has no z dependence, so a short z axis keeps the oracle fast
    box = o.Box((0, 0, 0), length, (K, K, 8), P)
    kvec = 2 * math.pi * np.asarray(n) / np.asarray(length)
    h = box.h
    z, y, x = np.meshgrid(np.arange(8) * h[2], np.arange(K) * h[1], np.arange(K) * h[0], indexing="ij")
    arg = kvec[0] * x + kvec[1] * y + kvec[2] * z
    A = 0.7
    rho = A * np.prod(h) * np.cos(arg)
    G = o.influence_function(box, g, diff)
    sol = o.poisson(rho, box, G, C, diff, want_phi=True)
    k2 = float(kvec @ kvec)
    amp = C * A * 4 * math.pi * math.exp(-k2 / (4 * g * g)) / k2
    err = np.max(np.abs(sol["phi"] - amp * np.cos(arg))) / amp
    if diff == "ik":
        for comp, kd in zip(("ex", "ey", "ez"), kvec):
            if kd != 0:
                err = max(err, np.max(np.abs(sol[comp] - amp * kd * np.sin(arg))) / (amp * abs(kd)))
            else:
                err = max(err, np.max(np.abs(sol[comp])) / amp)
    return err


@pytest.mark.parametrize("diff", ["ik", "ad"])
@pytest.mark.parametrize("P", [3, 5, 7])
def test_single_mode_converges_to_continuum(diff, P):
    length, n = np.array([30.0, 36.0, 24.0]), np.array([1, 2, 0])
    kvec = 2 * math.pi * n / length
    errs = {K: mode_error(K, P, diff) for K in (64, 128)}
    for K, err in errs.items():
        # for a smooth mode G ~ R / U^2(k): the mesh solution exceeds the
        # continuum by the B-spline deconvolution, 1 + P sum_d (k_d h_d)^2 / 12
        lead = P * float(np.sum((kvec * length / np.array([K, K, 8])) ** 2)) / 12.0
        assert abs(err / lead - 1.0) < 0.05
    # second-order convergence to the screened Poisson solution
    assert 3.8 < errs[64] / errs[128] < 4.2


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_parseval_energy_forms_agree(diff):
    length, mesh = (14.0, 11.0, 17.0), (14, 12, 16)
    pos, q = random_system(80, length, seed=5)
    box = o.Box((0, 0, 0), length, mesh, 5)
    rho = o.make_rho(pos, q, box)
    G = o.influence_function(box, 0.35, diff)
    sol = o.poisson(rho, box, G, 1.7, diff, want_phi=True)
    e_real_space = 0.5 * float(np.sum(rho * sol["phi"]))
    assert abs(sol["e_mesh"] - e_real_space) < 1e-12 * abs(sol["e_mesh"])
    assert sol["e_mesh"] > 0


@pytest.mark.parametrize("diff", ["ik", "ad"])
@pytest.mark.parametrize("P", [2, 5, 7])
def test_influence_function_symmetry_and_small_k_limit(diff, P):
    box = o.Box((0, 0, 0), (40.0, 40.0, 40.0), (64, 64, 64), P)
    g = 0.3
    G = o.influence_function(box, g, diff)
    assert G[0, 0, 0] == 0.0
    # G(k) = G(-k)
    flipped = np.roll(G[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))
    np.testing.assert_allclose(G, flipped, rtol=1e-12, atol=0)
    # G / R -> 1 as k h -> 0 (lowest mode along x)
    k = 2 * math.pi / 40.0
    R = 4 * math.pi * math.exp(-k * k / (4 * g * g)) / (k * k)
    assert abs(G[0, 0, 1] / R - 1.0) < P * (k * box.h[0]) ** 2 / 12.0 * 1.5
    if diff == "ad":
        assert np.all(G >= 0)  # every alias term of the ad numerator is non-negative


def test_mesh_energy_scales_quadratically_in_charge():
    length, mesh = (12.0, 12.0, 12.0), (16, 16, 16)
    pos, q = random_system(60, length, seed=9)
    base = o.pppm(pos, q, (0, 0, 0), length, mesh, 5, 0.3, 1.0, "ad")
    for alpha in (-1.0, 2.5):
        r = o.pppm(pos, alpha * q, (0, 0, 0), length, mesh, 5, 0.3, 1.0, "ad", G=base["G"])
        assert abs(r["e_mesh"] - alpha ** 2 * base["e_mesh"]) < 1e-12 * alpha ** 2 * base["e_mesh"]
