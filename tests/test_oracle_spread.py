"""Pins of the oracle's Map-Charge step (Section 2.1 step 1, Section 3.1).

Brute force: the mesh charge at every grid point written from the charge
assignment function itself (truncated-power B-spline, all periodic images),
with no stencil-start or fraction bookkeeping.  Plus exact invariants: total
charge, linearity, translation by a mesh vector, mirror symmetry, dipole.
"""
import math

import numpy as np
import pytest

from oracle import oracle as o
from workloads import random_system


def m_spline(n, x):
    total = 0.0
    for k in range(n + 1):
        if x - k > 0:
            total += (-1) ** k * math.comb(n, k) * (x - k) ** (n - 1)
    return total / math.factorial(n - 1)


def brute_force_rho(pos, q, lo, length, mesh, P):
    """rho_m = sum_i q_i prod_d sum_n W(u_id - m_d - n K_d),  W(t) = M_P(t + P/2)."""
    lo = np.asarray(lo, float)
    length = np.asarray(length, float)
    mesh = np.asarray(mesh)
    h = length / mesh
    rho = np.zeros((mesh[2], mesh[1], mesh[0]))
    for i in range(len(q)):
        u = np.mod((pos[i] - lo) / h, mesh)
        fac = []
        for d in range(3):
            K = mesh[d]
            fac.append(np.array([sum(m_spline(P, u[d] - m - n * K + 0.5 * P) for n in (-1, 0, 1))
                                 for m in range(K)]))
        rho += q[i] * fac[2][:, None, None] * fac[1][None, :, None] * fac[0][None, None, :]
    return rho


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6, 7])
def test_brute_force_mesh_charge(P):
    lo, length, mesh = (-1.5, 0.25, 3.0), (9.0, 7.5, 11.0), (8, 9, 10)
    pos, q = random_system(7, length, seed=10 + P, box_lo=lo)
    box = o.Box(lo, length, mesh, P)
    rho = o.make_rho(pos, q, box)
    ref = brute_force_rho(pos, q, lo, length, mesh, P)
    # the truncated-power sum cancels terms of size ~P^(P-1)/(P-1)!, so allow ~1e-11
    np.testing.assert_allclose(rho, ref, atol=1e-11 * np.abs(q).sum())


@pytest.mark.parametrize("P", [2, 3, 5, 7])
def test_total_charge_and_linearity(P):
    lo, length, mesh = (0.0, 0.0, 0.0), (12.0, 10.0, 14.0), (12, 10, 16)
    pos, q = random_system(300, length, seed=P, charge="positive")
    box = o.Box(lo, length, mesh, P)
    rho = o.make_rho(pos, q, box)
    assert abs(rho.sum() - q.sum()) < 1e-12 * q.sum()
    q2 = np.random.default_rng(1).normal(size=q.shape)
    rho2 = o.make_rho(pos, q2, box)
    rho3 = o.make_rho(pos, 2.0 * q - 3.0 * q2, box)
    np.testing.assert_allclose(rho3, 2.0 * rho - 3.0 * rho2, atol=1e-12)


@pytest.mark.parametrize("P", [3, 4, 5, 7])
def test_translation_by_mesh_vector_rolls_the_mesh(P):
    lo, length, mesh = (0.0, 0.0, 0.0), (10.0, 12.0, 9.0), (10, 12, 9)
    h = np.asarray(length) / np.asarray(mesh)
    pos, q = random_system(50, length, seed=20 + P)
    box = o.Box(lo, length, mesh, P)
    rho = o.make_rho(pos, q, box)
    a = np.array([3, -5, 7])  # mesh vector (x, y, z)
    rho_t = o.make_rho(pos + a * h, q, box)
    np.testing.assert_allclose(rho_t, np.roll(rho, (a[2], a[1], a[0]), axis=(0, 1, 2)), atol=1e-12)


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6, 7])
def test_mirror_symmetry(P):
    # x -> 2 lo - x maps mesh point m to -m (mod K) for a centred stencil
    lo, length, mesh = (1.0, -2.0, 0.5), (8.0, 9.0, 10.0), (8, 9, 10)
    pos, q = random_system(40, length, seed=30 + P, box_lo=lo)
    box = o.Box(lo, length, mesh, P)
    rho = o.make_rho(pos, q, box)
    rho_m = o.make_rho(2 * np.asarray(lo) - pos, q, box)
    flipped = np.roll(rho[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))
    np.testing.assert_allclose(rho_m, flipped, atol=1e-12)


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6, 7])
def test_dipole_moment_is_exact(P):
    # charges far from the faces: no stencil wraps, so sum_m m rho_m = sum_i q_i u_i
    K = 24
    box = o.Box((0, 0, 0), (24.0, 24.0, 24.0), (K, K, K), P)
    rng = np.random.default_rng(40 + P)
    pos = rng.uniform(P, K - P, size=(30, 3))
    q = rng.normal(size=30)
    rho = o.make_rho(pos, q, box)
    m = np.arange(K)
    dip = np.array([np.sum(rho * m[None, None, :]), np.sum(rho * m[None, :, None]),
                    np.sum(rho * m[:, None, None])])
    np.testing.assert_allclose(dip, q @ pos, atol=1e-11)
    if P >= 3:
        # second moment about each charge: sum_m (m - u)^2 W = P / 12 per axis
        quad = np.sum(rho * (m[None, None, :] ** 2)) - np.sum(q * pos[:, 0] ** 2)
        assert abs(quad - P / 12.0 * q.sum()) < 1e-10
