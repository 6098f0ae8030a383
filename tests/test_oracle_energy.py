"""Pins of the oracle's energy terms and adjoint.

* Madelung: the rock-salt lattice energy, a closed form from the lattice-sum
  literature (tests/golden/madelung_nacl.txt), reached by mesh + self +
  real-space terms (the real-space erfc sum is the test-only short-range part
  of the Ewald split of Section 2.1).
* Independence of the total energy from the splitting parameter g for a
  system with net charge: pins E_self and the neutralising-background term.
* Adjoint dE/dq and dE/dr against central finite differences of the FP64
  energy (exact for q, because E is quadratic in the charges).
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as o
from workloads import nacl_lattice, random_system


def madelung_constant():
    with open(os.path.join(os.path.dirname(__file__), "golden", "madelung_nacl.txt")) as fh:
        for line in fh:
            if line.startswith("M "):
                return float(line.split()[1])
    raise RuntimeError("no Madelung constant in the fixture")


@pytest.mark.parametrize("K,tol", [(16, 1e-6), (32, 1e-8)])
@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_madelung_energy_of_rock_salt(K, tol, diff):
    pos, q, L = nacl_lattice(8, 2.5)
    g = 0.3
    r = o.pppm(pos, q, (0, 0, 0), (L,) * 3, (K,) * 3, 5, g, 1.0, diff)
    e_real, _ = o.ewald_real(pos, q, (L,) * 3, g)
    exact = -(len(q) / 2) * madelung_constant() / 2.5
    assert abs((r["energy"] + e_real - exact) / exact) < tol
    # every ion of a perfect lattice is a centre of symmetry: zero force
    assert np.max(np.abs(r["forces"])) < 1e-9


def test_total_energy_independent_of_splitting_for_charged_system():
    # net charge +2.3: the background term matters; total must not depend on g
    length = (9.0, 10.0, 11.0)
    pos, q = random_system(12, length, seed=55, charge="positive")
    energies = []
    for g in (0.45, 0.55, 0.65):
        e_tot, _ = o.ewald_total(pos, q, length, g)
        energies.append(e_tot)
    assert max(energies) - min(energies) < 1e-9 * abs(energies[0])
    # PPPM mesh term in place of the Ewald k-sum: same within discretisation error
    pppm_e = []
    for g in (0.45, 0.55, 0.65):
        r = o.pppm(pos, q, (0, 0, 0), length, (48, 48, 48), 7, g, 1.0, "ad")
        e_real, _ = o.ewald_real(pos, q, length, g)
        pppm_e.append(r["energy"] + e_real)
    assert max(abs(e - energies[0]) for e in pppm_e) < 1e-5 * abs(energies[0])
    # the background term is what makes this hold: without it the spread is large
    bg = [o.background_energy(q, g, 1.0, float(np.prod(length))) for g in (0.45, 0.65)]
    assert abs(bg[0] - bg[1]) > 1e-3 * abs(energies[0])


@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_adjoint_against_finite_differences(diff):
    lo, length, mesh, P, g, C = (0.0, 1.0, -2.0), (8.0, 9.0, 10.0), (8, 10, 12), 5, 0.5, 1.7
    pos, q = random_system(5, length, seed=77, box_lo=lo)
    q = q + 0.3  # net charge, so the background term enters dE/dq
    adj = o.energy_gradients(pos, q, lo, length, mesh, P, g, C, diff)
    G = adj["res"]["G"]

    def energy(p, qq):
        return o.pppm(p, qq, lo, length, mesh, P, g, C, diff, G=G)["energy"]

    hq = 1e-3
    fd_q = np.array([(energy(pos, q + hq * e) - energy(pos, q - hq * e)) / (2 * hq)
                     for e in np.eye(len(q))])
    np.testing.assert_allclose(adj["grad_q"], fd_q, rtol=1e-9, atol=1e-9 * np.abs(fd_q).max())
    hr = 1e-4
    fd_r = np.zeros_like(pos)
    for i in range(pos.shape[0]):
        for d in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, d] += hr
            p2[i, d] -= hr
            fd_r[i, d] = (energy(p1, q) - energy(p2, q)) / (2 * hr)
    err = np.linalg.norm(adj["grad_pos"] - fd_r) / np.linalg.norm(fd_r)
    assert err < 1e-6


def test_self_energy_of_isolated_gaussian_split():
    # the self term equals minus the smooth part of a unit charge's own
    # potential at its centre: C q^2 lim_{r->0} erf(g r)/r / 2 = C q^2 g/sqrt(pi)
    g, C = 0.37, 2.0
    r = 1e-7
    own = C * math.erf(g * r) / r
    assert abs(o.self_energy(np.array([1.0]), g, C) + 0.5 * own) < 1e-12
