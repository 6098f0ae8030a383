"""Pins of the ad self-force correction: the leading-harmonic self-force of
oracle.ad_self_force_coefficients against the exact force on a lone charge
(which is all self-force), its symmetry, and the net-force improvement it
brings to a neutral system."""
import numpy as np
import pytest

from oracle import oracle as o


def lone_charge_forces(P, K, L, g, seed=1, n=30):
    box = o.Box((0, 0, 0), (L,) * 3, (K,) * 3, P)
    G = o.influence_function(box, g, "ad")
    coef = o.ad_self_force_coefficients(box, G)
    rng = np.random.default_rng(seed)
    exact, harm = [], []
    for _ in range(n):
        pos = rng.uniform(0, L, size=(1, 3))
        r = o.pppm(pos, np.array([1.3]), (0, 0, 0), (L,) * 3, (K,) * 3, P, g, 1.0, "ad", G=G)
        exact.append(r["forces"][0])
        harm.append(o.ad_self_force(pos, np.array([1.3]), box, coef, 1.0)[0])
    return np.array(exact), np.array(harm)


@pytest.mark.parametrize("P,tol", [(3, 0.06), (4, 0.08), (5, 0.01), (7, 0.01)])
def test_harmonics_match_the_lone_charge_force(P, tol):
    exact, harm = lone_charge_forces(P, 16, 16.0, 0.6)
    rel = np.sqrt(((exact - harm) ** 2).sum() / (exact ** 2).sum())
    assert rel < tol


def test_self_force_is_odd_and_vanishes_on_nodes_and_midpoints():
    box = o.Box((0, 0, 0), (12.0,) * 3, (12,) * 3, 5)
    coef = o.ad_self_force_coefficients(box, o.influence_function(box, 0.5, "ad"))
    q = np.ones(4)
    on = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5], [3.0, 7.5, 11.0], [1.5, 2.0, 4.5]])
    assert np.abs(o.ad_self_force(on, q, box, coef, 1.0)).max() < 1e-15
    u = np.array([[0.3, 1.2, 5.7]])
    f = o.ad_self_force(u, q[:1], box, coef, 1.0)
    fm = o.ad_self_force(-u, q[:1], box, coef, 1.0)
    np.testing.assert_allclose(fm, -f, rtol=1e-12, atol=0)


def test_correction_reduces_the_net_force_of_a_dilute_system():
    # with few, well separated charges the self-forces make up most of the
    # (non-zero) ad net force; in dense systems the pair terms' asymmetry
    # dominates it and the correction does not remove that part
    ratios = []
    for seed in range(6):
        rng = np.random.default_rng(seed)
        n, L, K = 8, 14.0, 16
        pos = rng.uniform(0, L, size=(n, 3))
        q = rng.normal(size=n)
        q -= q.mean()
        r = o.pppm(pos, q, (0, 0, 0), (L,) * 3, (K,) * 3, 5, 0.5, 1.0, "ad", self_force=True)
        ratios.append(np.linalg.norm(r["forces"].sum(0)) / np.linalg.norm(r["forces_uncorrected"].sum(0)))
    assert max(ratios) < 0.5 and np.mean(ratios) < 0.15


def test_forces_minus_self_force_is_the_pair_part():
    # the mesh is linear in the charges, so the self part of F_i is the
    # even part under flipping the sign of every other charge; with the
    # correction applied that part must be (nearly) gone
    rng = np.random.default_rng(3)
    n, L, K = 12, 12.0, 12
    pos = rng.uniform(0, L, size=(n, 3))
    q = rng.normal(size=n)
    box = o.Box((0, 0, 0), (L,) * 3, (K,) * 3, 5)
    G = o.influence_function(box, 0.6, "ad")
    sign = -np.ones(n)
    sign[0] = 1.0
    a = o.pppm(pos, q, (0, 0, 0), (L,) * 3, (K,) * 3, 5, 0.6, 1.0, "ad", G=G, self_force=True)
    b = o.pppm(pos, q * sign, (0, 0, 0), (L,) * 3, (K,) * 3, 5, 0.6, 1.0, "ad", G=G, self_force=True)
    even = 0.5 * (a["forces"][0] + b["forces"][0])
    even_raw = 0.5 * (a["forces_uncorrected"][0] + b["forces_uncorrected"][0])
    assert np.linalg.norm(even) < 0.01 * np.linalg.norm(even_raw)
