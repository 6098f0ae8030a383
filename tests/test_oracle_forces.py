"""Pins of the oracle's Distribute-Force steps and energy (Section 2.1, Section 3.1, Section 4.1).

* ik conserves momentum exactly (the paper checks that the sum of forces stays
  nearly zero, Section 4.1); here the identity is exact, so roundoff.
* ad forces are exactly minus the gradient of the mesh energy: central
  finite differences of the FP64 energy.
* Both modes converge to the exact Ewald reciprocal-space forces and energy
  (the paper's accuracy yardstick, Section 4.1) as the mesh is refined and as
  the order rises; ik and ad agree within the same discretisation error.
* Euler identity: sum_i q_i phi(r_i) = 2 E_mesh ties the gather to the spread.
Non-cubic boxes and meshes catch any axis mix-up.
"""
import numpy as np
import pytest

from oracle import oracle as o
from workloads import config, random_system

LO = (0.5, -1.0, 2.0)
LEN = (11.0, 9.0, 13.0)
MESH = (12, 10, 16)


@pytest.mark.parametrize("P", [2, 3, 5, 7])
def test_ik_net_force_is_zero(P):
    pos, q = random_system(200, LEN, seed=100 + P, box_lo=LO)
    r = o.pppm(pos, q, LO, LEN, MESH, P, 0.4, 1.3, "ik")
    f = r["forces"]
    assert np.linalg.norm(f.sum(axis=0)) < 1e-12 * np.abs(f).sum()


@pytest.mark.parametrize("P", [2, 4, 5, 7])
def test_ad_forces_are_minus_energy_gradient(P):
    pos, q = random_system(6, LEN, seed=200 + P, box_lo=LO)
    r = o.pppm(pos, q, LO, LEN, MESH, P, 0.45, 1.0, "ad")
    G = r["G"]
    eps = 1e-4
    fd = np.zeros_like(pos)
    for i in range(pos.shape[0]):
        for d in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, d] += eps
            p2[i, d] -= eps
            e1 = o.pppm(p1, q, LO, LEN, MESH, P, 0.45, 1.0, "ad", G=G)["e_mesh"]
            e2 = o.pppm(p2, q, LO, LEN, MESH, P, 0.45, 1.0, "ad", G=G)["e_mesh"]
            fd[i, d] = -(e1 - e2) / (2 * eps)
    err = np.linalg.norm(fd - r["forces"]) / np.linalg.norm(r["forces"])
    assert err < 1e-6


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_euler_identity(diff):
    pos, q = random_system(150, LEN, seed=7, box_lo=LO)
    r = o.pppm(pos, q, LO, LEN, MESH, 5, 0.4, 2.0, diff, want_phi=True)
    assert abs(float(q @ r["pot"]) - 2.0 * r["e_mesh"]) < 1e-12 * abs(r["e_mesh"])


@pytest.fixture(scope="module")
def c1_ewald():
    w = config(1)
    e_k, f_k = o.ewald_reciprocal(w.pos, w.q, w.box_len, w.g_ewald)
    return w, e_k, f_k


def _rms_rel(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_converges_to_ewald_as_mesh_refines(c1_ewald, diff):
    w, e_k, f_k = c1_ewald
    errs_f, errs_e = [], []
    for K in (16, 32, 64):
        r = o.pppm(w.pos, w.q, w.box_lo, w.box_len, (K,) * 3, 5, w.g_ewald, 1.0, diff)
        errs_f.append(_rms_rel(r["forces"], f_k))
        errs_e.append(abs(r["e_mesh"] - e_k) / abs(e_k))
    assert errs_f[0] < 1e-3 and errs_e[0] < 1e-5
    for a, b in zip(errs_f, errs_f[1:]):
        assert a / b > 10.0
    for a, b in zip(errs_e, errs_e[1:]):
        assert a / b > 10.0


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_converges_to_ewald_as_order_rises(c1_ewald, diff):
    w, e_k, f_k = c1_ewald
    errs = []
    for P in (3, 5, 7):
        r = o.pppm(w.pos, w.q, w.box_lo, w.box_len, (24,) * 3, P, w.g_ewald, 1.0, diff)
        errs.append(_rms_rel(r["forces"], f_k))
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 20.0


def test_ik_and_ad_agree_within_discretisation_error(c1_ewald):
    w, _, f_k = c1_ewald
    r_ik = o.pppm(w.pos, w.q, w.box_lo, w.box_len, (32,) * 3, 5, w.g_ewald, 1.0, "ik")
    r_ad = o.pppm(w.pos, w.q, w.box_lo, w.box_len, (32,) * 3, 5, w.g_ewald, 1.0, "ad")
    d = _rms_rel(r_ik["forces"], r_ad["forces"])
    bound = _rms_rel(r_ik["forces"], f_k) + _rms_rel(r_ad["forces"], f_k)
    assert d <= bound
    # the ad mesh force has a small non-zero net force (self-force), ik does not
    assert np.linalg.norm(r_ad["forces"].sum(0)) > 1e3 * np.linalg.norm(r_ik["forces"].sum(0))


@pytest.mark.parametrize("K", [12, 16])
def test_influence_function_is_optimal_for_its_mode(c1_ewald, K):
    # Each mode's influence function minimises that mode's RMS force error, so
    # with strong aliasing (P = 2) swapping in the other mode's G is worse.
    w, _, f_k = c1_ewald
    box = o.Box(w.box_lo, w.box_len, (K,) * 3, 2)
    G = {d: o.influence_function(box, w.g_ewald, d) for d in ("ik", "ad")}
    err = {}
    for mode in ("ik", "ad"):
        for g_of in ("ik", "ad"):
            r = o.pppm(w.pos, w.q, w.box_lo, w.box_len, (K,) * 3, 2, w.g_ewald, 1.0, mode, G=G[g_of])
            err[mode, g_of] = _rms_rel(r["forces"], f_k)
    assert err["ik", "ik"] < 0.8 * err["ik", "ad"]
    assert err["ad", "ad"] < err["ad", "ik"]


def test_shift_work_reference_setting_is_converged():
    # The order/mesh trade study (Section 2.3, Section 4) measures the force
    # error of each (P, K) against the FP64 path at P = 7 on a mesh of
    # spacing 0.59 A with g = 0.30, Ewald sums over half a million charges
    # being out of reach.  On a 592-charge system of the same density,
    # spacing and split, that setting is within 1e-6 of the exact Ewald
    # reciprocal forces in both differentiation modes (three orders of
    # magnitude below the study's tightest target), while a coarse setting
    # of the same system is measurably worse.
    L, K = 17.7, 30
    pos, q = random_system(592, (L,) * 3, seed=21, charge="pm1")
    _, f_ewald = o.ewald_reciprocal(pos, q, (L,) * 3, 0.3)
    den = (f_ewald ** 2).sum()
    for diff in ("ad", "ik"):
        ref = o.pppm(pos, q, (0, 0, 0), (L,) * 3, (K,) * 3, 7, 0.3, 1.0, diff)
        assert np.sqrt(((ref["forces"] - f_ewald) ** 2).sum() / den) < 1e-6
    coarse = o.pppm(pos, q, (0, 0, 0), (L,) * 3, (16,) * 3, 5, 0.3, 1.0, "ad")
    assert np.sqrt(((coarse["forces"] - f_ewald) ** 2).sum() / den) > 1e-5
