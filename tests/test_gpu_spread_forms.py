"""make_rho's two forms in the mixed precision, each against the oracle on the
same inputs: the owner-computes form (each tile pulls the charges whose
stencils reach it) and the push form (each tile sums its own charges' whole
stencils into a box extended by P - 1, then a fold adds the overlapping
boxes).  The plan takes the push form at P >= 6 by itself, and at P = 5
when there are fewer mesh tiles than CUs; PPPM_SPREAD forces either form at
plan creation.  Cases: the benchmark system at P = 5, 6 and 7,
ragged meshes with axes of one tile (the boxes wrap onto the start of the
axis), a dense cluster at P = 7 (64-bit box sums), and the mesh charge of
the FP64 output (the fold also writes the caller's FP64 mesh), and two
inputs that need the 64-bit sums although their tiles stay under the
visit count that selects them: 26 charges per mesh point, two charges per
mesh point on 64^3, and charges whose magnitudes span e^+-6."""
import os

import numpy as np
import pytest
import torch

import workloads as W
from gpu_cases import TOL, compare, gpu_run, io_round, make_plan, oracle_run, strict_energy_err

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1702_04250_amd as pkg  # noqa: E402


def plan_in_form(form, box_lo, box_len, mesh, P, g, diff, nmax, launch=None):
    old = os.environ.get("PPPM_SPREAD")
    os.environ["PPPM_SPREAD"] = form
    try:
        plan = make_plan(pkg, box_lo, box_len, mesh, P, g, 1.0, diff, "mixed", torch.float32, nmax)
    finally:
        if old is None:
            del os.environ["PPPM_SPREAD"]
        else:
            os.environ["PPPM_SPREAD"] = old
    if launch:
        plan.set_launch(0, *launch)
    return plan


def both_forms(pos, q, box_lo, box_len, mesh, P, g, diff, label, launch=None, strict_energy=False):
    pos_r, q_r = io_round(pos, q, torch.float32)
    ref = oracle_run(pos_r, q_r, box_lo, box_len, mesh, P, g, 1.0, diff)
    out = {}
    for form in ("visit", "push"):
        plan = plan_in_form(form, box_lo, box_len, mesh, P, g, diff, len(q), launch)
        print(f"case {label} {form} n={len(q)} mesh={mesh} P={P} {diff}", flush=True)
        gpu = gpu_run(plan, pos_r, q_r, torch.float32)
        plan.close()
        errs, bad = compare(gpu, ref, "mixed")
        print(f"  errors {errs}", flush=True)
        assert not bad, f"{label} {form}: {bad}"
        if strict_energy:
            assert strict_energy_err(gpu["energy"], ref) <= TOL["mixed"]["energy"]
        out[form] = gpu
    # the two forms round the same contributions with different units: they
    # agree to about the fixed-point resolution
    d = np.abs(out["push"]["rho"] - out["visit"]["rho"]).max() / np.abs(ref["rho"]).max()
    print(f"  push vs owner-computes mesh charge {d:.2e}", flush=True)
    assert d <= 2 * TOL["mixed"]["rho"]
    return out, ref


@pytest.mark.parametrize("P", [5, 6, 7])
def test_benchmark_system_in_both_forms(P):
    w = W.config(3, order=P)
    both_forms(w.pos, w.q, w.box_lo, w.box_len, w.mesh, P, w.g_ewald, "ad", f"uniform 524k P={P}",
               strict_energy=True)


@pytest.mark.parametrize("mesh,P,tile", [
    ((18, 20, 13), 5, None),        # rocFFT mesh, default tiles
    ((7, 9, 11), 7, None),          # every axis a single tile: boxes wrap
    ((40, 24, 30), 4, (16, 8, 12)),  # ragged last tiles (40 = 16+16+8, 30 = 12+12+6)
    ((32, 16, 20), 3, (32, 4, 8)),   # x a single tile, y thin tiles, z ragged
    ((16, 16, 16), 2, (8, 8, 8)),
])
@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_ragged_and_single_tile_meshes(mesh, P, tile, diff):
    lo, length = (-2.0, 1.0, 0.5), (13.0, 15.5, 11.0)
    pos, q = W.random_system(3000, length, seed=sum(mesh) + P, box_lo=lo)
    launch = (tile, 512) if tile else None
    both_forms(pos, q, lo, length, mesh, P, 0.5, diff, f"mesh {mesh} tile {tile}", launch=launch)


def test_dense_cluster_in_both_forms():
    # about 200 times the mean density: the cluster's tiles sum in 64 bits
    w = W.clustered("one_sign")
    out, ref = both_forms(w.pos, w.q, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, "ad", w.name,
                          strict_energy=True)
    sl = (slice(40, 57), slice(40, 57), slice(40, 57))
    for form, gpu in out.items():
        err = np.abs(gpu["rho"][sl] - ref["rho"][sl]).max() / np.abs(ref["rho"][sl]).max()
        print(f"  {form}: cluster mesh charge {err:.2e}", flush=True)
        assert err <= 1e-4


def expected_form(plan, mesh, P):
    # the plan's rule: the push form at P >= 6, and at P = 5 when there are
    # fewer tiles than CUs; the owner-computes form otherwise
    tile, _ = plan.get_launch(0)
    ntiles = int(np.prod([-(-k // b) for k, b in zip(mesh, tile)]))
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    if P >= 6:
        return "push"
    if P == 5:
        return "push" if ntiles < ncu else "visit"
    return "visit"


@pytest.mark.parametrize("idx,P", [(1, 7), (1, 6), (1, 5), (1, 4), (2, 5), (3, 5), (3, 6)])
def test_default_form_of_make_rho(idx, P):
    # no variable set: the plan's default form matches the plan forced to
    # that form bit for bit
    w = W.config(idx, order=P)
    pos_r, q_r = io_round(w.pos, w.q, torch.float32)
    assert "PPPM_SPREAD" not in os.environ
    default = make_plan(pkg, w.box_lo, w.box_len, w.mesh, P, w.g_ewald, 1.0, "ad", "mixed", torch.float32, w.n)
    form = expected_form(default, w.mesh, P)
    forced = plan_in_form(form, w.box_lo, w.box_len, w.mesh, P, w.g_ewald, "ad", w.n)
    other = plan_in_form("visit" if form == "push" else "push", w.box_lo, w.box_len, w.mesh, P, w.g_ewald, "ad", w.n)
    print(f"case default form config {idx} P={P}: {form}", flush=True)
    a = gpu_run(default, pos_r, q_r, torch.float32)
    b = gpu_run(forced, pos_r, q_r, torch.float32)
    c = gpu_run(other, pos_r, q_r, torch.float32)
    for p in (default, forced, other):
        p.close()
    assert np.array_equal(a["rho"], b["rho"]) and a["energy"] == b["energy"]
    same = np.array_equal(a["rho"], c["rho"])
    print(f"  other form bitwise the same: {same}", flush=True)
    if idx == 3:
        # on the benchmark system the forms' exponents and FP32 box sums
        # differ, so the bits tell them apart (on 1,000 charges they can
        # coincide)
        assert not same


@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_dense_mesh_in_both_forms(diff):
    # 20,000 Gaussian charges on 8 x 8 x 12 points (26 per point): the push
    # form's second tile holds fewer than 8,192 charges, and its reach bound
    # sends it to the 64-bit sums (with 32-bit sums its mesh charge was off
    # by 1.3e-4 of the maximum)
    rng = np.random.default_rng(97)
    lo, length = (-2.3, 8.2, 5.9), (5.78, 14.79, 11.6)
    pos = np.asarray(lo) + rng.uniform(-0.5, 1.5, size=(20000, 3)) * np.asarray(length)
    q = rng.normal(0, 1, size=20000)
    out, ref = both_forms(pos, q, lo, length, (8, 8, 12), 5, 0.487, diff, f"dense 8x8x12 {diff}")
    for form, gpu in out.items():
        err = np.abs(gpu["rho"] - ref["rho"]).max() / np.abs(ref["rho"]).max()
        print(f"  {form}: mesh charge {err:.2e}", flush=True)
        assert err <= 1e-5


def test_wide_charge_range_in_both_forms():
    # |q| spread over e^+-6 (max |q| about 14 times the RMS), 60,000 charges
    # mostly in one cluster on 16 x 12 x 16 points: the 32-bit unit follows
    # max |q|, so these take the 64-bit sums in every tile
    rng = np.random.default_rng(31)
    lo, length = (1.0, -3.0, 2.0), (12.0, 9.0, 12.0)
    pos = np.asarray(lo) + rng.uniform(0.0, 1.0, size=(60000, 3)) * np.asarray(length)
    pos[:48000] = np.asarray(lo) + 0.5 * np.asarray(length) + rng.normal(0, 1, size=(48000, 3)) * 0.05 * np.asarray(length)
    q = rng.normal(0, 1, size=60000) * np.exp(rng.uniform(-6, 6, size=60000))
    assert np.abs(q).max() > 8 * np.sqrt((q ** 2).mean())
    out, ref = both_forms(pos, q, lo, length, (16, 12, 16), 3, 0.28, "ad", "wide |q| 16x12x16", launch=((4, 4, 4), 1024))
    for form, gpu in out.items():
        err = np.abs(gpu["rho"] - ref["rho"]).max() / np.abs(ref["rho"]).max()
        print(f"  {form}: mesh charge {err:.2e}", flush=True)
        assert err <= 1e-5


def test_two_charges_per_point_in_both_forms():
    # 524,288 Gaussian charges on 64^3 points (two per point, eight times the
    # benchmark system's density): the reach bound exceeds the 32-bit switch,
    # so both forms sum in 64 bits (with 32-bit sums the visit form's mesh
    # charge was off by 2.0e-5 of the maximum)
    rng = np.random.default_rng(5)
    lo, length = (0.0, 0.0, 0.0), (40.0, 40.0, 40.0)
    pos = rng.uniform(0, 40, size=(524288, 3))
    q = rng.normal(0, 1, size=524288)
    out, ref = both_forms(pos, q, lo, length, (64, 64, 64), 5, 0.5, "ad", "two per point 64^3")
    for form, gpu in out.items():
        err = np.abs(gpu["rho"] - ref["rho"]).max() / np.abs(ref["rho"]).max()
        print(f"  {form}: mesh charge {err:.2e}", flush=True)
        assert err <= 2e-6
