"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, element by element.  Tolerances: mesh charge max-relative
1e-6 (FP64) / 1e-4 (mixed), forces RMS-relative 1e-5 / 1e-3, energy relative
1e-6 / 1e-5."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_cases import TOL, compare, gpu_run, io_round, make_plan, oracle_run, rho_err, rms_rel, strict_energy_err
from oracle import oracle

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1702_04250_amd as pkg  # noqa: E402

PRECS = [("fp64", torch.float64), ("mixed", torch.float32), ("mixed", torch.float64), ("fp64", torch.float32)]


def run_and_check(pos, q, box_lo, box_len, mesh, P, g, C, diff, prec, io, launch=None, G=None, label="",
                  strict_energy=False):
    pos_r, q_r = io_round(pos, q, io)
    plan = make_plan(pkg, box_lo, box_len, mesh, P, g, C, diff, prec, io, len(q))
    if launch:
        for which, (tile, thr) in launch.items():
            plan.set_launch(which, tile, thr)
    print(f"case {label} n={len(q)} mesh={mesh} P={P} {diff} {prec} io={io}", flush=True)
    gpu = gpu_run(plan, pos_r, q_r, io)
    ref = oracle_run(pos_r, q_r, box_lo, box_len, mesh, P, g, C, diff, G=G)
    errs, bad = compare(gpu, ref, prec)
    print(f"  errors {errs}", flush=True)
    assert not bad, f"{label}: {bad}"
    if strict_energy:
        # one of the path's own configurations: |dE| / |E| within the energy
        # tolerance outright
        assert strict_energy_err(gpu["energy"], ref) <= TOL[prec]["energy"]
    # energy terms
    terms = gpu["terms"]
    t = TOL[prec]["energy"]
    assert abs(terms[0] - ref["e_mesh"]) <= t * abs(ref["e_mesh"]) + 1e-12
    assert abs(terms[1] - ref["e_self"]) <= 1e-12 * max(abs(ref["e_self"]), 1) or prec == "mixed"
    plan.close()
    return gpu, ref


@pytest.mark.parametrize("prec,io", PRECS)
@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_config1(diff, prec, io):
    w = W.config(1)
    run_and_check(w.pos, w.q, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, prec, io, label="C1", strict_energy=True)


@pytest.mark.parametrize("prec,io", [("fp64", torch.float64), ("mixed", torch.float32)])
@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_config2_water(diff, prec, io):
    w = W.config(2)
    run_and_check(w.pos, w.q, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, prec, io, label="C2", strict_energy=True)


@pytest.mark.parametrize("P", [3, 4, 5, 6, 7])
def test_config3_order_sweep_ad_mixed(P):
    w = W.config(3, order=P)
    run_and_check(w.pos, w.q, w.box_lo, w.box_len, w.mesh, P, w.g_ewald, 1.0, "ad", "mixed", torch.float32,
                  label=f"C3 P={P}", strict_energy=True)


@pytest.mark.parametrize("diff,prec,io", [("ik", "mixed", torch.float32), ("ad", "fp64", torch.float64),
                                          ("ik", "fp64", torch.float64)])
def test_config3_p5_other_forms(diff, prec, io):
    w = W.config(3)
    run_and_check(w.pos, w.q, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, diff, prec, io, label="C3 P=5", strict_energy=True)


# ---- edge cases --------------------------------------------------------------

EDGE_BOX = ((-3.0, 2.0, 0.5), (11.0, 13.0, 7.5))


@pytest.mark.parametrize("mesh", [(8, 16, 32), (32, 8, 16), (16, 64, 8), (128, 16, 8), (32, 32, 16), (256, 32, 8),
                                  (48, 40, 36), (20, 28, 72), (112, 12, 18), (36, 56, 24), (160, 10, 14),
                                  (32, 32, 12), (64, 32, 20)])
@pytest.mark.parametrize("diff", ["ad", "ik"])
@pytest.mark.parametrize("prec,io", [("mixed", torch.float32), ("fp64", torch.float64)])
def test_meshes_with_own_transforms(mesh, diff, prec, io):
    # meshes whose sizes are powers of two, or in the mixed form 2^a m with m
    # in {3, 5, 7, 9}, take the library's own transforms (other sizes take
    # rocFFT): anisotropic shapes, smallest axes, radix 3, 5, 7 and 9 stages,
    # planes with and without the fused x-y passes, fused passes split over
    # two blocks per plane with the plane count a multiple of 8 and not
    lo = (-3.0, 1.0, 2.0)
    length = (mesh[0] * 0.9, mesh[1] * 1.1, mesh[2] * 1.0)
    pos, q = W.random_system(700, length, seed=mesh[0] * 7 + mesh[1], box_lo=lo)
    run_and_check(pos, q, lo, length, mesh, 5, 0.5, 1.3, diff, prec, io, label="pow2")


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("mesh", [(18, 20, 13), (7, 9, 11), (32, 8, 24)])
@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_ragged_meshes_and_orders(P, mesh, diff):
    if min(mesh) < P:
        pytest.skip("mesh smaller than the order")
    lo, length = EDGE_BOX
    pos, q = W.random_system(257, length, seed=P * 100 + mesh[0], box_lo=lo)
    run_and_check(pos, q, lo, length, mesh, P, 0.45, 1.7, diff, "fp64", torch.float64, label="ragged")


@pytest.mark.parametrize("P", [3, 5, 7])
@pytest.mark.parametrize("mesh", [(18, 20, 13), (7, 9, 11), (11, 16, 10)])
@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_ragged_meshes_mixed(P, mesh, diff):
    # sizes the library's transforms do not take (an axis under 8, or not of
    # the form 2^a m with m in {1, 3, 5, 7, 9}) run on rocFFT; in the mixed
    # form that is an FP32 real transform pair around the FP32 G multiply
    if min(mesh) < P:
        pytest.skip("mesh smaller than the order")
    lo, length = EDGE_BOX
    pos, q = W.random_system(900, length, seed=P * 31 + mesh[2], box_lo=lo)
    run_and_check(pos, q, lo, length, mesh, P, 0.45, 1.7, diff, "mixed", torch.float32, label="ragged mixed")


@pytest.mark.parametrize("kind", ["pm1", "one_sign"])
@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_dense_cluster(kind, diff):
    # 200,000 charges in a 16-cell cube (about 200 times the mean density)
    # at P = 7: the tiles over the cluster read tens of thousands of charges,
    # which the mixed form sums in 64-bit fixed point
    w = W.clustered(kind)
    gpu, ref = run_and_check(w.pos, w.q, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, "mixed",
                             torch.float32, label=w.name, strict_energy=True)
    # the mesh charge inside the cluster, where it is largest, point by point
    kz, ky, kx = ref["rho"].shape
    sl = (slice(40, 57), slice(40, 57), slice(40, 57))
    err = np.abs(gpu["rho"][sl] - ref["rho"][sl]).max() / np.abs(ref["rho"][sl]).max()
    print(f"  cluster mesh charge {err:.2e}", flush=True)
    assert err <= 1e-4


def test_tile_switches_between_map_forms():
    # one plan through the device-atomic and the histogram forms of the
    # particle map and back again: each form must start from counters the
    # other leaves behind (the histogram form leaves its bin totals)
    w = W.config(3, order=5)
    pos_r, q_r = io_round(w.pos, w.q, torch.float32)
    ref = oracle_run(pos_r, q_r, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ad")
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ad", "mixed", torch.float32, w.n)
    default_tile, default_threads = plan.get_launch(0)
    for tile, threads in (((4, 4, 4), 256), (default_tile, default_threads), ((8, 4, 4), 256),
                          (default_tile, default_threads)):
        plan.set_launch(0, tile, threads)
        print(f"case tile switch {tile}", flush=True)
        gpu = gpu_run(plan, pos_r, q_r, torch.float32)
        errs, bad = compare(gpu, ref, "mixed")
        print(f"  errors {errs}", flush=True)
        assert not bad, f"tile {tile}: {bad}"
    plan.close()


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_minimum_mesh_equal_to_order(diff):
    lo, length = EDGE_BOX
    pos, q = W.random_system(50, length, seed=3, box_lo=lo)
    run_and_check(pos, q, lo, length, (5, 5, 5), 5, 0.6, 1.0, diff, "fp64", torch.float64, label="K=P")
    run_and_check(pos, q, lo, length, (2, 3, 2), 2, 0.6, 1.0, diff, "fp64", torch.float64, label="K=2")


@pytest.mark.parametrize("prec,io", [("fp64", torch.float64), ("mixed", torch.float32)])
def test_positions_outside_box_and_on_faces(prec, io):
    lo, length = EDGE_BOX
    pos, q = W.random_system(400, length, seed=11, box_lo=lo)
    L = np.asarray(length)
    pos[:50] += 3 * L          # far images
    pos[50:100] -= 2 * L
    pos[100:110] = np.asarray(lo)            # lower corner
    pos[110:120] = np.asarray(lo) + L        # upper faces == lower faces
    pos[120:130, 0] = lo[0] + L[0] * (1 - 1e-16)
    q[130:140] = 0.0                          # zero charges
    run_and_check(pos, q, lo, length, (16, 16, 12), 5, 0.45, 1.0, "ad", prec, io, label="faces")


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_single_particle_and_empty(diff):
    lo, length = EDGE_BOX
    dev = torch.device("cuda:0")
    pos = np.array([[0.3, 4.1, 2.2]])
    q = np.array([1.5])
    plan = make_plan(pkg, lo, length, (12, 12, 12), 5, 0.5, 1.0, diff, "fp64", torch.float64, 1)
    gpu = gpu_run(plan, pos, q, torch.float64)
    ref = oracle_run(pos, q, lo, length, (12, 12, 12), 5, 0.5, 1.0, diff)
    assert rho_err(gpu["rho"], ref["rho"]) < 1e-12
    assert abs(gpu["energy"] - ref["energy"]) < 1e-12 * abs(ref["energy"])
    if diff == "ik":
        # one charge: momentum conservation makes its ik mesh force vanish
        assert np.abs(gpu["forces"]).max() < 1e-12 and np.abs(ref["forces"]).max() < 1e-12
    else:
        # the ad mesh self-force of a lone charge is small but not zero
        assert np.abs(ref["forces"]).max() > 1e-8
        assert rms_rel(gpu["forces"], ref["forces"]) < 1e-9
    plan.close()
    # empty system: zero mesh, zero energy; plan with max_particles 0 and n = 0
    plan = make_plan(pkg, lo, length, (12, 12, 12), 5, 0.5, 1.0, diff, "fp64", torch.float64, 0)
    out = plan.compute(torch.zeros((0, 3), dtype=torch.float64, device=dev),
                       torch.zeros((0,), dtype=torch.float64, device=dev), want_rho=True)
    plan.sync()
    assert float(out["rho"].abs().max()) == 0.0
    assert float(out["energy"]) == 0.0
    assert out["forces"].shape == (0, 3)
    plan.close()


def test_charged_system_background_term():
    lo, length = EDGE_BOX
    pos, q = W.random_system(300, length, seed=5, charge="positive", box_lo=lo)
    gpu, ref = run_and_check(pos, q, lo, length, (16, 16, 12), 5, 0.45, 2.0, "ad", "fp64", torch.float64,
                             label="charged")
    assert abs(gpu["terms"][2] - ref["e_bg"]) < 1e-10 * abs(ref["e_bg"])


GEOMETRIES = [
    (0, (8, 8, 8), 128), (0, (16, 8, 4), 64), (0, (32, 16, 8), 512), (0, (4, 4, 4), 256), (0, (64, 16, 8), 1024),
    (1, (8, 8, 8), 128), (1, (16, 16, 4), 512), (1, (4, 8, 16), 64), (1, (32, 8, 8), 256),
]
# the ik gather stages three field meshes of the shared tile: 64 x 16 x 8 needs
# more LDS than a workgroup has (test_launch_geometry_beyond_the_lds_is_refused)
REFUSED = {("ik", 0, (64, 16, 8))}


@pytest.mark.parametrize("diff,which,tile,threads",
                         [(d, *g) for d in ("ik", "ad") for g in GEOMETRIES if (d, g[0], g[1]) not in REFUSED])
def test_launch_geometries_agree(diff, which, tile, threads):
    w = W.config(2)
    run_and_check(w.pos, w.q, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, "mixed", torch.float32,
                  launch={which: (tile, threads)}, label=f"launch {which} {tile} {threads}")


def test_launch_geometry_beyond_the_lds_is_refused():
    # refused on the host (PPPM_ERR_ARG), never launched; the plan keeps its
    # geometry and still computes to parity
    w = W.config(2)
    pos_r, q_r = io_round(w.pos, w.q, torch.float32)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ik", "mixed", torch.float32, w.n)
    before = plan.get_launch(0)
    for diff, which, tile in sorted(REFUSED):
        with pytest.raises(pkg.PPPMError) as ei:
            plan.set_launch(which, tile, 1024)
        assert ei.value.status == -1
        assert "LDS" in str(ei.value)
    assert plan.get_launch(0) == before
    print("case refused geometry, then compute", flush=True)
    gpu = gpu_run(plan, pos_r, q_r, torch.float32)
    ref = oracle_run(pos_r, q_r, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ik")
    errs, bad = compare(gpu, ref, "mixed")
    assert not bad, bad
    plan.close()


def test_nonfinite_input_flag():
    lo, length = EDGE_BOX
    pos, q = W.random_system(100, length, seed=9, box_lo=lo)
    pos[7, 1] = np.nan
    pos[8, 0] = np.inf
    q[9] = np.nan
    dev = torch.device("cuda:0")
    plan = make_plan(pkg, lo, length, (12, 12, 12), 5, 0.5, 1.0, "ad", "fp64", torch.float64, 100,
                     check_finite=True)
    out = plan.compute(torch.tensor(pos, device=dev), torch.tensor(q, device=dev))
    with pytest.raises(pkg.PPPMError) as ei:
        plan.sync()
    assert ei.value.status == -5
    plan.sync()  # flag cleared
    # finite inputs afterwards: no flag
    pos[7, 1] = pos[8, 0] = 0.0
    q[9] = 0.0
    plan.compute(torch.tensor(pos, device=dev), torch.tensor(q, device=dev))
    plan.sync()
    plan.close()


def test_state_errors():
    lo, length = EDGE_BOX
    dev = torch.device("cuda:0")
    plan = make_plan(pkg, lo, length, (12, 12, 12), 5, 0.5, 1.0, "ad", "fp64", torch.float64, 10)
    with pytest.raises(pkg.PPPMError) as ei:
        plan.make_rho()
    assert ei.value.status == -9
    pos = torch.zeros((11, 3), dtype=torch.float64, device=dev)
    q = torch.zeros((11,), dtype=torch.float64, device=dev)
    with pytest.raises(pkg.PPPMError) as ei:
        plan.compute(pos, q)
    assert ei.value.status == -1  # n > max_particles
    pos, q = pos[:10].contiguous(), q[:10].contiguous()
    plan.compute(pos, q)
    ge = torch.ones((), dtype=torch.float64, device=dev)
    other = pos.clone()
    with pytest.raises(pkg.PPPMError) as ei:
        plan.energy_backward(ge, other, q)
    assert ei.value.status == -9
    plan.sync()
    plan.close()


def test_repeated_calls_are_stable():
    # the binning counters are reset by each call: same result every time
    w = W.config(2)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ad", "fp64", torch.float64, w.n)
    dev = torch.device("cuda:0")
    pos, q = torch.tensor(w.pos, device=dev), torch.tensor(w.q, device=dev)
    first = plan.compute(pos, q, want_rho=True)
    f0, r0, e0 = first["forces"].clone(), first["rho"].clone(), float(first["energy"])
    for _ in range(3):
        out = plan.compute(pos, q, want_rho=True)
        plan.sync()
        assert rms_rel(out["forces"].cpu().numpy(), f0.cpu().numpy()) < 1e-13
        assert rho_err(out["rho"].cpu().numpy(), r0.cpu().numpy()) < 1e-13
        assert abs(float(out["energy"]) - e0) < 1e-12 * abs(e0)
    # a smaller system on the same plan
    out = plan.compute(pos[:1000].contiguous(), q[:1000].contiguous(), want_rho=True)
    plan.sync()
    ref = oracle_run(w.pos[:1000], w.q[:1000], w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ad")
    assert rms_rel(out["forces"].cpu().numpy(), ref["forces"]) < 1e-5
    plan.close()


def test_separate_steps_match_compute():
    w = W.config(2)
    dev = torch.device("cuda:0")
    pos = torch.tensor(w.pos, dtype=torch.float32, device=dev)
    q = torch.tensor(w.q, dtype=torch.float32, device=dev)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ik", "mixed", torch.float32, w.n)
    a = plan.compute(pos, q, want_rho=True)
    fa, ra, ea = a["forces"].clone(), a["rho"].clone(), a["energy"].clone()
    plan.particle_map(pos, q)
    rho = torch.empty_like(ra)
    plan.make_rho(rho)
    e = torch.empty((), dtype=torch.float64, device=dev)
    plan.poisson(e)
    f = torch.empty_like(fa)
    plan.fieldforce(f)
    plan.sync()
    assert rms_rel(f.cpu().numpy(), fa.cpu().numpy()) < 1e-6
    assert rho_err(rho.cpu().numpy(), ra.cpu().numpy()) < 1e-6
    assert abs(float(e) - float(ea)) < 1e-9 * abs(float(ea))
    plan.close()


@pytest.mark.parametrize("tile", [(4, 4, 4), (8, 4, 4)])
def test_atomic_particle_map_form(tile):
    # tiles this fine give more bins than one block's LDS histogram holds, so
    # the particle map takes its device-atomic form
    w = W.config(3, order=5)
    run_and_check(w.pos, w.q, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ad", "mixed", torch.float32,
                  launch={0: (tile, 256), 1: (tile, 256)}, label=f"atomic map {tile}")


def test_gather_workgroup_limit():
    w = W.config(1)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ad", "mixed", torch.float32, w.n)
    for which in (1, 2):
        with pytest.raises(pkg.PPPMError) as ei:
            plan.set_launch(which, (8, 8, 8), 1024)
        assert ei.value.status == -1
    plan.set_launch(0, (8, 8, 8), 1024)  # make_rho takes up to 1024 threads
    assert plan.get_launch(0)[1] == 1024
    plan.close()


def test_mixed_ik_gather_width():
    # the mixed ik gather takes up to 1024 threads (768 by default where the
    # LDS allows), the same forces at every width
    w = W.config(1)
    pos_r, q_r = io_round(w.pos, w.q, torch.float32)
    ref = oracle_run(pos_r, q_r, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ik")
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ik", "mixed", torch.float32, w.n)
    tile, threads = plan.get_launch(1)
    assert threads == 768
    forces = {}
    for t in (768, 1024, 512):
        plan.set_launch(1, tile, t)
        print(f"case mixed ik gather {t} threads", flush=True)
        gpu = gpu_run(plan, pos_r, q_r, torch.float32)
        errs, bad = compare(gpu, ref, "mixed")
        assert not bad, bad
        forces[t] = gpu["forces"]
    assert np.array_equal(forces[768], forces[1024]) and np.array_equal(forces[768], forces[512])
    with pytest.raises(pkg.PPPMError) as ei:
        plan.set_launch(1, tile, 1088)
    assert ei.value.status == -1
    plan.close()
    # a tile whose three staged meshes leave no room for 1024 threads' lane
    # buffers (P = 7, 32 x 16 x 9: 150 KB of meshes): that width is refused
    # and the plan keeps its geometry; 512 threads take the tile
    lo, length, mesh = (0.0, 0.0, 0.0), (30.0, 30.0, 17.0), (64, 64, 36)
    pos, q = W.random_system(2000, length, seed=4, box_lo=lo)
    plan = make_plan(pkg, lo, length, mesh, 7, 0.45, 1.0, "ik", "mixed", torch.float32, 2000)
    before = (plan.get_launch(0), plan.get_launch(1))
    with pytest.raises(pkg.PPPMError) as ei:
        plan.set_launch(1, (32, 16, 9), 1024)
    assert ei.value.status == -1 and "LDS" in str(ei.value)
    assert (plan.get_launch(0), plan.get_launch(1)) == before
    # 768 threads on a smaller tile (96 KB of meshes), then make_rho moves
    # the shared tile to 32 x 16 x 9: the gather narrows to a width that fits
    plan.set_launch(1, (32, 8, 9), 768)
    plan.set_launch(0, (32, 16, 9), 1024)
    assert plan.get_launch(1)[0] == (32, 16, 9) and 512 <= plan.get_launch(1)[1] < 768
    pos_r, q_r = io_round(pos, q, torch.float32)
    print("case mixed ik gather after tile changes", flush=True)
    gpu = gpu_run(plan, pos_r, q_r, torch.float32)
    errs, bad = compare(gpu, oracle_run(pos_r, q_r, lo, length, mesh, 7, 0.45, 1.0, "ik"), "mixed")
    assert not bad, bad
    plan.close()


def test_tile_finer_than_bin_arrays_is_refused():
    w = W.config(3, order=2)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, 2, w.g_ewald, 1.0, "ad", "mixed", torch.float32, 16)
    with pytest.raises(pkg.PPPMError) as ei:
        plan.set_launch(0, (1, 1, 1), 256)
    assert ei.value.status == -1
    # the plan keeps its previous geometry and still works
    pos = torch.rand((16, 3), dtype=torch.float32, device="cuda:0") * 170.0
    q = torch.ones(16, dtype=torch.float32, device="cuda:0")
    plan.compute(pos, q)
    plan.sync()
    plan.close()


@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_interfacial_slab(diff):
    # half the tiles empty, the rest at twice the average load
    w = W.interfacial()
    run_and_check(w.pos, w.q, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, "mixed", torch.float32,
                  label="interfacial", strict_energy=True)


@pytest.mark.parametrize("prec,io", [("mixed", torch.float32), ("fp64", torch.float64)])
def test_mesh_charge_independent_of_particle_order(prec, io):
    # make_rho sums in exact fixed point: any order of the charges (and of the
    # LDS atomics) gives the same bits
    w = W.config(2)
    dev = torch.device("cuda:0")
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, 5, w.g_ewald, 1.0, "ad", prec, io, w.n)
    pos = torch.tensor(w.pos, dtype=io, device=dev)
    q = torch.tensor(w.q, dtype=io, device=dev)
    perm = torch.tensor(np.random.default_rng(11).permutation(w.n), device=dev)
    r1 = plan.compute(pos, q, want_rho=True)["rho"].clone()
    r2 = plan.compute(pos[perm].contiguous(), q[perm].contiguous(), want_rho=True)["rho"]
    plan.sync()
    assert torch.equal(r1, r2)
    plan.close()


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("T", [500, 5000])
@pytest.mark.parametrize("prec,io", [("mixed", torch.float32), ("fp64", torch.float64)])
@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_weight_table_variant(T, prec, io, diff, order):
    # the tabulated stencil weights against the oracle's tabulated variant
    # (at P = 7 the mixed form's make_rho takes its push form)
    w = W.config(2, order=order)
    pos_r, q_r = io_round(w.pos, w.q, io)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, prec, io, w.n,
                     weight_table=T)
    print(f"case weight table T={T} {diff} {prec} io={io} P={order}", flush=True)
    gpu = gpu_run(plan, pos_r, q_r, io)
    plan.close()
    ref = oracle.pppm(pos_r, q_r, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, table=T)
    errs, bad = compare(gpu, ref, prec)
    print(f"  errors {errs}", flush=True)
    assert not bad, bad


@pytest.mark.parametrize("order", [4, 5, 6, 7])
@pytest.mark.parametrize("prec,io", [("mixed", torch.float32), ("fp64", torch.float64)])
def test_ad_self_force_correction(prec, io, order):
    # corrected ad forces against the oracle's corrected forces, and the
    # correction itself (corrected minus uncorrected plan) against the
    # oracle's self-force; even and odd orders place the stencil fraction
    # differently relative to u (the sign of the first harmonic)
    w = W.config(2, order=order)
    pos_r, q_r = io_round(w.pos, w.q, io)
    print(f"case ad self-force {prec} io={io} P={order}", flush=True)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ad", prec, io, w.n,
                     self_force=True)
    gpu = gpu_run(plan, pos_r, q_r, io)
    plan.close()
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ad", prec, io, w.n)
    raw = gpu_run(plan, pos_r, q_r, io)
    plan.close()
    ref = oracle.pppm(pos_r, q_r, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ad", self_force=True)
    errs, bad = compare(gpu, ref, prec)
    corr = raw["forces"] - gpu["forces"]
    sf_err = rms_rel(corr, ref["self_force"])
    # in FP32 the correction is measured as the difference of two force
    # arrays, so it carries their rounding (about 1e-7 of the force); the
    # correction shrinks quickly with P (about 1e-5 of the force at P = 7)
    f_scale = float(np.sqrt((ref["forces"] ** 2).mean()))
    abs_err = float(np.sqrt(((corr - ref["self_force"]) ** 2).mean())) / f_scale
    print(f"  errors {errs} self-force {sf_err:.3e} ({abs_err:.2e} of the force)", flush=True)
    assert not bad, bad
    if prec == "fp64":
        assert sf_err < 1e-9
    else:
        assert sf_err < 5e-3 and abs_err < 3e-7


@pytest.mark.parametrize("P", [4, 5, 7])
def test_ad_self_force_of_a_lone_charge(P):
    # a lone charge's ad force is all self-force: the correction removes
    # almost all of it (what is left are the harmonics beyond the second);
    # even and odd orders place the stencil differently relative to the cell.
    # In the mixed form the correction (uncorrected minus corrected force)
    # is as large as the force itself, so it checks the FP32 sines directly.
    L, K = 16.0, 16
    rng = np.random.default_rng(11)
    pos = rng.uniform(0, L, size=(4, 3))
    q = np.array([1.0])
    for k in range(len(pos)):
        p1 = pos[k:k + 1]
        out = {}
        for prec, io in (("fp64", torch.float64), ("mixed", torch.float32)):
            for sf in (False, True):
                plan = make_plan(pkg, (0, 0, 0), (L,) * 3, (K,) * 3, P, 0.6, 1.0, "ad", prec, io, 1,
                                 self_force=sf)
                out[prec, sf] = gpu_run(plan, p1, q, io)["forces"].astype(np.float64)
                plan.close()
        ref = oracle.pppm(p1, q, (0, 0, 0), (L,) * 3, (K,) * 3, P, 0.6, 1.0, "ad", self_force=True)
        before, after = np.linalg.norm(out["fp64", False]), np.linalg.norm(out["fp64", True])
        err = rms_rel(out["fp64", True], ref["forces"])
        corr32 = out["mixed", False] - out["mixed", True]
        err32 = rms_rel(corr32, ref["self_force"])
        print(f"case lone charge P={P} #{k}: |F| {before:.3e} -> {after:.3e}, vs oracle {err:.2e}; "
              f"mixed correction vs oracle {err32:.2e}", flush=True)
        # the residual is a small difference of FP64 values: relative to it
        # the error is larger than relative to the uncorrected force
        assert err < 1e-8
        assert before > 0 and after < {4: 0.08, 5: 0.01, 7: 0.01}[P] * before
        assert err32 < 2e-5


@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_order_2_charges_just_below_grid_points(diff):
    # P = 2: the ad derivative weights jump at grid points.  Charges one
    # FP32 step below a grid point have a fraction within half a step of 1,
    # where the stored coordinate s + f would round up to s + 1; the map keeps
    # it below, so the gathers use the cell the map (and the oracle) chose
    # (rounded up, single forces were off by 7 % of the RMS force)
    rng = np.random.default_rng(12)
    lo, length, K = (0.25, -1.5, 2.0), (16.0, 16.0, 16.0), (16, 16, 16)
    h = np.asarray(length) / np.asarray(K)
    pos = np.asarray(lo) + rng.uniform(0, 1, size=(3000, 3)) * np.asarray(length)
    grid = np.asarray(lo) + rng.integers(1, 16, size=(600, 3)) * h
    below = np.nextafter(grid.astype(np.float32), np.float32(-np.inf)).astype(np.float64)
    pos = np.concatenate([pos, below])
    q = rng.choice([-1.0, 1.0], size=len(pos))
    print(f"case order 2 below grid points {diff}", flush=True)
    pos_r, q_r = io_round(pos, q, torch.float32)
    plan = make_plan(pkg, lo, length, K, 2, 0.6, 1.0, diff, "mixed", torch.float32, len(q))
    gpu = gpu_run(plan, pos_r, q_r, torch.float32)
    plan.close()
    ref = oracle.pppm(pos_r, q_r, lo, length, K, 2, 0.6, 1.0, diff)
    errs, bad = compare(gpu, ref, "mixed")
    print(f"  errors {errs}", flush=True)
    assert not bad, bad
    assert errs["forces_max"] < 1e-4
