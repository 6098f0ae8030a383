"""GPU: the allocation-free one-shot call (pppm_compute_noalloc) through the
C ABI against pppm_compute on a regular plan, on the same inputs: two calls
in a row on one GPU, the second with a smaller system (the static scratch
keeps the first call's contents), in the mixed and FP64 forms, ad and ik,
at P = 5 and 7 (the two forms of make_rho);
and the refusals (a request larger than the scratch, a rocFFT mesh)."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_cases import TOL, io_round, make_plan

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1702_04250_amd as pkg  # noqa: E402

DEV = torch.device("cuda:0")


def plan_result(w, diff, prec, io, pos, q):
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, prec, io, w.n)
    out = plan.compute(pos, q, want_rho=True)
    plan.sync()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    plan.close()
    return res


@pytest.mark.parametrize("order", [5, 7])
@pytest.mark.parametrize("diff", ["ad", "ik"])
@pytest.mark.parametrize("prec,io", [("mixed", torch.float32), ("fp64", torch.float64)])
def test_noalloc_matches_plan_twice(diff, prec, io, order):
    # 32,001 charges of water, 64^3; at P = 7 the mixed form's make_rho takes
    # the push form, whose boxes are carved from the scratch too
    w = W.config(2, order=order)
    pos_r, q_r = io_round(w.pos, w.q, io)
    params = pkg.make_params(w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, prec, io, max_particles=w.n)
    for n in (w.n, 9000):
        print(f"case noalloc {diff} {prec} n={n}", flush=True)
        pos = torch.tensor(pos_r[:n], dtype=io, device=DEV).contiguous()
        q = torch.tensor(q_r[:n], dtype=io, device=DEV).contiguous()
        ref = plan_result(w, diff, prec, io, pos, q)
        out = pkg.compute_noalloc(params, pos, q, want_rho=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        # the same kernels on the same tiling: the mesh charge is an exact
        # fixed-point sum, every force a per-charge sum and the energy a
        # fixed-order reduction, so the results agree bit for bit
        rho_err = np.abs(got["rho"] - ref["rho"]).max() / np.abs(ref["rho"]).max()
        f_err = np.sqrt(((got["forces"].astype(np.float64) - ref["forces"]) ** 2).sum() / (ref["forces"] ** 2).sum())
        e_err = abs(float(got["energy"]) - float(ref["energy"])) / abs(float(ref["energy"]))
        print(f"  rho {rho_err:.2e} forces {f_err:.2e} energy {e_err:.2e}", flush=True)
        assert rho_err <= TOL[prec]["rho"] and f_err <= TOL[prec]["forces"] and e_err <= TOL[prec]["energy"]
        assert np.array_equal(got["rho"], ref["rho"])
        assert np.array_equal(got["forces"], ref["forces"])
        assert float(got["energy"]) == float(ref["energy"])


def test_noalloc_refusals():
    w = W.config(2)
    pos = torch.zeros((4, 3), dtype=torch.float32, device=DEV)
    q = torch.zeros((4,), dtype=torch.float32, device=DEV)
    # more particles than the scratch can hold
    big = pkg.make_params(w.box_lo, w.box_len, w.mesh, 5, 0.3, 1.0, "ad", "mixed", torch.float32,
                          max_particles=2 ** 31 - 1)
    with pytest.raises(pkg.PPPMError) as ei:
        pkg.compute_noalloc(big, pos, q)
    assert ei.value.status == -1 and "scratch" in str(ei.value)
    # a mesh that only rocFFT takes
    ragged = pkg.make_params((0, 0, 0), (10, 11, 12), (18, 20, 13), 5, 0.45, 1.0, "ad", "mixed", torch.float32,
                             max_particles=4)
    with pytest.raises(pkg.PPPMError) as ei:
        pkg.compute_noalloc(ragged, pos, q)
    assert ei.value.status == -3
    # the checked mode needs a plan
    checked = pkg.make_params(w.box_lo, w.box_len, w.mesh, 5, 0.3, 1.0, "ad", "mixed", torch.float32,
                              max_particles=4, check_finite=True)
    with pytest.raises(pkg.PPPMError) as ei:
        pkg.compute_noalloc(checked, pos, q)
    assert ei.value.status == -1
    torch.cuda.synchronize()
