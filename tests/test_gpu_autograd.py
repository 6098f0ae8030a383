"""GPU energy backward (the adjoint gather behind torch.autograd) on the
65,536-charge Gaussian system (mesh 64^3, P = 5): against the oracle's
analytic gradients and against central finite differences of the FP64
energy on 64 sampled particles (h = 1e-4 A for positions, 1e-4 e for
charges).

Tolerances (RMS relative): analytic vs oracle 1e-10 (FP64) / 1e-3 (mixed);
vs finite differences of the FP64 energy 1e-6 (FP64) / 1e-3 (mixed)."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_cases import io_round, make_plan, rms_rel
from oracle import oracle

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1702_04250_amd as pkg  # noqa: E402

DEV = torch.device("cuda:0")
TOL_ORACLE = {"fp64": 1e-10, "mixed": 1e-3}
TOL_FD = {"fp64": 1e-6, "mixed": 1e-3}
H_POS, H_Q = 1e-4, 1e-4


@pytest.fixture(scope="module")
def c4():
    w = W.config(4)
    rng = np.random.default_rng(w.seed)
    sample = rng.choice(w.n, 64, replace=False)
    return w, sample


@pytest.fixture(scope="module")
def fd_reference(c4):
    """Central differences of the FP64 GPU energy at the sampled particles."""
    w, sample = c4
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ad", "fp64", torch.float64, w.n)
    pos0 = torch.tensor(w.pos, dtype=torch.float64, device=DEV)
    q0 = torch.tensor(w.q, dtype=torch.float64, device=DEV)

    def energy(pos, q):
        return float(plan.compute(pos, q, want_forces=False)["energy"])

    print(f"case C4 finite differences: {len(sample)} particles, h={H_POS}", flush=True)
    gpos = np.zeros((len(sample), 3))
    gq = np.zeros(len(sample))
    for k, i in enumerate(sample):
        for d in range(3):
            p = pos0.clone()
            p[i, d] += H_POS
            ep = energy(p, q0)
            p[i, d] -= 2 * H_POS
            em = energy(p, q0)
            gpos[k, d] = (ep - em) / (2 * H_POS)
        qq = q0.clone()
        qq[i] += H_Q
        ep = energy(pos0, qq)
        qq[i] -= 2 * H_Q
        em = energy(pos0, qq)
        gq[k] = (ep - em) / (2 * H_Q)
    plan.close()
    return gpos, gq


def gpu_gradients(w, prec, io, diff="ad", scale=1.0):
    """E and its gradients through torch.autograd (PPPMEnergy)."""
    pos_r, q_r = io_round(w.pos, w.q, io)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, prec, io, w.n)
    pos = torch.tensor(pos_r, dtype=io, device=DEV, requires_grad=True)
    q = torch.tensor(q_r, dtype=io, device=DEV, requires_grad=True)
    e = pkg.pppm_energy(pos, q, plan)
    (scale * e).backward()
    torch.cuda.synchronize()
    plan.sync()
    out = (float(e), pos.grad.cpu().numpy().astype(np.float64), q.grad.cpu().numpy().astype(np.float64),
           pos_r, q_r)
    plan.close()
    return out


@pytest.mark.parametrize("prec,io", [("fp64", torch.float64), ("mixed", torch.float32)])
@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_backward_matches_oracle_gradients(c4, prec, io, diff):
    w, _ = c4
    print(f"case C4 backward {diff} {prec} io={io}", flush=True)
    e, gp, gq, pos_r, q_r = gpu_gradients(w, prec, io, diff)
    ref = oracle.energy_gradients(pos_r, q_r, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff)
    ep, eq = rms_rel(gp, ref["grad_pos"]), rms_rel(gq, ref["grad_q"])
    print(f"  grad_pos {ep:.3e} grad_q {eq:.3e} energy {abs(e - ref['energy']) / abs(ref['energy']):.3e}",
          flush=True)
    assert ep <= TOL_ORACLE[prec] and eq <= TOL_ORACLE[prec]


@pytest.mark.parametrize("prec,io", [("fp64", torch.float64), ("mixed", torch.float32)])
def test_backward_matches_finite_differences(c4, fd_reference, prec, io):
    w, sample = c4
    fd_pos, fd_q = fd_reference
    print(f"case C4 backward vs finite differences {prec} io={io}", flush=True)
    _, gp, gq, _, _ = gpu_gradients(w, prec, io)
    ep, eq = rms_rel(gp[sample], fd_pos), rms_rel(gq[sample], fd_q)
    print(f"  grad_pos {ep:.3e} grad_q {eq:.3e}", flush=True)
    assert ep <= TOL_FD[prec] and eq <= TOL_FD[prec]


def test_backward_scales_with_upstream_gradient(c4):
    w, _ = c4
    _, gp1, gq1, _, _ = gpu_gradients(w, "fp64", torch.float64)
    _, gp3, gq3, _, _ = gpu_gradients(w, "fp64", torch.float64, scale=-3.0)
    # two plans bin the charges in different orders, so the FP64 sums round
    # differently: compare in norm, not element by element
    assert rms_rel(gp3, -3.0 * gp1) < 1e-12
    assert rms_rel(gq3, -3.0 * gq1) < 1e-12


def test_position_gradient_is_minus_ad_force(c4):
    # dE/dr = -F(ad): the backward and the forward gather agree on one plan
    w, _ = c4
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ad", "fp64", torch.float64, w.n)
    pos = torch.tensor(w.pos, dtype=torch.float64, device=DEV)
    q = torch.tensor(w.q, dtype=torch.float64, device=DEV)
    out = plan.compute(pos, q)
    gp, _ = plan.energy_backward(torch.ones((), dtype=torch.float64, device=DEV), pos, q, True, False)
    plan.sync()
    f = out["forces"].cpu().numpy()
    assert rms_rel(gp.cpu().numpy(), -f) < 1e-12
    plan.close()


def test_stale_forward_is_rejected(c4):
    w, _ = c4
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ad", "fp64", torch.float64, w.n)
    pos = torch.tensor(w.pos, dtype=torch.float64, device=DEV, requires_grad=True)
    q = torch.tensor(w.q, dtype=torch.float64, device=DEV, requires_grad=True)
    e1 = pkg.pppm_energy(pos, q, plan)
    plan.compute(pos.detach(), q.detach())  # another forward on the same plan
    with pytest.raises(RuntimeError):
        e1.backward()
    plan.sync()
    plan.close()


@pytest.mark.parametrize("mesh", [(48, 40, 36), (32, 64, 16)])
def test_ik_backward_on_meshes_of_the_library_transforms(mesh):
    # the ik adjoint needs the potential, which ik plans compute on demand
    # (a potential-only z pass and the inverse passes); mixed-radix and
    # power-of-two meshes, mixed precision, against the oracle's adjoint
    lo = (0.0, 0.0, 0.0)
    length = (mesh[0] * 1.05, mesh[1] * 0.95, mesh[2] * 1.1)
    pos, q = W.random_system(600, length, seed=mesh[0] + mesh[2])
    q = q - q.mean()
    print(f"case ik backward mesh={mesh}", flush=True)
    plan = make_plan(pkg, lo, length, mesh, 5, 0.5, 1.0, "ik", "mixed", torch.float32, len(q))
    pos_r, q_r = io_round(pos, q, torch.float32)
    tp = torch.tensor(pos_r, dtype=torch.float32, device=DEV, requires_grad=True)
    tq = torch.tensor(q_r, dtype=torch.float32, device=DEV, requires_grad=True)
    e = pkg.pppm_energy(tp, tq, plan)
    e.backward()
    torch.cuda.synchronize()
    plan.sync()
    gp = tp.grad.cpu().numpy().astype(np.float64)
    gq = tq.grad.cpu().numpy().astype(np.float64)
    plan.close()
    ref = oracle.energy_gradients(pos_r, q_r, lo, length, mesh, 5, 0.5, 1.0, "ik")
    ep, eq = rms_rel(gp, ref["grad_pos"]), rms_rel(gq, ref["grad_q"])
    print(f"  grad_pos {ep:.3e} grad_q {eq:.3e}", flush=True)
    assert ep <= TOL_ORACLE["mixed"] and eq <= TOL_ORACLE["mixed"]


@pytest.mark.parametrize("prec,io", [("fp64", torch.float64), ("mixed", torch.float32)])
def test_ik_backward_on_a_rocfft_mesh(prec, io):
    # the ik adjoint on a mesh the library's transforms do not take: the
    # potential comes from the extra G multiply and one rocFFT real inverse
    mesh = (18, 20, 13)
    lo = (-1.0, 0.5, 2.0)
    length = (19.0, 21.0, 14.5)
    pos, q = W.random_system(800, length, seed=17, box_lo=lo)
    print(f"case ik backward rocFFT mesh={mesh} {prec}", flush=True)
    plan = make_plan(pkg, lo, length, mesh, 5, 0.45, 1.0, "ik", prec, io, len(q))
    pos_r, q_r = io_round(pos, q, io)
    tp = torch.tensor(pos_r, dtype=io, device=DEV, requires_grad=True)
    tq = torch.tensor(q_r, dtype=io, device=DEV, requires_grad=True)
    e = pkg.pppm_energy(tp, tq, plan)
    e.backward()
    torch.cuda.synchronize()
    plan.sync()
    gp = tp.grad.cpu().numpy().astype(np.float64)
    gq = tq.grad.cpu().numpy().astype(np.float64)
    plan.close()
    ref = oracle.energy_gradients(pos_r, q_r, lo, length, mesh, 5, 0.45, 1.0, "ik")
    ep, eq = rms_rel(gp, ref["grad_pos"]), rms_rel(gq, ref["grad_q"])
    print(f"  grad_pos {ep:.3e} grad_q {eq:.3e}", flush=True)
    assert ep <= TOL_ORACLE[prec] and eq <= TOL_ORACLE[prec]


def test_backward_ignores_positions_changed_after_the_forward(c4):
    # the C ABI backward reads the charges binned by the forward call, not
    # pos and q again: values written there in place afterwards do not move
    # the gradient, which stays that of the forward's energy
    w, _ = c4
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ad", "fp64", torch.float64, w.n)
    pos = torch.tensor(w.pos, dtype=torch.float64, device=DEV)
    q = torch.tensor(w.q, dtype=torch.float64, device=DEV)
    ge = torch.ones((), dtype=torch.float64, device=DEV)
    plan.compute(pos, q, want_forces=False)
    gp0, gq0 = plan.energy_backward(ge, pos, q)
    gp0, gq0 = gp0.clone(), gq0.clone()
    plan.compute(pos, q, want_forces=False)
    pos.add_(0.37)
    q.mul_(-2.0)
    gp1, gq1 = plan.energy_backward(ge, pos, q)
    plan.sync()
    assert torch.equal(gp0, gp1) and torch.equal(gq0, gq1)
    plan.close()


def test_autograd_refuses_positions_changed_in_place(c4):
    # through PPPMEnergy the saved inputs carry torch's version counter: an
    # in-place change between forward and backward is an error
    w, _ = c4
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, "ad", "fp64", torch.float64, w.n)
    leaf = torch.tensor(w.pos, dtype=torch.float64, device=DEV, requires_grad=True)
    pos = leaf * 1.0
    q = torch.tensor(w.q, dtype=torch.float64, device=DEV)
    e = pkg.pppm_energy(pos, q, plan)
    with torch.no_grad():
        pos.add_(0.1)
    with pytest.raises(RuntimeError):
        e.backward()
    plan.sync()
    plan.close()
