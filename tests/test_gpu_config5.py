"""GPU parity at the largest workload: 4,194,304 charges of SPC/E-like water
(1,398,101 molecules and one zero charge) in a 340 A cube, mesh 256^3,
P = 7, ik and ad, mixed and FP64 forms, with the plan's default launch
geometry.  The FP64 oracle runs once per differentiation mode (about half a
minute each on one host core) and is shared by both precisions."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_cases import TOL, compare, gpu_run, io_round, make_plan, oracle_run, strict_energy_err

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1702_04250_amd as pkg  # noqa: E402

_ORACLE = {}


@pytest.fixture(scope="module")
def c5():
    return W.config(5)


def oracle_for(w, diff, io):
    # the FP32 inputs of the mixed form round positions; the oracle sees the
    # same rounded values, so each (mode, input dtype) pair has its own result
    key = (diff, io)
    if key not in _ORACLE:
        pos_r, q_r = io_round(w.pos, w.q, io)
        print(f"  oracle {w.name} {diff} io={io}", flush=True)
        _ORACLE[key] = (pos_r, q_r, oracle_run(pos_r, q_r, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald,
                                               1.0, diff))
    return _ORACLE[key]


@pytest.mark.parametrize("prec,io", [("mixed", torch.float32), ("fp64", torch.float64)])
@pytest.mark.parametrize("diff", ["ad", "ik"])
def test_config5_full_size(c5, diff, prec, io):
    w = c5
    print(f"case {w.name} n={w.n} mesh={w.mesh} P={w.order} {diff} {prec} io={io}", flush=True)
    pos_r, q_r, ref = oracle_for(w, diff, io)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, prec, io, w.n)
    gpu = gpu_run(plan, pos_r, q_r, io)
    plan.close()
    errs, bad = compare(gpu, ref, prec)
    print(f"  errors {errs}", flush=True)
    assert not bad, bad
    assert strict_energy_err(gpu["energy"], ref) <= TOL[prec]["energy"]
    # the zero charge gets exactly zero force
    assert np.all(gpu["forces"][q_r == 0.0] == 0.0)
