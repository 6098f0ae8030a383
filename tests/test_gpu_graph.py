"""The forward step captured in a HIP graph (torch's graph capture on the
plan's stream).  The step's kernels are deterministic and the step records
no memset nodes, so every replay, with eager work of the program between
replays, reproduces the eager step bitwise; a replay after the positions
change in place matches an eager step on the new positions."""
import pytest
import torch

import workloads as W
from gpu_cases import make_plan

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1702_04250_amd as pkg  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("diff,prec,io,order", [("ad", "mixed", torch.float32, 5), ("ik", "mixed", torch.float32, 5),
                                                ("ad", "fp64", torch.float64, 5), ("ad", "mixed", torch.float32, 7)])
def test_graph_replays_match_eager(diff, prec, io, order):
    # at P = 7 the mixed form's make_rho is the push form (two kernels)
    w = W.config(2, order=order)
    print(f"case graph replay C2 {diff} {prec} P={order}", flush=True)
    stream = torch.cuda.Stream(device=DEV)
    plan = make_plan(pkg, w.box_lo, w.box_len, w.mesh, w.order, w.g_ewald, 1.0, diff, prec, io, w.n, stream=stream)
    pos = torch.tensor(w.pos, dtype=io, device=DEV).contiguous()
    q = torch.tensor(w.q, dtype=io, device=DEV).contiguous()
    forces = torch.empty((w.n, 3), dtype=io, device=DEV)
    energy = torch.empty((), dtype=torch.float64, device=DEV)

    def step():
        plan.particle_map(pos, q)
        plan.make_rho(None)
        plan.poisson(energy)
        plan.fieldforce(forces)

    with torch.cuda.stream(stream):
        step()
        torch.cuda.synchronize()
        f_eager, e_eager = forces.clone(), energy.clone()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            step()
        torch.cuda.synchronize()
        for _ in range(3):
            forces.zero_()
            energy.zero_()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(forces, f_eager) and torch.equal(energy, e_eager)
            step()  # eager work between replays
            torch.cuda.synchronize()
        # new positions, same buffers
        pos.add_(0.37)
        step()
        torch.cuda.synchronize()
        f_new, e_new = forces.clone(), energy.clone()
        assert not torch.equal(f_new, f_eager)
        forces.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(forces, f_new) and torch.equal(energy, e_new)
    plan.sync()
    plan.close()
