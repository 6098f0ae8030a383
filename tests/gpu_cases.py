"""Shared helpers of the GPU parity tests: run one case through the C ABI and
through the FP64 oracle on the same inputs, and measure the differences."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle

# Tolerances (GPU vs FP64 oracle): mesh charge max-relative, forces RMS
# relative, energy relative (all as stated for the path); forces_max bounds
# every single particle's force error by the RMS tolerance taken against the
# typical force, max_i |dF_i| / sqrt(mean_i |F_i|^2), so that a defect
# confined to a few tiles' charges cannot hide in the RMS over all of them.
TOL = {
    "fp64": {"rho": 1e-6, "forces": 1e-5, "forces_max": 1e-5, "energy": 1e-6},
    "mixed": {"rho": 1e-4, "forces": 1e-3, "forces_max": 1e-3, "energy": 1e-5},
}


def rho_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rms_rel(a, b):
    den = float((b ** 2).sum())
    return float(np.sqrt(((a - b) ** 2).sum() / den)) if den > 0 else float(np.sqrt(((a - b) ** 2).sum()))


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def io_round(pos, q, io_dtype):
    """The inputs exactly as the GPU sees them, promoted back to FP64 for the oracle."""
    npdt = np.float32 if io_dtype == torch.float32 else np.float64
    return pos.astype(npdt).astype(np.float64), q.astype(npdt).astype(np.float64)


def make_plan(pkg, box_lo, box_len, mesh, order, g, C, diff, prec, io_dtype, nmax, **kw):
    return pkg.Plan(box_lo, box_len, mesh, order, g, C, diff, prec, io_dtype, max_particles=max(nmax, 1),
                    device=torch.device("cuda:0"), **kw)


def gpu_run(plan, pos, q, io_dtype, want_rho=True):
    dev = torch.device("cuda:0")
    tp = torch.tensor(pos, dtype=io_dtype, device=dev).reshape(-1, 3).contiguous()
    tq = torch.tensor(q, dtype=io_dtype, device=dev).reshape(-1).contiguous()
    out = plan.compute(tp, tq, want_rho=want_rho)
    terms = plan.energy_terms()
    plan.sync()
    return {
        "rho": out["rho"].cpu().numpy() if want_rho else None,
        "energy": float(out["energy"].cpu()),
        "forces": out["forces"].cpu().numpy().astype(np.float64),
        "terms": terms.cpu().numpy(),
    }


def oracle_run(pos, q, box_lo, box_len, mesh, order, g, C, diff, G=None):
    return oracle.pppm(pos, q, box_lo, box_len, mesh, order, g, C, diff, G=G)


def energy_err(gpu_e, ref, prec="fp64"):
    """|dE| over its allowed scale, E = E_mesh + E_self + E_bg (the Ewald
    split): |dE| / |E| in FP64.  In the mixed form each term is computed in
    FP32 arithmetic to about 1e-6 of its own magnitude, so on a system whose
    E cancels strongly (E_mesh and E_self nearly opposite) the error is
    measured against |E| + 0.1 (|E_mesh| + |E_self| + |E_bg|): the gate
    |dE| <= 1e-5 |E| + 1e-6 sum |terms|.  The path's own configurations are
    also held to |dE| / |E| <= 1e-5 outright (strict_energy_err)."""
    if prec == "fp64":
        return rel(gpu_e, ref["energy"])
    terms = abs(ref["e_mesh"]) + abs(ref["e_self"]) + abs(ref["e_bg"])
    return abs(gpu_e - ref["energy"]) / max(abs(ref["energy"]) + 0.1 * terms, 1e-300)


def strict_energy_err(gpu_e, ref):
    """|dE| / |E|."""
    return rel(gpu_e, ref["energy"])


def max_force_err(a, b):
    """Largest per-particle force error relative to the RMS force."""
    scale = float(np.sqrt((b ** 2).sum(axis=1).mean())) if len(b) else 0.0
    err = float(np.sqrt(((a - b) ** 2).sum(axis=1)).max()) if len(b) else 0.0
    return err / scale if scale > 0 else err


def compare(gpu, ref, prec, check_rho=True):
    tol = TOL[prec]
    errs = {"forces": rms_rel(gpu["forces"], ref["forces"]),
            "forces_max": max_force_err(gpu["forces"], ref["forces"]),
            "energy": energy_err(gpu["energy"], ref, prec)}
    if check_rho and gpu["rho"] is not None:
        errs["rho"] = rho_err(gpu["rho"], ref["rho"])
    bad = {k: v for k, v in errs.items() if not v <= tol[k]}
    return errs, bad
