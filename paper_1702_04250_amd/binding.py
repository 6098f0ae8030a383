"""ctypes binding of libpppm_mi355x.so (the C ABI declared in include/pppm.h).

Argument marshalling only: every step of the PPPM path runs in the library's
HIP kernels (and, for meshes that are not powers of two, rocFFT).  PyTorch supplies device memory and the stream.
There is no CPU fallback: if the library is not built, or no GPU is present,
creating a plan raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from pathlib import Path

import torch

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "lib" / "libpppm_mi355x.so"
HEADER = PKG.parent / "include" / "pppm.h"

PPPM_OK = 0
STATUS = {
    0: "PPPM_OK", -1: "PPPM_ERR_ARG", -2: "PPPM_ERR_ORDER", -3: "PPPM_ERR_MESH", -4: "PPPM_ERR_DTYPE",
    -5: "PPPM_ERR_NONFINITE", -6: "PPPM_ERR_OOM", -7: "PPPM_ERR_HIP", -8: "PPPM_ERR_FFT", -9: "PPPM_ERR_STATE",
}
DIFF = {"ik": 0, "ad": 1}
PREC = {"fp64": 0, "mixed": 1}
IO_DTYPE = {torch.float32: 0, torch.float64: 1}
FLAG_CHECK_FINITE = 1
FLAG_WEIGHT_TABLE = 2
FLAG_AD_SELF_FORCE = 4


class PPPMError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


class Params(ctypes.Structure):
    _fields_ = [
        ("box_lo", ctypes.c_double * 3),
        ("box_len", ctypes.c_double * 3),
        ("mesh", ctypes.c_int32 * 3),
        ("order", ctypes.c_int32),
        ("g_ewald", ctypes.c_double),
        ("coulomb_c", ctypes.c_double),
        ("diff", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("io_dtype", ctypes.c_int),
        ("max_particles", ctypes.c_int64),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def declared_functions() -> list[str]:
    """Names of the functions include/pppm.h declares."""
    text = HEADER.read_text()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(pppm_[a-z_0-9]+)\s*\(", text, re.M)))


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python -m paper_1702_04250_amd.build")
    lib = ctypes.CDLL(str(LIB_PATH))
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    P = ctypes.POINTER
    sig = {
        "pppm_validate": [P(Params)],
        "pppm_plan_create": [P(Params), vp, P(vp)],
        "pppm_plan_destroy": [vp],
        "pppm_particle_map": [vp, i64, vp, vp],
        "pppm_make_rho": [vp, vp],
        "pppm_poisson": [vp, vp],
        "pppm_fieldforce": [vp, vp],
        "pppm_compute": [vp, i64, vp, vp, vp, vp, vp],
        "pppm_compute_noalloc": [P(Params), vp, i64, vp, vp, vp, vp, vp],
        "pppm_energy_backward": [vp, vp, i64, vp, vp, vp, vp],
        "pppm_energy_terms": [vp, vp],
        "pppm_sync": [vp],
        "pppm_plan_set_launch": [vp, i32, P(i32), i32],
        "pppm_plan_get_launch": [vp, i32, P(i32), P(i32)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.pppm_status_string.argtypes = [ctypes.c_int]
    lib.pppm_status_string.restype = ctypes.c_char_p
    lib.pppm_last_error.argtypes = [vp]
    lib.pppm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def make_params(box_lo, box_len, mesh, order, g_ewald, coulomb_c=1.0, diff="ad", prec="mixed",
                io_dtype=torch.float32, max_particles=0, check_finite=False, weight_table=0,
                self_force=False) -> Params:
    """weight_table: 0 = polynomial stencil weights; T > 0 = a table of T + 1
    entries per weight (PPPM_FLAG_WEIGHT_TABLE with PPPM_WEIGHT_TABLE_SIZE(T)).
    self_force: subtract the ad self-force (PPPM_FLAG_AD_SELF_FORCE)."""
    p = Params()
    p.box_lo[:] = [float(v) for v in box_lo]
    p.box_len[:] = [float(v) for v in box_len]
    p.mesh[:] = [int(v) for v in mesh]
    p.order = int(order)
    p.g_ewald = float(g_ewald)
    p.coulomb_c = float(coulomb_c)
    p.diff = DIFF[diff] if isinstance(diff, str) else int(diff)
    p.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    p.io_dtype = IO_DTYPE[io_dtype] if isinstance(io_dtype, torch.dtype) else int(io_dtype)
    p.max_particles = int(max_particles)
    p.flags = FLAG_CHECK_FINITE if check_finite else 0
    if weight_table:
        p.flags |= FLAG_WEIGHT_TABLE | ((int(weight_table) & 0xFFFF) << 8)
    if self_force:
        p.flags |= FLAG_AD_SELF_FORCE
    return p


def validate(params: Params) -> int:
    """pppm_validate: pure host check; returns the status code."""
    return load().pppm_validate(ctypes.byref(params))


def compute_noalloc(params: Params, pos, q, want_rho=False, want_energy=True, want_forces=True, stream=None,
                    out=None):
    """pppm_compute_noalloc: steps 1-4 without a plan, every device buffer in
    the library's static scratch array (see include/pppm.h).  pos, q and the
    outputs are caller tensors on the current device; out may hold
    preallocated outputs (rho, energy, forces), so that the call itself
    allocates nothing.  Returns dict(rho, energy, forces)."""
    lib = load()
    n = pos.shape[0]
    dev = pos.device
    kz = int(params.mesh[2]); ky = int(params.mesh[1]); kx = int(params.mesh[0])
    out = dict(out or {})
    if want_rho and out.get("rho") is None:
        out["rho"] = torch.empty((kz, ky, kx), dtype=torch.float64, device=dev)
    if want_energy and out.get("energy") is None:
        out["energy"] = torch.empty((), dtype=torch.float64, device=dev)
    if want_forces and out.get("forces") is None:
        out["forces"] = torch.empty((n, 3), dtype=pos.dtype, device=dev)
    rho = out.get("rho") if want_rho else None
    energy = out.get("energy") if want_energy else None
    forces = out.get("forces") if want_forces else None
    st = torch.cuda.current_stream(dev) if stream is None else stream
    status = lib.pppm_compute_noalloc(ctypes.byref(params), ctypes.c_void_p(st.cuda_stream), n, _ptr(pos), _ptr(q),
                                      _ptr(rho), _ptr(energy), _ptr(forces))
    if status != PPPM_OK:
        raise PPPMError(status, last_error(None))
    return {"rho": rho, "energy": energy, "forces": forces}


def last_error(handle=None) -> str:
    return (load().pppm_last_error(handle) or b"").decode()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """A PPPM plan on one device and stream (see include/pppm.h)."""

    def __init__(self, box_lo, box_len, mesh, order, g_ewald, coulomb_c=1.0, diff="ad", prec="mixed",
                 io_dtype=torch.float32, max_particles=1, check_finite=False, device=None, stream=None,
                 weight_table=0, self_force=False):
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the PPPM library runs only on an MI355X")
        self.device = torch.device(device if device is not None else "cuda", )
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.io_dtype = io_dtype
        self.diff = diff
        self.prec = prec
        self.mesh = tuple(int(k) for k in mesh)
        self.max_particles = int(max_particles)
        self.params = make_params(box_lo, box_len, mesh, order, g_ewald, coulomb_c, diff, prec, io_dtype,
                                  max_particles, check_finite, weight_table, self_force)
        self.generation = 0
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.pppm_plan_create(ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(handle))
        if st != PPPM_OK:
            raise PPPMError(st, last_error(None))
        self._h = handle
        self._lib = lib

    # -- helpers -------------------------------------------------------------
    def _check(self, st):
        if st != PPPM_OK:
            raise PPPMError(st, last_error(self._h))

    def _particles(self, pos, q):
        if pos.device != self.device or q.device != self.device:
            raise ValueError("pos and q must be on the plan's device")
        if pos.dtype != self.io_dtype or q.dtype != self.io_dtype:
            raise TypeError(f"pos and q must be {self.io_dtype}")
        if pos.dim() != 2 or pos.shape[1] != 3 or q.dim() != 1 or q.shape[0] != pos.shape[0]:
            raise ValueError("pos must be (N, 3) and q (N,)")
        if not (pos.is_contiguous() and q.is_contiguous()):
            raise ValueError("pos and q must be contiguous")
        return pos.shape[0]

    def _empty(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=self.device)

    # -- the C ABI, one call each ------------------------------------------
    def particle_map(self, pos, q):
        n = self._particles(pos, q)
        self.generation += 1
        self._check(self._lib.pppm_particle_map(self._h, n, _ptr(pos), _ptr(q)))

    def make_rho(self, rho=None):
        if rho is not None:
            assert rho.dtype == torch.float64 and rho.numel() == self.mesh[0] * self.mesh[1] * self.mesh[2]
        self._check(self._lib.pppm_make_rho(self._h, _ptr(rho)))
        return rho

    def poisson(self, energy=None):
        self._check(self._lib.pppm_poisson(self._h, _ptr(energy)))
        return energy

    def fieldforce(self, forces):
        self._check(self._lib.pppm_fieldforce(self._h, _ptr(forces)))
        return forces

    def compute(self, pos, q, want_rho=False, want_energy=True, want_forces=True, out=None):
        """Steps 1-4; returns dict(rho=(Kz,Ky,Kx) f64 | None, energy=() f64 | None, forces=(N,3) | None)."""
        n = self._particles(pos, q)
        out = out or {}
        kx, ky, kz = self.mesh
        rho = out.get("rho") if want_rho else None
        if want_rho and rho is None:
            rho = self._empty((kz, ky, kx), torch.float64)
        energy = out.get("energy") if want_energy else None
        if want_energy and energy is None:
            energy = self._empty((), torch.float64)
        forces = out.get("forces") if want_forces else None
        if want_forces and forces is None:
            forces = self._empty((n, 3), self.io_dtype)
        self.generation += 1
        self._check(self._lib.pppm_compute(self._h, n, _ptr(pos), _ptr(q), _ptr(rho), _ptr(energy), _ptr(forces)))
        return {"rho": rho, "energy": energy, "forces": forces}

    def energy_backward(self, grad_energy, pos, q, want_pos=True, want_q=True):
        n = self._particles(pos, q)
        assert grad_energy.dtype == torch.float64 and grad_energy.numel() == 1 and grad_energy.device == self.device
        gp = self._empty((n, 3), self.io_dtype) if want_pos else None
        gq = self._empty((n,), self.io_dtype) if want_q else None
        self._check(self._lib.pppm_energy_backward(self._h, _ptr(grad_energy), n, _ptr(pos), _ptr(q),
                                                   _ptr(gp), _ptr(gq)))
        return gp, gq

    def energy_terms(self):
        out = self._empty((3,), torch.float64)
        self._check(self._lib.pppm_energy_terms(self._h, _ptr(out)))
        return out

    def sync(self):
        self._check(self._lib.pppm_sync(self._h))

    def set_launch(self, which, tile, threads):
        arr = (ctypes.c_int32 * 3)(*[int(t) for t in tile])
        self._check(self._lib.pppm_plan_set_launch(self._h, int(which), arr, int(threads)))

    def get_launch(self, which):
        arr = (ctypes.c_int32 * 3)()
        thr = ctypes.c_int32()
        self._check(self._lib.pppm_plan_get_launch(self._h, int(which), arr, ctypes.byref(thr)))
        return tuple(arr), thr.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pppm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PPPMEnergy(torch.autograd.Function):
    """E(pos, q) = E_mesh + E_self + E_bg with a hand-written backward.

    forward runs particle map, make_rho and the Poisson step (no gather);
    backward calls pppm_energy_backward, which recomputes the stencil weights
    from pos and gathers the retained potential mesh.  The plan must not be
    used for another forward between this forward and its backward.
    """

    @staticmethod
    def forward(ctx, pos, q, plan):
        res = plan.compute(pos.detach(), q.detach(), want_energy=True, want_forces=False)
        ctx.save_for_backward(pos, q)
        ctx.plan = plan
        ctx.generation = plan.generation
        return res["energy"]

    @staticmethod
    def backward(ctx, grad_energy):
        pos, q = ctx.saved_tensors
        plan = ctx.plan
        if plan.generation != ctx.generation:
            raise RuntimeError("PPPMEnergy: the plan ran another forward before this backward")
        ge = grad_energy.detach().to(torch.float64).reshape(()).contiguous()
        gp, gq = plan.energy_backward(ge, pos.detach(), q.detach(), ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return gp, gq, None


def pppm_energy(pos, q, plan):
    return PPPMEnergy.apply(pos, q, plan)
