"""Plain FP64 CPU oracle for the PPPM particle-mesh path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this module; the product path never does.  It shares no
code with the GPU library (it builds and loads its own C file, ``oracle.c``).

PPPM (Section 2.1 of the paper) splits the Coulomb sum in the Ewald way into a
short-range real-space part and a smooth long-range part that is solved on a
periodic mesh in three steps: (1) charges are spread onto the grid with a
stencil, (2) Poisson's equation is solved by FFT, (3) the result is mapped
back to the atoms with the same stencil.  The gradient is taken in k-space
(ik: three inverse FFTs, three field grids gathered) or analytically from the
scalar potential (ad: one inverse FFT, derivative coefficients in the gather).

Steps (1) and (3) and the influence function are C loops in ``oracle.c``.
The FFTs of step (2), the energy terms and the adjoint are written here with
NumPy.  The
test-only Ewald sums give the exact result the mesh method approximates.

Readings where the paper is silent (the influence function, the Nyquist
derivative, the energy, the mesh-charge units, the ad self-force) are stated at
each function.  The optional ad self-force correction is pinned against the
exact force on a lone charge, which is all self-force.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None


def build(force: bool = True) -> Path:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, FP64, no fast-math).

    OpenMP only splits the setup-time influence-function loop over planes;
    every other loop runs on one thread.
    """
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-o", str(tmp), str(_SRC), "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        lib = ctypes.CDLL(str(_LIB))
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_weights.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        lib.oracle_particle_map.argtypes = [ctypes.c_int64, dp, dp, dp, ip, ctypes.c_int, lp, dp]
        lib.oracle_make_rho.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ip, ctypes.c_int, ctypes.c_int, dp]
        lib.oracle_fieldforce_ik.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ip, ctypes.c_int, ctypes.c_int,
                                             dp, dp, dp, dp]
        lib.oracle_fieldforce_ad.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ip, ctypes.c_int, ctypes.c_int,
                                             dp, dp, dp]
        lib.oracle_influence_function.argtypes = [dp, ip, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                                  ctypes.c_int, dp]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Box:
    """Orthorhombic periodic box with an FFT mesh and a stencil order.

    table = 0: stencil weights from their polynomials; T > 0: the tabulated
    variant of the mapping functions (Section 3.1), weights read from a table
    of their values at fractions i / T (nearest entry)."""

    def __init__(self, box_lo, box_len, mesh, order, table=0):
        self.lo = _f64(box_lo).reshape(3)
        self.len = _f64(box_len).reshape(3)
        self.mesh = np.ascontiguousarray(mesh, dtype=np.int32).reshape(3)
        self.order = int(order)
        if not 2 <= self.order <= 7:
            raise ValueError("order must be in [2, 7]")
        self.h = self.len / self.mesh
        self.volume = float(np.prod(self.len))
        self.table = int(table)

    @property
    def shape(self):
        """Mesh array shape, C order (Kz, Ky, Kx)."""
        kx, ky, kz = (int(k) for k in self.mesh)
        return (kz, ky, kx)


# ---------------------------------------------------------------------------
# Step 1 and the stencil (Section 3.1)
# ---------------------------------------------------------------------------

def weights(order: int, f: float):
    """Stencil coefficients of one axis at fraction f: (w[0..P-1], dw/du)."""
    lib = _load()
    w = np.zeros(order)
    dw = np.zeros(order)
    lib.oracle_weights(order, float(f), _dp(w), _dp(dw))
    return w, dw


def particle_map(pos, box: Box):
    """Stencil start s (unwrapped, int64) and fraction f for each particle and axis."""
    lib = _load()
    pos = _f64(pos).reshape(-1, 3)
    n = pos.shape[0]
    s = np.zeros((n, 3), dtype=np.int64)
    f = np.zeros((n, 3))
    lib.oracle_particle_map(n, _dp(pos), _dp(box.lo), _dp(box.len),
                            box.mesh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), box.order,
                            s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(f))
    return s, f


def make_rho(pos, q, box: Box):
    """Map-Charge: mesh charge per grid point, shape (Kz, Ky, Kx); sum equals sum(q)."""
    lib = _load()
    pos = _f64(pos).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    rho = np.zeros(box.shape)
    lib.oracle_make_rho(pos.shape[0], _dp(pos), _dp(q), _dp(box.lo), _dp(box.len),
                        box.mesh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), box.order, box.table, _dp(rho))
    return rho


def fieldforce_ik(pos, q, box: Box, ex, ey, ez):
    lib = _load()
    pos = _f64(pos).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    ex, ey, ez = _f64(ex), _f64(ey), _f64(ez)
    force = np.zeros((pos.shape[0], 3))
    lib.oracle_fieldforce_ik(pos.shape[0], _dp(pos), _dp(q), _dp(box.lo), _dp(box.len),
                             box.mesh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), box.order, box.table,
                             _dp(ex), _dp(ey), _dp(ez), _dp(force))
    return force


def fieldforce_ad(pos, q, box: Box, phi):
    """Returns (forces (N,3), potential at each particle (N,))."""
    lib = _load()
    pos = _f64(pos).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    phi = _f64(phi)
    force = np.zeros((pos.shape[0], 3))
    pot = np.zeros(pos.shape[0])
    lib.oracle_fieldforce_ad(pos.shape[0], _dp(pos), _dp(q), _dp(box.lo), _dp(box.len),
                             box.mesh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), box.order, box.table,
                             _dp(phi), _dp(force), _dp(pot))
    return force, pot


# ---------------------------------------------------------------------------
# Step 2: Poisson's equation in k-space (Equation 2; Section 2.1, Section 3.2)
# ---------------------------------------------------------------------------

ALIAS_RANGE = 2  # aliases m_d in [-2, 2] in the influence-function sums


def wave_numbers(box: Box):
    """Per-axis k = 2 pi n / L with n in FFT order, n in [-K/2, K/2)."""
    ks = []
    for d in range(3):
        K = int(box.mesh[d])
        n = np.fft.fftfreq(K, d=1.0 / K)  # integers in FFT order
        ks.append(2.0 * math.pi * n / box.len[d])
    return ks  # (kx, ky, kz) 1-D arrays


def influence_function(box: Box, g_ewald: float, diff: str):
    """Optimal influence function G(k), shape (Kz, Ky, Kx), FFT order.

    The paper leaves the Green function of the Poisson step unspecified
    (Section 3.2 only names the FFTs).  Reading: the influence function that
    minimises the RMS force error for the order-P B-spline assignment, with
    U(k) = prod_d sinc(k_d h_d / 2)^P, the Ewald-screened reference
    R(k) = 4 pi exp(-k^2 / 4g^2) / k^2 and aliases k_m = k + 2 pi m / h,
    |m_d| <= 2:
      ik: G = sum_m U^2(k_m) (k . k_m) R(k_m) / (|k|^2 [sum_m U^2(k_m)]^2)
      ad: G = sum_m U^2(k_m) |k_m|^2 R(k_m)
              / ([sum_m U^2(k_m)] [sum_m |k_m|^2 U^2(k_m)])
    G(0) = 0 (no net-charge mode).  Evaluated point by point in oracle.c.
    """
    if diff not in ("ik", "ad"):
        raise ValueError(diff)
    lib = _load()
    G = np.zeros(box.shape)
    lib.oracle_influence_function(_dp(box.len), box.mesh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  box.order, float(g_ewald), 0 if diff == "ik" else 1, ALIAS_RANGE, _dp(G))
    return G


def ad_self_force_coefficients(box: Box, G):
    """Leading harmonics of the ad self-force (Section 2.1's ad gradient of
    the mesh energy, applied to a charge's own mesh charge).

    A lone charge q at mesh coordinate u has, with the B-spline transform
    U(k) = prod_d sinc(k_d h_d / 2)^P and aliases k_a = k + 2 pi a / h,
      rho_hat(k) = q sum_a U(k_a) exp(-i 2 pi a.u) exp(-i k.u h),
    so E_mesh(u) = (C q^2 / 2V) sum_k G sum_{a,b} U(k_a) U(k_b) cos(2 pi (a-b).u).
    The terms a - b = +-e_d and +-2 e_d give
      E(u) = const + (C q^2 / V) sum_d [S1_d cos(2 pi u_d) + S2_d cos(4 pi u_d)] + ...,
      S1_d = sum_k G(k) prod_{d' != d} [sum_a U_d'(a)^2] sum_a U_d(a) U_d(a + 1),
      S2_d likewise with U_d(a) U_d(a + 2), aliases |a_d'| <= 2.
    Returns (S1[3], S2[3]); the mixed differences (a - b along two axes) and
    higher harmonics are left out.
    """
    ks = wave_numbers(box)
    P = box.order
    A = ALIAS_RANGE
    ua = []  # per axis: U_d(a, n) for a = -A..A
    for d in range(3):
        h = box.h[d]
        rows = []
        for a in range(-A, A + 1):
            x = 0.5 * (ks[d] + 2.0 * math.pi * a / h) * h
            s = np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))
            rows.append(s ** P)
        ua.append(np.array(rows))
    sq = [np.sum(u * u, axis=0) for u in ua]
    s1, s2 = np.zeros(3), np.zeros(3)
    for d in range(3):
        b1 = np.sum(ua[d][:-1] * ua[d][1:], axis=0)
        b2 = np.sum(ua[d][:-2] * ua[d][2:], axis=0)
        for b, out in ((b1, s1), (b2, s2)):
            f = [sq[0], sq[1], sq[2]]
            f[d] = b
            fz, fy, fx = np.meshgrid(f[2], f[1], f[0], indexing="ij")
            out[d] = float(np.sum(G * fz * fy * fx))
    return s1, s2


def ad_self_force(pos, q, box: Box, coef, coulomb_c: float):
    """The self-force of each charge from its own mesh charge, to the leading
    harmonics of ad_self_force_coefficients:
      F_d = (C q^2 / (V h_d)) [2 pi S1_d sin(2 pi u_d) + 4 pi S2_d sin(4 pi u_d)],
    u_d = (x_d - lo_d) / h_d."""
    pos = _f64(pos).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    s1, s2 = coef
    u = (pos - box.lo) / box.h
    pref = coulomb_c * (q * q)[:, None] / (box.volume * box.h[None, :])
    return pref * (2 * math.pi * s1 * np.sin(2 * math.pi * u) + 4 * math.pi * s2 * np.sin(4 * math.pi * u))


def derivative_wave_numbers(box: Box):
    """Per-axis derivative wavenumber for ik: k, except 0 at n = -K/2.

    The paper does not say how the ik gradient treats the Nyquist plane.
    Reading: zero there, which keeps the three field meshes real and the
    net force exactly zero.
    """
    out = []
    for d, k in enumerate(wave_numbers(box)):
        K = int(box.mesh[d])
        kd = k.copy()
        if K % 2 == 0:
            kd[K // 2] = 0.0
        out.append(kd)
    return out


def poisson(rho, box: Box, G, coulomb_c: float, diff: str, want_phi: bool = False):
    """Solve for the mesh potential / field from mesh charge rho (charge per point).

    rho_hat = FFT(rho) (unnormalised, exp(-i k.r)).  The mesh potential is
    phi_m = (C / (hx hy hz)) * IFFT(G rho_hat)_m, i.e. (C/V) sum_k G rho_hat
    exp(i k.r_m).  ik fields: E_d = (C / (hx hy hz)) IFFT(-i kappa_d G rho_hat).
    E_mesh = (C / 2V) sum_k G |rho_hat|^2 = 1/2 sum_m rho_m phi_m.
    Returns a dict with e_mesh and either phi (ad) or the fields (ik), plus
    phi as well when want_phi is set.
    """
    rho_hat = np.fft.fftn(rho)
    scale = coulomb_c / float(np.prod(box.h))
    out = {"e_mesh": 0.5 * coulomb_c / box.volume * float(np.sum(G * np.abs(rho_hat) ** 2))}
    if diff == "ad" or want_phi:
        out["phi"] = scale * np.fft.ifftn(G * rho_hat).real
    if diff == "ik":
        kxd, kyd, kzd = derivative_wave_numbers(box)
        KZ, KY, KX = np.meshgrid(kzd, kyd, kxd, indexing="ij")
        out["ex"] = scale * np.fft.ifftn(-1j * KX * G * rho_hat).real
        out["ey"] = scale * np.fft.ifftn(-1j * KY * G * rho_hat).real
        out["ez"] = scale * np.fft.ifftn(-1j * KZ * G * rho_hat).real
    return out


# ---------------------------------------------------------------------------
# Energy terms of the Ewald split (Section 2.1)
# ---------------------------------------------------------------------------

def self_energy(q, g_ewald, coulomb_c):
    """E_self = -C g / sqrt(pi) sum q_i^2 (each charge's own smooth part)."""
    q = _f64(q)
    return -coulomb_c * g_ewald / math.sqrt(math.pi) * float(np.sum(q * q))


def background_energy(q, g_ewald, coulomb_c, volume):
    """E_bg = -C pi Q^2 / (2 V g^2): uniform neutralising background for net charge Q."""
    Q = float(np.sum(_f64(q)))
    return -coulomb_c * math.pi * Q * Q / (2.0 * volume * g_ewald ** 2)


def pppm(pos, q, box_lo, box_len, mesh, order, g_ewald, coulomb_c=1.0, diff="ad",
         want_phi=False, G=None, table=0, self_force=False):
    """One full PPPM long-range evaluation in FP64.

    Returns dict: rho, G, e_mesh, e_self, e_bg, energy, forces, and phi/pot
    (ad, or when want_phi), ex/ey/ez (ik).  table: tabulated stencil weights
    (Box).  self_force (ad): forces minus each charge's self-force to its
    leading harmonics (ad_self_force), the uncorrected ones kept as
    forces_uncorrected; energy and potential are unchanged.
    """
    box = Box(box_lo, box_len, mesh, order, table)
    pos = _f64(pos).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    if G is None:
        G = influence_function(box, g_ewald, diff)
    rho = make_rho(pos, q, box)
    sol = poisson(rho, box, G, coulomb_c, diff, want_phi=want_phi)
    res = {"rho": rho, "G": G, "box": box, "e_mesh": sol["e_mesh"]}
    res["e_self"] = self_energy(q, g_ewald, coulomb_c)
    res["e_bg"] = background_energy(q, g_ewald, coulomb_c, box.volume)
    res["energy"] = res["e_mesh"] + res["e_self"] + res["e_bg"]
    if diff == "ik":
        res.update(ex=sol["ex"], ey=sol["ey"], ez=sol["ez"])
        res["forces"] = fieldforce_ik(pos, q, box, sol["ex"], sol["ey"], sol["ez"])
    if "phi" in sol:
        res["phi"] = sol["phi"]
        f_ad, pot = fieldforce_ad(pos, q, box, sol["phi"])
        res["pot"] = pot
        if diff == "ad":
            res["forces"] = f_ad
            if self_force:
                res["forces_uncorrected"] = f_ad
                res["self_force"] = ad_self_force(pos, q, box, ad_self_force_coefficients(box, G), coulomb_c)
                res["forces"] = f_ad - res["self_force"]
        else:
            res["forces_ad_phi"] = f_ad
    return res


def energy_gradients(pos, q, box_lo, box_len, mesh, order, g_ewald, coulomb_c=1.0, diff="ad", G=None, table=0):
    """Adjoint of E = E_mesh + E_self + E_bg with respect to positions and charges.

    E_mesh = 1/2 rho^T A rho with A symmetric, so
      dE/dq_i = phi(r_i) - 2 C g q_i / sqrt(pi) - C pi Q / (V g^2),
      dE/dr_i = q_i grad phi(r_i) = -F_i(ad gather of phi),
    where phi is the mesh potential of the same influence function that
    defines E (that of the plan's differentiation mode).
    """
    res = pppm(pos, q, box_lo, box_len, mesh, order, g_ewald, coulomb_c, diff, want_phi=True, G=G, table=table)
    box = res["box"]
    q = _f64(q).reshape(-1)
    f_ad, pot = fieldforce_ad(pos, q, box, res["phi"])
    Q = float(np.sum(q))
    dq = pot - 2.0 * coulomb_c * g_ewald * q / math.sqrt(math.pi) \
        - coulomb_c * math.pi * Q / (box.volume * g_ewald ** 2)
    return {"grad_pos": -f_ad, "grad_q": dq, "energy": res["energy"], "res": res}


# ---------------------------------------------------------------------------
# Test-only exact references: Ewald sums (the paper's accuracy yardstick,
# Section 4.1) and the real-space part of the split.
# ---------------------------------------------------------------------------

def ewald_reciprocal(pos, q, box_len, g_ewald, coulomb_c=1.0, tol=1e-16):
    """Exact Ewald k-space energy and forces (k != 0 terms).

    E_rec = (C / 2V) sum_k R(k) |S(k)|^2, S(k) = sum_j q_j exp(i k.r_j),
    F_i = (C / V) q_i sum_k R(k) k Im(exp(i k.r_i) S*(k)),
    with R(k) = 4 pi exp(-k^2/4g^2) / k^2 and all k with exp(-k^2/4g^2) > tol.
    """
    pos = _f64(pos).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    L = _f64(box_len).reshape(3)
    kmax = 2.0 * g_ewald * math.sqrt(-math.log(tol))
    nmax = [int(math.ceil(kmax * L[d] / (2 * math.pi))) for d in range(3)]
    rng = [np.arange(-nmax[d], nmax[d] + 1) for d in range(3)]
    NX, NY, NZ = np.meshgrid(*rng, indexing="ij")
    kv = np.stack([NX.ravel() * 2 * math.pi / L[0], NY.ravel() * 2 * math.pi / L[1],
                   NZ.ravel() * 2 * math.pi / L[2]], axis=1)
    k2 = np.sum(kv * kv, axis=1)
    keep = (k2 > 0) & (np.exp(-k2 / (4 * g_ewald ** 2)) > tol)
    kv, k2 = kv[keep], k2[keep]
    R = 4 * math.pi * np.exp(-k2 / (4 * g_ewald ** 2)) / k2
    V = float(np.prod(L))
    energy = 0.0
    forces = np.zeros_like(pos)
    chunk = 4096
    for a in range(0, kv.shape[0], chunk):
        kc, Rc = kv[a:a + chunk], R[a:a + chunk]
        phase = pos @ kc.T  # (N, nk)
        c, s = np.cos(phase), np.sin(phase)
        S_re = q @ c
        S_im = q @ s
        energy += 0.5 * coulomb_c / V * float(np.sum(Rc * (S_re ** 2 + S_im ** 2)))
        # Im(exp(i k.r_i) S*) = sin(k.r_i) S_re - cos(k.r_i) S_im
        im = s * S_re[None, :] - c * S_im[None, :]
        forces += (coulomb_c / V) * q[:, None] * ((im * Rc[None, :]) @ kc)
    return energy, forces


def ewald_real(pos, q, box_len, g_ewald, coulomb_c=1.0, tol=1e-16):
    """Real-space part (C/2) sum' q_i q_j erfc(g r)/r over images, and its forces."""
    from scipy.special import erfc

    pos = _f64(pos).reshape(-1, 3)
    q = _f64(q).reshape(-1)
    L = _f64(box_len).reshape(3)
    # erfc(g r_c) < tol
    rc = 1.0
    while erfc(g_ewald * rc) > tol:
        rc += 0.25
    nimg = [int(math.ceil(rc / L[d])) for d in range(3)]
    energy = 0.0
    forces = np.zeros_like(pos)
    n = pos.shape[0]
    for ix in range(-nimg[0], nimg[0] + 1):
        for iy in range(-nimg[1], nimg[1] + 1):
            for iz in range(-nimg[2], nimg[2] + 1):
                shift = np.array([ix * L[0], iy * L[1], iz * L[2]])
                d = pos[:, None, :] - pos[None, :, :] - shift[None, None, :]  # r_i - r_j - n
                r = np.sqrt(np.sum(d * d, axis=2))
                mask = (r > 0) & (r < rc)
                if ix == 0 and iy == 0 and iz == 0:
                    mask &= ~np.eye(n, dtype=bool)
                rr = np.where(mask, r, 1.0)
                qq = q[:, None] * q[None, :]
                e = np.where(mask, qq * erfc(g_ewald * rr) / rr, 0.0)
                energy += 0.5 * coulomb_c * float(np.sum(e))
                # -dV/dr * rhat, V = erfc(g r)/r
                dvdr = -(erfc(g_ewald * rr) / rr ** 2
                         + 2 * g_ewald / math.sqrt(math.pi) * np.exp(-(g_ewald * rr) ** 2) / rr)
                fmag = np.where(mask, -coulomb_c * qq * dvdr / rr, 0.0)
                forces += np.sum(fmag[:, :, None] * d, axis=1)
    return energy, forces


def ewald_total(pos, q, box_len, g_ewald, coulomb_c=1.0):
    """Full Ewald energy and forces (real + reciprocal + self + background)."""
    e_r, f_r = ewald_real(pos, q, box_len, g_ewald, coulomb_c)
    e_k, f_k = ewald_reciprocal(pos, q, box_len, g_ewald, coulomb_c)
    V = float(np.prod(_f64(box_len)))
    e = e_r + e_k + self_energy(q, g_ewald, coulomb_c) + background_energy(q, g_ewald, coulomb_c, V)
    return e, f_r + f_k
