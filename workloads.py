"""Seeded synthetic particle systems shaped like the paper's water benchmarks.

The paper measures on a cubic SPC/E water box of 36,000 atoms and on
64x-replicated copies of it (Section 2.4, Section 4.2).  That dataset is not
available here, so these generators build stand-ins with the same shape:
atom counts, water number density, the O/H partial charges and geometry of
SPC/E, and overall charge neutrality.  Uniform random systems of +-1 or
Gaussian charges cover the larger synthetic cases.

This module holds no PPPM arithmetic: it only draws positions and charges and
describes the box, mesh and method parameters of each workload.  Both the
FP64 oracle and the GPU path consume its output; neither imports the other.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# SPC/E water: O-H bond 1.0 A, H-O-H angle 109.47 degrees, charges in e.
SPCE_Q_O = -0.8476
SPCE_Q_H = 0.4238
SPCE_OH = 1.0
SPCE_ANGLE_DEG = 109.47


@dataclass(frozen=True)
class Workload:
    """One synthetic system plus the PPPM parameters it is run with."""

    name: str
    pos: np.ndarray  # (N, 3) float64, wrapped into [0, L)
    q: np.ndarray  # (N,) float64
    box_lo: tuple
    box_len: tuple
    mesh: tuple  # (Kx, Ky, Kz)
    order: int
    g_ewald: float
    diffs: tuple = ("ad",)
    seed: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q.shape[0])

    @property
    def cells(self) -> int:
        return int(self.mesh[0] * self.mesh[1] * self.mesh[2])


def uniform_alternating(n: int, length: float, seed: int):
    """Uniform positions in a cube, charges +1, -1, +1, ... (q_i = (-1)^i)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, length, size=(n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return _wrap(pos, length), q


def uniform_pm1_neutral(n: int, length: float, seed: int):
    """Uniform positions; exactly n/2 charges of +1 and n/2 of -1, shuffled."""
    if n % 2:
        raise ValueError("exact neutrality with +-1 charges needs an even count")
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, length, size=(n, 3))
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    q = rng.permutation(q)
    return _wrap(pos, length), q


def gaussian_neutral(n: int, length: float, sigma: float, seed: int):
    """Uniform positions; charges N(0, sigma) shifted so that they sum to zero."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, length, size=(n, 3))
    q = rng.normal(0.0, sigma, size=n)
    q = q - q.mean()
    return _wrap(pos, length), q


def _random_rotations(rng, m: int) -> np.ndarray:
    """m uniform random rotation matrices from normalised 4-D Gaussian quaternions."""
    quat = rng.normal(size=(m, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    w, x, y, z = quat.T
    rot = np.empty((m, 3, 3))
    rot[:, 0, 0] = 1 - 2 * (y * y + z * z)
    rot[:, 0, 1] = 2 * (x * y - z * w)
    rot[:, 0, 2] = 2 * (x * z + y * w)
    rot[:, 1, 0] = 2 * (x * y + z * w)
    rot[:, 1, 1] = 1 - 2 * (x * x + z * z)
    rot[:, 1, 2] = 2 * (y * z - x * w)
    rot[:, 2, 0] = 2 * (x * z - y * w)
    rot[:, 2, 1] = 2 * (y * z + x * w)
    rot[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return rot


def water_lattice(n_mol: int, length: float, seed: int, extra_zero: int = 0):
    """SPC/E-like water on a jittered cubic lattice with random orientations.

    Lattice of n = ceil(n_mol^(1/3)) sites per side, spacing a = L/n, site
    centres at (i + 1/2) a; n_mol distinct sites are drawn without
    replacement; each O sits at its site centre plus U(-0.1a, 0.1a)^3; the two
    H atoms sit 1.0 A from O at +-half the H-O-H angle in the molecule's body
    frame, which is rotated uniformly at random.  Atom order is O, H, H.
    ``extra_zero`` zero-charge atoms at uniform positions are appended.
    """
    rng = np.random.default_rng(seed)
    n_side = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    while n_side ** 3 < n_mol:
        n_side += 1
    a = length / n_side
    sites = rng.choice(n_side ** 3, size=n_mol, replace=False)
    ix = sites % n_side
    iy = (sites // n_side) % n_side
    iz = sites // (n_side * n_side)
    centre = (np.stack([ix, iy, iz], axis=1) + 0.5) * a
    o_pos = centre + rng.uniform(-0.1 * a, 0.1 * a, size=(n_mol, 3))
    half = math.radians(SPCE_ANGLE_DEG) / 2.0
    body = np.array(
        [
            [SPCE_OH * math.sin(half), 0.0, SPCE_OH * math.cos(half)],
            [-SPCE_OH * math.sin(half), 0.0, SPCE_OH * math.cos(half)],
        ]
    )
    rot = _random_rotations(rng, n_mol)
    h_off = np.einsum("mij,hj->mhi", rot, body)  # (m, 2, 3)
    pos = np.empty((n_mol, 3, 3))
    pos[:, 0] = o_pos
    pos[:, 1] = o_pos + h_off[:, 0]
    pos[:, 2] = o_pos + h_off[:, 1]
    pos = pos.reshape(-1, 3)
    q = np.tile(np.array([SPCE_Q_O, SPCE_Q_H, SPCE_Q_H]), n_mol)
    if extra_zero:
        pos = np.concatenate([pos, rng.uniform(0.0, length, size=(extra_zero, 3))])
        q = np.concatenate([q, np.zeros(extra_zero)])
    return _wrap(pos, length), q


def nacl_lattice(n_side: int = 8, r0: float = 2.5):
    """Rock-salt ion lattice: n_side^3 ions at spacing r0, q = (-1)^(i+j+k)."""
    idx = np.arange(n_side)
    iz, iy, ix = np.meshgrid(idx, idx, idx, indexing="ij")
    pos = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64) * r0
    q = np.where((ix + iy + iz).ravel() % 2 == 0, 1.0, -1.0)
    return pos, q, n_side * r0


def _wrap(pos: np.ndarray, length: float) -> np.ndarray:
    out = np.mod(pos, length)
    out[out >= length] -= length  # np.mod can round up to exactly L
    return out


# The five benchmark systems.  g = 0.30 / A throughout; seeds 1..5.
CONFIG_NAMES = {
    1: "uniform-1k-L20-K16-P5",
    2: "spce-water-32k-L68-K64-P5",
    3: "uniform-524k-L170-K128",
    4: "gaussian-65k-L85-K64-P5",
    5: "spce-water-4.19M-L340-K256-P7",
}


def config(idx: int, order: int | None = None) -> Workload:
    """Workload ``idx`` (1..5).  ``order`` overrides P for the P sweep of config 3."""
    g = 0.30
    if idx == 1:
        pos, q = uniform_alternating(1000, 20.0, seed=1)
        return Workload(CONFIG_NAMES[1], pos, q, (0.0,) * 3, (20.0,) * 3, (16,) * 3,
                        order or 5, g, ("ik",), 1,
                        "1,000 charges, +-1 alternating, uniform in a 20 A cube")
    if idx == 2:
        pos, q = water_lattice(10667, 68.0, seed=2)
        return Workload(CONFIG_NAMES[2], pos, q, (0.0,) * 3, (68.0,) * 3, (64,) * 3,
                        order or 5, g, ("ik", "ad"), 2,
                        "10,667 SPC/E-like molecules (32,001 atoms), 68 A cube")
    if idx == 3:
        pos, q = uniform_pm1_neutral(524288, 170.0, seed=3)
        return Workload(CONFIG_NAMES[3], pos, q, (0.0,) * 3, (170.0,) * 3, (128,) * 3,
                        order or 5, g, ("ad", "ik"), 3,
                        "524,288 +-1 charges (exactly neutral), uniform in a 170 A cube")
    if idx == 4:
        pos, q = gaussian_neutral(65536, 85.0, 0.5, seed=4)
        return Workload(CONFIG_NAMES[4], pos, q, (0.0,) * 3, (85.0,) * 3, (64,) * 3,
                        order or 5, g, ("ad",), 4,
                        "65,536 N(0, 0.5) charges shifted to sum zero, 85 A cube")
    if idx == 5:
        pos, q = water_lattice(1398101, 340.0, seed=5, extra_zero=1)
        return Workload(CONFIG_NAMES[5], pos, q, (0.0,) * 3, (340.0,) * 3, (256,) * 3,
                        order or 7, g, ("ik", "ad"), 5,
                        "1,398,101 SPC/E-like molecules + 1 zero charge (4,194,304 atoms), 340 A cube")
    raise ValueError(f"no workload {idx}")


def interfacial(order: int = 5) -> Workload:
    """Non-uniform load: the 524,288 +-1 charges of the benchmark system packed
    into the lower half of the box along z (a slab at twice the density, the
    upper half vacuum), same box, mesh and split.  Half of the mesh tiles hold
    no charge and the others twice the average."""
    rng = np.random.default_rng(6)
    n, length = 524288, 170.0
    pos = rng.uniform(0.0, 1.0, size=(n, 3)) * np.array([length, length, 0.5 * length])
    q = rng.permutation(np.concatenate([np.ones(n // 2), -np.ones(n // 2)]))
    return Workload("interfacial-524k-L170-K128", _wrap(pos, length), q, (0.0,) * 3, (length,) * 3, (128,) * 3,
                    order, 0.30, ("ad", "ik"), 6,
                    "524,288 +-1 charges in the lower half (z < L/2) of a 170 A cube, vacuum above")


def clustered(kind: str = "pm1", order: int = 7) -> Workload:
    """Dense cluster: 200,000 charges packed into a cube of 16 mesh cells
    (21.25 A) of the 170 A box (mesh 128^3), its corner off the tile grid at
    mesh coordinate 40.3, about 200 times the average density, plus charges
    spread uniformly over the whole box.  kind "pm1": the cluster is +-1
    (exactly neutral) with 100,000 uniform +-1 charges; "one_sign": the
    cluster is all +1, neutralised by 200,000 uniform charges of -1."""
    if kind not in ("pm1", "one_sign"):
        raise ValueError(kind)
    rng = np.random.default_rng(7 if kind == "pm1" else 8)
    length, K = 170.0, 128
    h = length / K
    nc = 200000
    corner = 40.3 * h
    cl = corner + rng.uniform(0.0, 16 * h, size=(nc, 3))
    if kind == "pm1":
        qc = rng.permutation(np.concatenate([np.ones(nc // 2), -np.ones(nc // 2)]))
        nu = 100000
        qu = rng.permutation(np.concatenate([np.ones(nu // 2), -np.ones(nu // 2)]))
    else:
        qc = np.ones(nc)
        nu = nc
        qu = -np.ones(nu)
    un = rng.uniform(0.0, length, size=(nu, 3))
    pos = np.concatenate([cl, un])
    q = np.concatenate([qc, qu])
    perm = rng.permutation(len(q))
    return Workload(f"clustered-{kind}-L170-K128", _wrap(pos[perm], length), q[perm], (0.0,) * 3, (length,) * 3,
                    (K,) * 3, order, 0.30, ("ad", "ik"), 7 if kind == "pm1" else 8,
                    f"{nc:,} {'+-1' if kind == 'pm1' else '+1'} charges in a 16-cell cube of a 170 A box plus "
                    f"{nu:,} uniform charges")


def random_system(n: int, box_len, seed: int, charge: str = "gaussian", box_lo=(0.0, 0.0, 0.0)):
    """Small general test system: uniform positions in an orthorhombic box."""
    rng = np.random.default_rng(seed)
    box_len = np.asarray(box_len, dtype=np.float64)
    pos = np.asarray(box_lo) + rng.uniform(0.0, 1.0, size=(n, 3)) * box_len
    if charge == "gaussian":
        q = rng.normal(0.0, 1.0, size=n)
        q -= q.mean()
    elif charge == "pm1":
        q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    elif charge == "positive":
        q = rng.uniform(0.5, 1.5, size=n)
    else:
        raise ValueError(charge)
    return pos, q
