"""Seeded synthetic trap arrays shaped like the paper's workloads.

This module only draws inputs: SLM geometry, trap positions (x, y, z) in metres
and the random trap phases theta0.  It holds none of the hologram arithmetic, so
that both the FP64 oracle (under ``oracle/``) and the HIP path can be fed the
same numbers without sharing any code of the method.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).  The random
phases of random superposition (Eq. 3 of the paper, "theta_m is a random phase")
are drawn here and passed into both implementations.

Optics used for every workload: pixel pitch 15 um, wavelength 1.064 um,
effective focal length 5 mm.  The trap "box" of 40 x 40 x 20 um is read as
x, y in [-20, 20) um and z in [-10, 10) um, centred on the focus.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

PITCH = 15e-6
WAVELENGTH = 1.064e-6
FOCAL = 5e-3
UM = 1e-6
BOX_LO = np.array([-20.0, -20.0, -10.0]) * UM
BOX_HI = np.array([20.0, 20.0, 10.0]) * UM


@dataclass
class Slm:
    """SLM pixel grid and optics: nx columns (x), ny rows (y), SI units."""

    nx: int
    ny: int
    pitch: float = PITCH
    wavelength: float = WAVELENGTH
    focal: float = FOCAL

    @property
    def n(self) -> int:
        return self.nx * self.ny


@dataclass
class Problem:
    """One hologram problem: SLM + M traps (xyz [M,3] metres) + theta0 [M] radians."""

    slm: Slm
    xyz: np.ndarray
    theta0: np.ndarray
    iters: int = 0
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.xyz.shape[0])


@dataclass
class Batch:
    """B problems that share one SLM; traps concatenated (xyz [sum M, 3])."""

    slm: Slm
    counts: np.ndarray           # int32 [B]
    xyz: np.ndarray              # [sum M, 3]
    theta0: np.ndarray           # [sum M]
    iters: int = 0
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def b(self) -> int:
        return int(self.counts.shape[0])

    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)

    def problem(self, i: int) -> Problem:
        o = self.offsets()
        return Problem(self.slm, self.xyz[o[i]:o[i + 1]], self.theta0[o[i]:o[i + 1]],
                       self.iters, f"{self.name}[{i}]")


def box_uniform(rng: np.random.Generator, m: int) -> np.ndarray:
    """m points uniform in the 40 x 40 x 20 um box."""
    return rng.uniform(BOX_LO, BOX_HI, size=(m, 3))


def random_phases(seed: int, m: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, size=m)


def grid_4x4(spacing: float = 3 * UM) -> np.ndarray:
    """4 x 4 planar grid at z = 0, trap index m = 4*j + i, x = (i-1.5)s, y = (j-1.5)s."""
    xyz = np.zeros((16, 3))
    for j in range(4):
        for i in range(4):
            xyz[4 * j + i] = [(i - 1.5) * spacing, (j - 1.5) * spacing, 0.0]
    return xyz


def square_grid(n: int, spacing: float, z: float = 0.0) -> np.ndarray:
    """n x n planar grid centred on the axis (the paper's Fig. 7 trap arrays)."""
    xyz = np.zeros((n * n, 3))
    for j in range(n):
        for i in range(n):
            xyz[n * j + i] = [(i - (n - 1) / 2) * spacing, (j - (n - 1) / 2) * spacing, z]
    return xyz


def hex_patch(rows: int = 5, cols: int = 8, a: float = 3 * UM) -> np.ndarray:
    """rows x cols patch of a triangular lattice (row pitch a*sqrt(3)/2, odd rows
    shifted by a/2), centroid moved to the origin; returns [rows*cols, 2]."""
    pts = []
    for r in range(rows):
        for c in range(cols):
            pts.append([c * a + (a / 2 if r % 2 else 0.0), r * a * math.sqrt(3) / 2])
    pts = np.array(pts)
    return pts - pts.mean(axis=0)


# ---------------------------------------------------------------- the five workloads

def c1() -> Problem:
    """GSW, 256 x 256 SLM, 4 x 4 planar grid (3 um spacing), 30 iterations."""
    return Problem(Slm(256, 256), grid_4x4(), random_phases(1, 16), 30, "gsw-256sq-4x4grid")


def c1_mirror_theta(theta: np.ndarray) -> np.ndarray:
    """theta0 made equal on the x-mirror pairs i <-> 3-i of the 4 x 4 grid."""
    t = np.array(theta, dtype=np.float64).copy()
    for j in range(4):
        for i in range(2):
            t[4 * j + 3 - i] = t[4 * j + i]
    return t


def c2() -> Problem:
    """RS / GS / GSW, 512 x 512 SLM, 100 traps uniform in the box, 50 iterations."""
    rng = np.random.default_rng(2)
    return Problem(Slm(512, 512), box_uniform(rng, 100), random_phases(102, 100), 50,
                   "gsw-512sq-100traps")


def c3() -> Problem:
    """GSW, 1024 x 1024 SLM, 256 traps: 5 planes of a 40-point hex patch + 56 random."""
    patch = hex_patch()
    planes = []
    for z in (-8, -4, 0, 4, 8):
        p = np.zeros((patch.shape[0], 3))
        p[:, :2] = patch
        p[:, 2] = z * UM
        planes.append(p)
    rng = np.random.default_rng(3)
    xyz = np.concatenate(planes + [box_uniform(rng, 56)], axis=0)
    return Problem(Slm(1024, 1024), xyz, random_phases(103, 256), 40, "gsw-1024sq-256traps")


def c4(b: int = 64) -> Batch:
    """64 independent 512 x 512 holograms, trap counts uniform in [4, 256], 30 iterations."""
    rng = np.random.default_rng(4)
    counts = rng.integers(4, 257, 64).astype(np.int32)[:b]
    xyz = np.concatenate([box_uniform(rng, int(m)) for m in counts], axis=0)
    theta = random_phases(104, int(counts.sum()))
    return Batch(Slm(512, 512), counts, xyz, theta, 30, "gsw-batched-64x512sq")


def c5() -> Batch:
    """8 holograms, 512 x 512, 64 random 3D traps each; the differentiable-hologram workload."""
    rng = np.random.default_rng(5)
    counts = np.full(8, 64, dtype=np.int32)
    xyz = box_uniform(rng, 8 * 64)
    theta = random_phases(105, 8 * 64)
    return Batch(Slm(512, 512), counts, xyz, theta, 200, "adjoint-8x512sq-64traps",
                 extra={"adam_lr": 0.05, "adam_steps": 200})


def c5_fd_case() -> tuple[Problem, np.ndarray]:
    """Finite-difference check case: 64 x 64 SLM, 4 traps, random phase mask."""
    rng = np.random.default_rng(6)
    prob = Problem(Slm(64, 64), box_uniform(rng, 4), random_phases(6, 4), 0, "fd-64sq-4traps")
    phi = np.random.default_rng(106).uniform(0.0, 2.0 * math.pi, size=64 * 64)
    return prob, phi


def random_problem(seed: int, nx: int, ny: int, m: int, iters: int = 0) -> Problem:
    """Generic seeded problem (traps in the box) for tests at arbitrary sizes."""
    rng = np.random.default_rng(seed)
    return Problem(Slm(nx, ny), box_uniform(rng, m), rng.uniform(0, 2 * math.pi, m), iters,
                   f"rand-{nx}x{ny}-{m}")


def rotating_cube(frame: int, n_frames: int = 96, side: float = 5 * UM) -> np.ndarray:
    """8 traps on the vertices of a cube of the given side, rigidly rotated about y
    by 2*pi*frame/n_frames (the paper's interactive demonstration)."""
    h = side / 2
    v = np.array([[sx * h, sy * h, sz * h] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)])
    a = 2 * math.pi * frame / n_frames
    rot = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
    return v @ rot.T


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3}
