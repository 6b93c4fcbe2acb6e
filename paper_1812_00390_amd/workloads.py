"""Seeded workload definitions (meshes plus solver parameters) for the
benchmark and the serving loop.  Only configuration lives here; every step of
the method runs in the HIP library.

  cavity20k   lid-driven cavity, Re 1000, U 0.1, 100x100 tanh grid (growth 1.08)
              split into 20,000 jittered triangles (seed 0); four-stage RK
  cylinder98k O-grid 256 x 384 quads around a cylinder, h0 = 0.005 D to 30 D,
              Re 100, u_inf 0.1; four-stage RK, free-stream storage reference
  batched64   64 instances, cells log-uniform in [2e3, 2e5] (seed 1), half
              jittered-triangle cavities, half O-grid cylinders, Re uniform in
              [100, 3000], tau = 3 U L / Re per instance; four-stage RK,
              FP16-deviation storage
  streaming   the cavity20k tanh mapping refined to 2048 x 2048 quads, split:
              8.4M triangles, far larger than the on-chip caches
  served      requests of Couette channels, cavities, cylinders and two-cylinder
              meshes (see served_instance)
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import meshgen as mg

U_REF = 0.1

# Cell orders (the library's reorder codes): tiles are runs of consecutive cells,
# so the order sets their shapes.  Measured on one MI355X, Hilbert order is the
# faster for the cylinder O-grids (98k quads: 7.40 against 7.92 us per RK stage;
# the 64-instance batch: 6% more cell-updates/s) and graph bisection for the
# triangulated cavities and the streaming mesh.
ORDER_HILBERT = 2
ORDER_BISECT = 3


@dataclasses.dataclass
class Instance:
    mesh: mg.RawMesh
    tau: float
    u_ref: float             # CFL velocity scale
    u0: tuple                # initial (and storage-reference) velocity
    kind: str
    re: float
    order: int = ORDER_BISECT   # the cell order its mesh is built in

    @property
    def n_cells(self) -> int:
        return self.mesh.n_cells


# The stretching of the 100 x 100 cavity grid (wall growth ratio 1.08 on 100
# cells).  Cavities of other sizes use this same mapping: solving for the
# growth ratio 1.08 at every size would shrink the wall cell as the grid grows
# (1.5e-6 of the side at 282 cells, a twelve-thousandth of the interior cells).
CAVITY_BETA = mg.tanh_beta(100, 1.08)


def cavity_instance(n: int, re: float, seed: int = 0) -> Instance:
    """n x n cells split into 2 n^2 jittered triangles on the 100 x 100 cavity's
    tanh mapping (uniform below 20 cells a side)."""
    m = mg.cavity(n=n, ratio=1.08 if n >= 20 else 1.0, beta=CAVITY_BETA if n >= 20 else None, jitter=0.2,
                  seed=seed, lid_u=U_REF)
    return Instance(m, 3.0 * U_REF * 1.0 / re, U_REF, (0.0, 0.0), "cavity", re)


def cylinder_instance(nr: int, nt: int, re: float, h0: float = 0.005, R: float = 30.0) -> Instance:
    h0 = min(h0, 0.5 * (R - 0.5) / nr)
    m = mg.cylinder(nr=nr, nt=nt, R=R, h0=h0, u_inf=(U_REF, 0.0))
    return Instance(m, 3.0 * U_REF * 1.0 / re, 2 * U_REF, (U_REF, 0.0), "cylinder", re, ORDER_HILBERT)


def two_cylinder_instance(nr: int, nt: int, re: float) -> Instance:
    m = mg.two_cylinders(nr=nr, nt=nt, u_inf=(U_REF, 0.0), h0=min(0.005, 0.4 * 25.0 / nr))
    return Instance(m, 3.0 * U_REF * 1.0 / re, 2 * U_REF, (U_REF, 0.0), "two_cylinders", re, ORDER_HILBERT)


def cavity20k() -> Instance:
    return cavity_instance(100, 1000.0, seed=0)


def cylinder98k() -> Instance:
    return cylinder_instance(256, 384, 100.0)


def couette_instance(n: int) -> Instance:
    """Plate-driven Couette flow as the first configuration (Section 3.1): unit
    channel periodic in x, lid U = 0.1, tau = 0.8, here on n x n cells split
    into 2 n^2 triangles.  Steady and viscous (Re = U L / nu = 0.375), so it
    reaches a residual of 1e-6 within a few thousand steps."""
    m = mg.couette(n, n, U=U_REF, tri=True)
    tau = 0.8
    return Instance(m, tau, U_REF, (0.0, 0.0), "couette", U_REF * 1.0 / (tau / 3.0))


def served_instance(rng: np.random.Generator, n_cells: float,
                    kinds=("couette", "cavity", "cylinder", "two_cylinders")) -> Instance:
    """One request of the served workload: the kind drawn uniformly from `kinds`;
    Couette channels, cavities (Re uniform in [100, 3000]) and cylinders (Re
    uniform in [100, 3000]) of about n_cells cells; two-cylinder meshes of two
    128 x 256 O-blocks (65,536 cells, Re uniform in [100, 200])."""
    kind = kinds[int(rng.integers(len(kinds)))]
    if kind == "couette":
        return couette_instance(max(4, int(round(math.sqrt(n_cells / 2.0)))))
    if kind == "two_cylinders":
        return two_cylinder_instance(128, 256, float(rng.uniform(100.0, 200.0)))
    return random_instance(rng, n_cells, kinds=(kind,))


def random_instance(rng: np.random.Generator, n_cells: float, kinds=("cavity", "cylinder")) -> Instance:
    kind = kinds[int(rng.integers(len(kinds)))]
    re = float(rng.uniform(100.0, 3000.0))
    if kind == "cavity":
        n = max(6, int(round(math.sqrt(n_cells / 2.0))))
        return cavity_instance(n, re, seed=int(rng.integers(1 << 30)))
    if kind == "cylinder":
        nr = max(6, int(round(math.sqrt(n_cells / 1.5))))
        return cylinder_instance(nr, int(round(1.5 * nr)), re)
    nr = max(6, int(round(math.sqrt(n_cells / 4.0))))
    return two_cylinder_instance(nr, 2 * nr, float(rng.uniform(100.0, 200.0)))


def batched(n: int = 64, seed: int = 1, lo: float = 2e3, hi: float = 2e5) -> List[Instance]:
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))
    return [random_instance(rng, float(c)) for c in sizes]


def streaming() -> mg.RawMesh:
    return mg.streaming_cavity(2048)
