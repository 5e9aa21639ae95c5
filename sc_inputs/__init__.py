"""Seeded synthetic inputs for the two-component Shan-Chen lattice runs.

This module builds initial density fields only; it holds none of the lattice
Boltzmann arithmetic (no equilibria, forces, collisions or streaming). Both the
HIP library's tests/benchmarks and the CPU oracle take their inputs from here,
so that the two sides start from bitwise-identical host arrays.

Conventions
-----------
* Arrays are C-ordered ``[z][y][x]`` (x fastest), float64, shape
  ``(nz, ny, nx)``; 2D lattices have ``nz == 1``.
* Noise is independent U(-a, a) per site and species, drawn from
  ``numpy.random.default_rng(seed)`` (PCG64): first every site of species A in
  x-fastest order, then every site of species B.
* A drop profile is ``rho_A(r) = rho_out + (rho_in - rho_out) * (1 - tanh((r - R)/w)) / 2``
  with ``r`` the minimum-image distance from the centre ``(nx/2, ny/2[, nz/2])``
  in site units; "mirrored" means ``rho_B = rho_in + rho_out - rho_A``.
* A spinodal start is ``rho_A = rho_B = rho0`` plus the noise.

The workload shapes follow the paper's numerical tests (Sec. 4: a static drop
with R/L about 1/4 on a periodic grid) and the 3D spinodal-decomposition and
batched/served workloads of this library's benchmarks.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Fields",
    "min_image_radius",
    "drop",
    "spinodal",
    "flat_interface",
    "JobSpec",
    "batch_jobs",
    "serving_jobs",
    "poisson_arrivals",
]


@dataclasses.dataclass
class Fields:
    """Initial densities of one lattice (host, float64, shape (nz, ny, nx))."""

    rho_A: np.ndarray
    rho_B: np.ndarray
    centre: Tuple[float, float, float]
    radius: float  # nominal drop radius; 0 for a spinodal start

    @property
    def shape(self) -> Tuple[int, int, int]:
        return tuple(self.rho_A.shape)  # type: ignore[return-value]


def _coords(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def _min_image(d: np.ndarray, n: int) -> np.ndarray:
    return d - n * np.round(d / n)


def min_image_radius(nx: int, ny: int, nz: int,
                     centre: Tuple[float, float, float]) -> np.ndarray:
    """Minimum-image distance of every site from ``centre`` (site units)."""
    x, y, z = _coords(nx, ny, nz)
    dx = _min_image(x - centre[0], nx)
    dy = _min_image(y - centre[1], ny)
    r2 = dx * dx + dy * dy
    if nz > 1:
        dz = _min_image(z - centre[2], nz)
        r2 = r2 + dz * dz
    return np.sqrt(r2)


def _noise(rng: np.random.Generator, shape, amp: float) -> np.ndarray:
    if amp == 0.0:
        return np.zeros(shape)
    return rng.uniform(-amp, amp, size=shape)


def drop(nx: int, ny: int, nz: int = 1, *, radius: float, rho_in: float = 1.0,
         rho_out: float = 0.05, width: float = 2.0, noise: float = 1e-3,
         seed: int = 1, centre: Optional[Tuple[float, float, float]] = None) -> Fields:
    """A drop of species A (disc in 2D, sphere in 3D) in species B, mirrored."""
    if centre is None:
        centre = (nx / 2.0, ny / 2.0, nz / 2.0 if nz > 1 else 0.0)
    r = min_image_radius(nx, ny, nz, centre)
    prof = 0.5 * (1.0 - np.tanh((r - radius) / width))
    rho_A = rho_out + (rho_in - rho_out) * prof
    rho_B = rho_in + rho_out - rho_A
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    nA = _noise(rng, shape, noise)
    nB = _noise(rng, shape, noise)
    return Fields(np.ascontiguousarray(rho_A + nA), np.ascontiguousarray(rho_B + nB),
                  centre, float(radius))


def spinodal(nx: int, ny: int, nz: int = 1, *, rho0: float = 0.5, noise: float = 0.01,
             seed: int = 3) -> Fields:
    """Uniform symmetric mixture rho_A = rho_B = rho0 plus per-site noise."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    nA = _noise(rng, shape, noise)
    nB = _noise(rng, shape, noise)
    base = np.full(shape, rho0)
    return Fields(np.ascontiguousarray(base + nA), np.ascontiguousarray(base + nB),
                  (nx / 2.0, ny / 2.0, nz / 2.0 if nz > 1 else 0.0), 0.0)


def flat_interface(nx: int, ny: int = 1, nz: int = 1, *, rho_total: float,
                   phi0: float, width: float = 2.0) -> Fields:
    """Two flat interfaces along x: phi = +phi0 in the middle half, -phi0 outside.

    rho_A = (rho_total + phi)/2, rho_B = (rho_total - phi)/2 (Sec. 2.1 defines
    phi = rho_A - rho_B and rho = rho_A + rho_B).
    """
    x = np.arange(nx, dtype=np.float64)
    a, b = nx / 4.0, 3.0 * nx / 4.0
    prof = 0.5 * (np.tanh((x - a) / width) - np.tanh((x - b) / width))  # ~1 inside
    phi = phi0 * (2.0 * prof - 1.0)
    phi3 = np.broadcast_to(phi, (nz, ny, nx))
    rho_A = np.ascontiguousarray(0.5 * (rho_total + phi3))
    rho_B = np.ascontiguousarray(0.5 * (rho_total - phi3))
    return Fields(rho_A, rho_B, (nx / 2.0, 0.0, 0.0), 0.0)


# --------------------------------------------------------------------------
# Multi-job workloads (batched and served runs)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class JobSpec:
    """One independent lattice job."""

    job_id: int
    lattice: int            # 9 (D2Q9) or 19 (D3Q19)
    nx: int
    ny: int
    nz: int
    tau: float              # tau_A = tau_B
    G: float
    steps: int
    kind: str               # "drop" or "spinodal"
    radius: float = 0.0
    seed: int = 0
    arrival: float = 0.0    # seconds after the start of a served run

    @property
    def sites(self) -> int:
        return self.nx * self.ny * self.nz

    def fields(self) -> Fields:
        if self.kind == "drop":
            return drop(self.nx, self.ny, self.nz, radius=self.radius, seed=self.seed)
        return spinodal(self.nx, self.ny, self.nz, seed=self.seed)


def _r_lo(L: int) -> float:
    """Smallest drop radius drawn: 8 sites, less on lattices under 64 sites."""
    return min(8.0, L / 8.0)


def batch_jobs(n_jobs: int = 64, *, seed: int = 4, l_min: int = 64, l_max: int = 512,
               steps: int = 2000) -> List[JobSpec]:
    """Independent square D2Q9 drop lattices of uneven sizes.

    L ~ U{l_min..l_max}, R ~ U[8, L/4] (8 -> L/8 below L = 64), G ~ U[1.2, 1.6],
    tau ~ U[0.6, 1.5].
    """
    rng = np.random.default_rng(seed)
    jobs = []
    for k in range(n_jobs):
        L = int(rng.integers(l_min, l_max + 1))
        R = float(rng.uniform(_r_lo(L), L / 4.0))
        G = float(rng.uniform(1.2, 1.6))
        tau = float(rng.uniform(0.6, 1.5))
        jobs.append(JobSpec(k, 9, L, L, 1, tau, G, steps, "drop", R,
                            seed=int(rng.integers(0, 2**31 - 1))))
    return jobs


def poisson_arrivals(n: int, rate: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream with the given rate (1/s)."""
    gaps = rng.exponential(1.0 / rate, size=n)
    return np.cumsum(gaps) - gaps[0]


def serving_jobs(n_jobs: int = 200, *, seed: int = 5, rate: float = 1.0,
                 step_range: Tuple[int, int] = (500, 5000),
                 l2: Tuple[int, int] = (64, 512), l3: Tuple[int, int] = (64, 256),
                 frac_3d: float = 0.3) -> List[JobSpec]:
    """A Poisson stream of drop / spinodal jobs.

    70% D2Q9 drops L ~ U{l2}; 30% D3Q19 with L ~ U{l3}, half drops (tau = 1,
    G = 1.3) and half spinodal (tau = 1, G = 1.6). Steps ~ U{step_range}.
    """
    rng = np.random.default_rng(seed)
    arrivals = poisson_arrivals(n_jobs, rate, rng)
    jobs = []
    for k in range(n_jobs):
        steps = int(rng.integers(step_range[0], step_range[1] + 1))
        js = int(rng.integers(0, 2**31 - 1))
        if rng.uniform() >= frac_3d:
            L = int(rng.integers(l2[0], l2[1] + 1))
            R = float(rng.uniform(_r_lo(L), L / 4.0))
            G = float(rng.uniform(1.2, 1.6))
            tau = float(rng.uniform(0.6, 1.5))
            jobs.append(JobSpec(k, 9, L, L, 1, tau, G, steps, "drop", R, js,
                                float(arrivals[k])))
        else:
            L = int(rng.integers(l3[0], l3[1] + 1))
            if rng.uniform() < 0.5:
                R = float(rng.uniform(_r_lo(L), L / 4.0))
                jobs.append(JobSpec(k, 19, L, L, L, 1.0, 1.3, steps, "drop", R, js,
                                    float(arrivals[k])))
            else:
                jobs.append(JobSpec(k, 19, L, L, L, 1.0, 1.6, steps, "spinodal", 0.0, js,
                                    float(arrivals[k])))
    return jobs
