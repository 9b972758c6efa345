"""Seeded synthetic inputs for the Lennard-Jones hot path.

This module only *generates* inputs: lattice sites, seeded random numbers and
box sizes.  It holds none of the method's arithmetic (no potential, no cell
binning, no pair test, no integration), so both the CPU oracle and the GPU
path can take their inputs from here without sharing any computation.

Workload recipe (Sec. 4.5, benchmark conditions): particles start on a
face-centred cubic lattice at reduced number density rho = 0.5 in a periodic
cube.  The lattice constant a = (4/rho)^(1/3) is exactly 2 at rho = 0.5, so a
box of n_fcc unit cells per side has L = 2 n_fcc and N = 4 n_fcc^3.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "fcc_lattice",
    "fcc_lattice_box",
    "maxwell_boltzmann",
    "fixed_speed_velocities",
    "jittered_fcc",
    "uniform_box",
    "shuffle_labels",
    "CONFIGS",
    "PAPER_CONFIGS",
    "initial_velocities",
]

# The five workloads the hot path is exercised on (sizes only), Maxwell-Boltzmann
# velocities at temperature T.
CONFIGS = {
    "lj4k":   dict(n_fcc=10,  rho=0.5, rc=2.5, skin=0.3, T=1.0, dt=0.005, steps=100,  precision="fp64"),
    "lj4m":   dict(n_fcc=100, rho=0.5, rc=2.5, skin=0.3, T=1.0, dt=0.005, steps=1000, precision="fp64"),
    "lj32m":  dict(n_fcc=200, rho=0.5, rc=2.5, skin=0.3, T=1.0, dt=0.005, steps=1000, precision="mixed"),
    "lj256k": dict(n_fcc=40,  rho=0.5, rc=2.5, skin=0.3, T=1.0, dt=0.005, steps=200,  precision="fp64"),
    "lj131m": dict(n_fcc=320, rho=0.5, rc=2.5, skin=0.3, T=1.0, dt=0.005, steps=500,  precision="mixed"),
}

# The paper's own benchmark conditions (Sec. 4.5): 500,000 particles in a
# 100^3 box per process, |v| = 0.9 in random directions, dt = 0.001, rc = 2.5,
# rs = 2.8, 150 untimed steps then 1000 timed, FP64.  paper32m is 64 such
# cubes in one 400^3 box: the share of one node of the paper's first machine.
PAPER_CONFIGS = {
    "paper500k": dict(n_fcc=50,  rho=0.5, rc=2.5, skin=0.3, speed=0.9, dt=0.001, warmup=150, steps=1000,
                      precision="fp64"),
    "paper32m":  dict(n_fcc=200, rho=0.5, rc=2.5, skin=0.3, speed=0.9, dt=0.001, warmup=150, steps=1000,
                      precision="fp64"),
}


def initial_velocities(cfg: dict, n: int, seed: int = 0):
    """Velocities of a workload: fixed speed in random directions when the
    config names a speed (the paper's conditions), else Maxwell-Boltzmann at T."""
    if "speed" in cfg:
        return fixed_speed_velocities(n, cfg["speed"], seed=seed)
    return maxwell_boltzmann(n, cfg["T"], seed=seed)


def lattice_constant(rho: float) -> float:
    """fcc lattice constant for number density rho (4 sites per cubic cell)."""
    return float(np.cbrt(4.0 / rho))


def fcc_lattice(n_fcc: int, rho: float = 0.5):
    """Return (pos[N,3] float64, L) for an n_fcc^3-cell fcc lattice.

    Particle order: unit cells in C order over (ix, iy, iz), then the four
    basis sites (0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2) in units of a.
    No origin offset, so at rho = 0.5 every coordinate is a multiple of 1.0.
    """
    a = lattice_constant(rho)
    i = np.arange(n_fcc, dtype=np.float64)
    ix, iy, iz = np.meshgrid(i, i, i, indexing="ij")
    corners = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)  # [n^3, 3]
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    pos = (corners[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    L = n_fcc * a
    return np.ascontiguousarray(pos), float(L)


def maxwell_boltzmann(n: int, T: float = 1.0, seed: int = 0):
    """Seeded Maxwell-Boltzmann velocities (unit mass) with zero net momentum.

    Draws standard normals, removes the mean, then rescales so that the
    kinetic temperature is exactly T with 3(N-1) degrees of freedom.
    """
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v -= v.mean(axis=0)
    scale = np.sqrt(3.0 * (n - 1) * T / np.sum(v * v))
    return np.ascontiguousarray(v * scale)


def fcc_lattice_box(nx: int, ny: int, nz: int, rho: float = 0.5):
    """fcc lattice of nx x ny x nz unit cells (an anisotropic periodic box).
    Returns (pos[N,3], L[3]); same site order and basis as fcc_lattice."""
    a = lattice_constant(rho)
    ix, iy, iz = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nz, dtype=np.float64), indexing="ij")
    corners = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    pos = (corners[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return np.ascontiguousarray(pos), [nx * a, ny * a, nz * a]


def fixed_speed_velocities(n: int, speed: float = 0.9, seed: int = 0):
    """Velocities of fixed magnitude in random directions (Sec. 4.5 benchmark
    conditions use |v| = 0.9).  No momentum removal, as in the benchmark."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return np.ascontiguousarray(u * speed)


def wrap_into_box(pos: np.ndarray, L) -> np.ndarray:
    """Place coordinates in [0, L) (input preparation only); L scalar or per axis."""
    L = np.asarray(L, dtype=np.float64)
    p = np.mod(pos, L)
    p = np.where(p >= L, p - L, p)
    p = np.where(p < 0.0, p + L, p)
    return np.ascontiguousarray(p)


def jittered_fcc(n_fcc: int, amp: float = 0.15, rho: float = 0.5, seed: int = 1):
    """fcc lattice with seeded Gaussian displacements of std `amp` per axis,
    wrapped into the box: a disordered, overlap-free, liquid-like input."""
    pos, L = fcc_lattice(n_fcc, rho)
    rng = np.random.default_rng(seed)
    pos = pos + amp * rng.standard_normal(pos.shape)
    return wrap_into_box(pos, L), L


def uniform_box(n: int, L: float, seed: int = 2):
    """Uniform random positions in [0, L)^3 (ideal-gas input)."""
    rng = np.random.default_rng(seed)
    return wrap_into_box(rng.random((n, 3)) * L, L)


def shuffle_labels(pos: np.ndarray, vel: np.ndarray | None = None, seed: int = 3):
    """Randomly exchange particle labels, keeping positions and momenta
    (the index shuffle used before the re-sort comparison of Sec. 3.3)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(pos.shape[0])
    out_pos = np.ascontiguousarray(pos[perm])
    out_vel = None if vel is None else np.ascontiguousarray(vel[perm])
    return out_pos, out_vel, perm
