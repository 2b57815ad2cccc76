"""Seeded synthetic initial conditions for the direct N-body workloads.

This module draws inputs only; it holds none of the force, integrator or
adjoint arithmetic.  Both the FP64 oracle (tests) and the GPU path take
their particles from here, so the two sides see bit-identical inputs.

Workloads (the paper's runs use equal-mass Plummer spheres in N-body units,
Section 4, Results):

* :func:`plummer` -- Aarseth-Henon-Wielen sampling of a Plummer sphere,
  G = M = 1, virial radius 1 (scale radius b = 3*pi/16), optionally with
  Salpeter masses (slope 2.35 on [0.1, 100], normalised to total mass 1).
* :func:`clusters` -- many independent Plummer spheres with log-uniform
  particle counts and per-cluster softening 1/(4 N^(1/3)).

Every array is float64, C-contiguous; vectors are (3, n) rows x, y, z.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["SEED_BASE", "seed_for", "rng", "plummer", "salpeter_masses",
           "clusters", "Particles", "workload", "WORKLOADS"]

#: Seeds are SEED_BASE + workload index (0 .. 4); see :data:`WORKLOADS`.
SEED_BASE = 70743800

PLUMMER_B = 3.0 * math.pi / 16.0   # scale radius for virial radius 1 (G = M = 1)
X1_MAX = 0.999                     # mass-fraction cut of the radial draw


def seed_for(k: int) -> int:
    return SEED_BASE + int(k)


def rng(seed: int, *spawn_key: int) -> np.random.Generator:
    """PCG64 generator for ``seed`` and an optional spawn path."""
    ss = np.random.SeedSequence(seed, spawn_key=tuple(int(s) for s in spawn_key))
    return np.random.Generator(np.random.PCG64(ss))


@dataclass
class Particles:
    pos: np.ndarray    # (3, n) float64
    vel: np.ndarray    # (3, n) float64
    mass: np.ndarray   # (n,) float64

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])


def _isotropic(g: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere, shape (3, n)."""
    cz = g.uniform(-1.0, 1.0, n)
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz])


def salpeter_masses(n: int, seed: int, alpha: float = 2.35, m_lo: float = 0.1,
                    m_hi: float = 100.0) -> np.ndarray:
    """Power-law masses dN/dm ~ m^-alpha on [m_lo, m_hi], normalised to sum 1
    (inverse-CDF draw)."""
    g = rng(seed, 1)
    x = g.uniform(0.0, 1.0, n)
    p = 1.0 - alpha
    m = (m_lo ** p + x * (m_hi ** p - m_lo ** p)) ** (1.0 / p)
    return m / m.sum()


def plummer(n: int, seed: int, masses: str = "equal") -> Particles:
    """Plummer sphere by Aarseth-Henon-Wielen (1974) sampling in N-body units.

    Radius: r = b (X^(-2/3) - 1)^(-1/2) with X uniform on (0, 0.999).
    Speed: q v_esc(r), v_esc = sqrt(2/b) (1 + r^2/b^2)^(-1/4), q drawn by
    rejection from g(q) = q^2 (1 - q^2)^(7/2) under the bound 0.1.
    Directions isotropic; centre of mass moved to rest at the origin.
    Masses independent of position (no segregation).
    """
    if n <= 0:
        raise ValueError("n must be positive")
    g = rng(seed, 0)
    b = PLUMMER_B
    x1 = g.uniform(0.0, X1_MAX, n)
    x1 = np.where(x1 == 0.0, X1_MAX * 0.5, x1)
    r = b / np.sqrt(x1 ** (-2.0 / 3.0) - 1.0)
    pos = r * _isotropic(g, n)
    q = np.empty(n)
    filled = 0
    while filled < n:
        want = n - filled
        m = max(16, int(want * 2.2))
        x4 = g.uniform(0.0, 1.0, m)
        x5 = g.uniform(0.0, 1.0, m)
        ok = 0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
        acc = x4[ok][:want]
        q[filled:filled + acc.size] = acc
        filled += acc.size
    vesc = math.sqrt(2.0 / b) * (1.0 + (r / b) ** 2) ** (-0.25)
    vel = (q * vesc) * _isotropic(g, n)
    if masses == "equal":
        mass = np.full(n, 1.0 / n)
    elif masses == "salpeter":
        mass = salpeter_masses(n, seed)
    else:
        raise ValueError(f"unknown mass spectrum {masses!r}")
    mtot = mass.sum()
    pos -= (pos * mass).sum(axis=1, keepdims=True) / mtot
    vel -= (vel * mass).sum(axis=1, keepdims=True) / mtot
    return Particles(np.ascontiguousarray(pos), np.ascontiguousarray(vel),
                     np.ascontiguousarray(mass))


def clusters(n_clusters: int, seed: int, n_lo: int = 64, n_hi: int = 8192):
    """Independent Plummer clusters with log-uniform sizes.

    Returns (offsets int64 [n_clusters+1], eps float64 [n_clusters],
    Particles concatenated).  eps_c = 1 / (4 N_c^(1/3)).
    """
    g = rng(seed, 2)
    sizes = np.rint(np.exp(g.uniform(math.log(n_lo), math.log(n_hi), n_clusters))).astype(np.int64)
    sizes = np.clip(sizes, n_lo, n_hi)
    offsets = np.zeros(n_clusters + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    parts = [plummer(int(nc), seed * 1000 + c + 1) for c, nc in enumerate(sizes)]
    pos = np.ascontiguousarray(np.concatenate([p.pos for p in parts], axis=1))
    vel = np.ascontiguousarray(np.concatenate([p.vel for p in parts], axis=1))
    mass = np.ascontiguousarray(np.concatenate([p.mass for p in parts]))
    eps = 1.0 / (4.0 * sizes.astype(np.float64) ** (1.0 / 3.0))
    return offsets, eps, Particles(pos, vel, mass)


#: The five workloads: name -> (index, description).
WORKLOADS = {
    "plummer1k_hermite": 0,       # N=1024, eps=1/256, shared dt=1/256 to t=0.125
    "salpeter64k_block": 1,       # N=65536 Salpeter, eps=1e-3, block steps
    "plummer1m_force": 2,         # N=2^20, eps=1e-4, one full evaluation
    "plummer16k_adjoint": 3,      # N=16384, eps=1e-3, 64 steps dt=1/128 + VJP
    "clusters512_batched": 4,     # 512 clusters, N_c in [64, 8192]
}


def workload(name: str, n: int | None = None) -> Particles:
    """Particles of a named workload (optionally a smaller n, same recipe)."""
    k = WORKLOADS[name]
    sizes = {0: 1024, 1: 65536, 2: 1 << 20, 3: 16384}
    if k == 4:
        raise ValueError("use clusters() for the batched workload")
    nn = sizes[k] if n is None else int(n)
    return plummer(nn, seed_for(k), "salpeter" if k == 1 else "equal")
