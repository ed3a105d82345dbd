"""Counter-based seeded inputs on the integer node lattice.

Coordinates are integers (X, Y) in [0, M]^2 where M is the number of lattice
units across the domain (-10, 10)^2, so x = -10 + 20 X / M. Both the oracle
and the HIP path export node coordinates in these units.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np



def splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele et al. 2014) on uint64 arrays (wrapping)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _counter(seed: int, stream: int, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    X = np.asarray(X, dtype=np.uint64)
    Y = np.asarray(Y, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = splitmix64(np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(stream))
        c = key ^ (X << np.uint64(32)) ^ Y
        return splitmix64(c)


def uniform01(seed: int, stream: int, X, Y) -> np.ndarray:
    """Uniform numbers in (0, 1): the top 53 bits of the hash, offset by half a step."""
    h = _counter(seed, stream, X, Y)
    return ((h >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def normal(seed: int, stream: int, X, Y) -> np.ndarray:
    """Standard normals by Box-Muller from two independent uniform streams."""
    u1 = uniform01(seed, 2 * stream, X, Y)
    u2 = uniform01(seed, 2 * stream + 1, X, Y)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def crack_mask(X, Y, M: int, edge: int, half_length: float = 1.0) -> np.ndarray:
    """Lattice points of the prescribed crack (Sec. 4: half length l0, a width
    set by the smallest cell): |x| <= half_length and |y| <= h, with h the
    diagonal of the finest cell, whose edge is `edge` lattice units.

    Exact in integers: |y| <= h <=> (2Y - M)^2 <= 8 edge^2, and |x| <= a <=>
    |20X - 10M| <= a M (a is taken as a rational with denominator 1000).
    """
    X = np.asarray(X, dtype=np.int64)
    Y = np.asarray(Y, dtype=np.int64)
    a_num = int(round(half_length * 1000))
    return ((2 * Y - M) ** 2 <= 8 * int(edge) ** 2) & (1000 * np.abs(20 * X - 10 * M) <= a_num * M)


def sneddon_state(X, Y, M: int, edge: int, seed: int = 0, u_std: float = 1e-4,
                  phi_low: float = 0.5, random: bool = True):
    """Raw nodal state (u_x, u_y, phi) before any constraint is applied.

    edge: finest cell edge in lattice units (the degree p on a Q_p lattice).
    random=True: u ~ N(0, u_std) per component, phi ~ U[phi_low, 1] off the
    crack and 0 on it. random=False: u = 0, phi = 1 off the crack, 0 on it
    (the initial state of a load step). Dirichlet zeroing and hanging-node
    interpolation are the consumer's job.
    """
    X = np.asarray(X, dtype=np.int64)
    Y = np.asarray(Y, dtype=np.int64)
    crack = crack_mask(X, Y, M, edge)
    if random:
        ux = u_std * normal(seed, 0, X, Y)
        uy = u_std * normal(seed, 1, X, Y)
        phi = phi_low + (1.0 - phi_low) * uniform01(seed, 4, X, Y)
    else:
        ux = np.zeros(X.shape)
        uy = np.zeros(X.shape)
        phi = np.ones(X.shape)
    phi = np.where(crack, 0.0, phi)
    return ux, uy, phi


def random_vector(X, Y, seed: int, ncomp: int = 3) -> np.ndarray:
    """Blocked vector [c0(n) | c1(n) | ...] of standard normals."""
    return np.concatenate([normal(seed, 16 + c, X, Y) for c in range(ncomp)])


def bernoulli_mask(X, Y, seed: int, prob: float) -> np.ndarray:
    return uniform01(seed, 40, X, Y) < prob


@dataclass(frozen=True)
class WorkloadSpec:
    """Mesh and material parameters of one Sneddon-type workload."""

    name: str
    n_base: int
    n_local: int
    degree: int
    E: float = 1.0
    nu: float = 0.2
    Gc: float = 1.0
    kappa: float = 1e-10
    pressure: float = 1e-3
    coarse: int = 16
    band: tuple = field(default=(2.0, 0.5))

    @property
    def finest_edge(self) -> float:
        return 20.0 / (self.n_base * 2 ** self.n_local)

    @property
    def ell(self) -> float:
        """Length scale l = 2h, h = diagonal of the finest cell."""
        return 2.0 * np.sqrt(2.0) * self.finest_edge


def _w(n, L, p):
    return WorkloadSpec(name=f"sneddon_{n}x{n}_L{L}_Q{p}", n_base=n, n_local=L, degree=p)


WORKLOADS = {w.name: w for w in (
    _w(16, 2, 1), _w(16, 2, 2),
    _w(32, 2, 1), _w(32, 2, 2),
    _w(128, 2, 1), _w(128, 2, 2),
    _w(512, 3, 2),
    _w(1024, 3, 1), _w(1024, 3, 2),
    _w(2048, 4, 2),
)}
