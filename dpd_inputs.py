"""Seeded synthetic inputs for the DPD hot path.

This module is shared by the CPU oracle's tests and by the GPU path's tests
and benchmark.  It only draws random configurations (numpy PCG64 streams):
it holds none of the method's arithmetic (no forces, no neighbour rules, no
integration), so neither side can lean on the other through it.

Every workload mirrors a configuration the paper's method is run on:

* ``uniform_fluid``   single-species DPD fluid (Groot-Warren parameters),
* ``poiseuille``      the reverse-Poiseuille channel (body force +/-g along x),
* ``amphiphile``      solvent W plus H1T3 four-bead chains (harmonic bonds),
* ``batched_systems`` many small independent fluids of log-uniform size,
* ``binary_mixture``  an A/B fluid for the force-matching adjoint.

Arrays follow the library layout: positions / velocities ``float64[3, N]``
(structure of arrays), tags ``uint32[N]`` (tag = initial index), types
``uint8[N]``, bond partners ``int32[N, 2]`` indexed by tag (-1 = none).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One output of Vigna's SplitMix64 generator for state ``x``.

    Used only to derive independent 64-bit seeds for replica systems.
    """
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


@dataclass
class System:
    """A synthetic DPD system: state arrays plus the physical parameters."""

    box: np.ndarray                 # float64[3]
    x: np.ndarray                   # float64[3, N], in [0, box)
    v: np.ndarray                   # float64[3, N]
    tag: np.ndarray                 # uint32[N]
    type: np.ndarray                # uint8[N]
    n_types: int = 1
    a: np.ndarray = field(default_factory=lambda: np.array([[25.0]]))
    gamma: np.ndarray = field(default_factory=lambda: np.array([[4.5]]))
    sigma: np.ndarray = field(default_factory=lambda: np.array([[3.0]]))
    r_c: float = 1.0
    s: float = 0.5
    dt: float = 0.01
    lam: float = 0.5
    seed: int = 0
    body_g: float = 0.0             # +g for y < body_split, -g otherwise
    body_split: float = 0.0
    bond_k: float = 0.0
    bond_r0: float = 0.0
    partner: Optional[np.ndarray] = None   # int32[N, 2] by tag, -1 = none
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[1])


def _uniform_positions(rng, n, box):
    x = np.empty((3, n), dtype=np.float64)
    for k in range(3):
        x[k] = rng.uniform(0.0, box[k], size=n)
        # uniform() can round up to the upper bound; keep x in [0, L)
        x[k][x[k] >= box[k]] = 0.0
    return x


def _velocities(rng, n, kbt=1.0):
    v = rng.standard_normal(size=(3, n))
    if kbt != 1.0:
        v *= np.sqrt(kbt)                   # Maxwell-Boltzmann at k_B T (m = 1)
    v -= v.mean(axis=1, keepdims=True)      # zero total momentum
    return np.ascontiguousarray(v)


def uniform_fluid(n: int, box, seed: int, *, a=25.0, gamma=4.5, sigma=3.0,
                  r_c=1.0, s=0.5, dt=0.01, lam=0.5, rng_seed=None, kbt=1.0) -> System:
    """Single-species fluid: positions uniform in the box, v ~ N(0, k_B T)
    minus the mean."""
    box = np.asarray(box, dtype=np.float64).reshape(3)
    rng = np.random.Generator(np.random.PCG64(seed if rng_seed is None else rng_seed))
    x = _uniform_positions(rng, n, box)
    v = _velocities(rng, n, kbt)
    return System(box=box, x=x, v=v, tag=np.arange(n, dtype=np.uint32),
                  type=np.zeros(n, dtype=np.uint8), n_types=1,
                  a=np.array([[a]]), gamma=np.array([[gamma]]), sigma=np.array([[sigma]]),
                  r_c=r_c, s=s, dt=dt, lam=lam, seed=seed, name=f"fluid{n}")


def fluid_cube(n: int, rho: float, seed: int, **kw) -> System:
    side = (n / rho) ** (1.0 / 3.0)
    return uniform_fluid(n, (side, side, side), seed, **kw)


def small_fluid(seed: int = 1) -> System:
    """The 3,000-particle parity workload: box 10^3, density 3."""
    return uniform_fluid(3000, (10.0, 10.0, 10.0), seed)


def poiseuille(seed: int = 2, box=(20.0, 40.0, 20.0), rho=4.0, g=0.055) -> System:
    """Reverse-Poiseuille channel: +g along x for y < L_y/2, -g above."""
    box = np.asarray(box, dtype=np.float64)
    n = int(round(rho * box.prod()))
    sys_ = uniform_fluid(n, box, seed)
    sys_.body_g = g
    sys_.body_split = 0.5 * box[1]
    sys_.name = f"poiseuille{n}"
    return sys_


# type ids of the amphiphile workload
W, H, T = 0, 1, 2


def amphiphile(n: int = 16_000_000, seed: int = 3, rho: float = 3.0,
               chain_fraction: float = 0.1, bond_k=100.0, bond_r0=0.7) -> System:
    """Solvent W plus H1T3 chains (bonds 1-2, 2-3, 3-4) in a cubic periodic box.

    Chain c owns tags 4c..4c+3 (H, T, T, T); the first bead is uniform, each
    next bead sits at distance r0 from its predecessor in a uniform random
    direction (then wrapped into the box).  The rest of the tags are W.
    """
    side = (n / rho) ** (1.0 / 3.0)
    box = np.array([side, side, side])
    rng = np.random.Generator(np.random.PCG64(seed))
    n_chain_beads = int(round(chain_fraction * n)) // 4 * 4
    n_chains = n_chain_beads // 4
    x = _uniform_positions(rng, n, box)
    typ = np.zeros(n, dtype=np.uint8)
    partner = np.full((n, 2), -1, dtype=np.int32)
    if n_chains:
        heads = np.arange(n_chains, dtype=np.int64) * 4
        pos = x[:, heads].copy()
        for b in range(1, 4):
            u = rng.standard_normal(size=(3, n_chains))
            u /= np.linalg.norm(u, axis=0, keepdims=True)
            pos = pos + bond_r0 * u
            pos = np.mod(pos, box[:, None])
            for k in range(3):
                pk = pos[k]
                pk[pk >= box[k]] = 0.0
            x[:, heads + b] = pos
        typ[heads] = H
        for b in range(1, 4):
            typ[heads + b] = T
        # bonds 1-2, 2-3, 3-4: partner slot 0 = previous bead, slot 1 = next
        for b in range(1, 4):
            partner[heads + b, 0] = (heads + b - 1).astype(np.int32)
            partner[heads + b - 1, 1] = (heads + b).astype(np.int32)
    v = _velocities(rng, n)
    a = np.full((3, 3), 25.0)
    a[H, T] = a[T, H] = 75.0
    a[T, W] = a[W, T] = 75.0
    a[H, W] = a[W, H] = 35.0
    return System(box=box, x=x, v=v, tag=np.arange(n, dtype=np.uint32), type=typ,
                  n_types=3, a=a, gamma=np.full((3, 3), 4.5), sigma=np.full((3, 3), 3.0),
                  seed=seed, bond_k=bond_k, bond_r0=bond_r0, partner=partner,
                  name=f"amphiphile{n}")


@dataclass
class BatchSpec:
    n: np.ndarray        # int64[S]
    box: np.ndarray      # float64[S, 3]
    a: np.ndarray        # float64[S]
    gamma: np.ndarray    # float64[S]
    sigma: np.ndarray    # float64[S]
    seed: np.ndarray     # uint64[S]


def batched_spec(n_sys: int = 256, seed: int = 4, n_min=1000, n_max=64000,
                 rho=3.0) -> BatchSpec:
    """Replica ensemble: N_s log-uniform in [n_min, n_max], cubic boxes at rho,
    a ~ U[15,35], gamma ~ U[2,8], sigma = sqrt(2 gamma) (k_BT = 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.rint(np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=n_sys))).astype(np.int64)
    side = (n / rho) ** (1.0 / 3.0)
    box = np.repeat(side[:, None], 3, axis=1)
    a = rng.uniform(15.0, 35.0, size=n_sys)
    gamma = rng.uniform(2.0, 8.0, size=n_sys)
    sigma = np.sqrt(2.0 * gamma)
    seeds = np.array([splitmix64(seed * 1_000_003 + s) for s in range(n_sys)], dtype=np.uint64)
    return BatchSpec(n=n, box=box, a=a, gamma=gamma, sigma=sigma, seed=seeds)


def batched_systems(spec: BatchSpec, seed: int = 5) -> list:
    out = []
    for s in range(len(spec.n)):
        sy = uniform_fluid(int(spec.n[s]), spec.box[s], int(spec.seed[s]),
                           a=float(spec.a[s]), gamma=float(spec.gamma[s]),
                           sigma=float(spec.sigma[s]), rng_seed=seed * 7919 + s)
        out.append(sy)
    return out


def binary_mixture(n: int = 512_000, box=(80.0, 80.0, 80.0 / 3.0), seed: int = 6,
                   a_like=25.0, a_ab=None) -> System:
    """A/B mixture (50:50 random types); a_AB ~ U[25, 50] unless given."""
    box = np.asarray(box, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = _uniform_positions(rng, n, box)
    v = _velocities(rng, n)
    typ = rng.integers(0, 2, size=n).astype(np.uint8)
    if a_ab is None:
        a_ab = float(rng.uniform(25.0, 50.0))
    a = np.array([[a_like, a_ab], [a_ab, a_like]])
    return System(box=box, x=x, v=v, tag=np.arange(n, dtype=np.uint32), type=typ,
                  n_types=2, a=a, gamma=np.full((2, 2), 4.5), sigma=np.full((2, 2), 3.0),
                  seed=seed, name=f"binary{n}")


def shuffled(sys_: System, seed: int) -> System:
    """Same system with particles stored in a random order (tags travel along)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.permutation(sys_.n)
    out = System(**{**sys_.__dict__})
    out.x = np.ascontiguousarray(sys_.x[:, p])
    out.v = np.ascontiguousarray(sys_.v[:, p])
    out.tag = sys_.tag[p].copy()
    out.type = sys_.type[p].copy()
    return out


def edge_case_fluid(seed: int = 7, box=(5.0, 4.5, 3.5), n: int = 180) -> System:
    """A small fluid with planted geometric edge cases.

    Planted: particles at 0 and at the largest double below L; a pair exactly
    at r_c along x and pairs one ulp inside / outside it; a pair whose raw
    separation is exactly L/2 (the minimum-image tie); a pair straddling the
    periodic face.  The remaining particles are uniform.
    """
    box = np.asarray(box, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = _uniform_positions(rng, n, box)
    planted = []
    below = [np.nextafter(box[k], 0.0) for k in range(3)]
    planted.append((0.0, 0.0, 0.0))
    planted.append((below[0], below[1], below[2]))
    # pair at exactly r_c = 1 along x, and one ulp either side
    planted.append((1.25, 1.5, 1.5)); planted.append((2.25, 1.5, 1.5))
    planted.append((1.25, 2.5, 0.5)); planted.append((np.nextafter(2.25, 0.0), 2.5, 0.5))
    planted.append((1.25, 3.5, 2.5)); planted.append((np.nextafter(2.25, 9.0), 3.5, 2.5))
    # raw separation exactly L_x / 2 = 2.5 (min-image tie), far in y/z though
    planted.append((0.5, 0.2, 0.2)); planted.append((3.0, 0.2, 0.2))
    # straddling the x face: 0.1 and L - 0.3 -> separation 0.4 through the face
    planted.append((0.1, 2.0, 2.0)); planted.append((box[0] - 0.3, 2.0, 2.0))
    for idx, p in enumerate(planted):
        x[:, idx] = p
    v = _velocities(rng, n)
    return System(box=box, x=x, v=v, tag=np.arange(n, dtype=np.uint32),
                  type=np.zeros(n, dtype=np.uint8), seed=seed, name="edge")


def clustered_fluid(seed: int = 8, box=(6.0, 6.0, 6.0), n_cluster: int = 150, n_rest: int = 100,
                    size: float = 1.2) -> System:
    """Most particles packed in a small corner region (rows far longer than
    the box-average density suggests), the rest uniform."""
    box = np.asarray(box, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    xc = rng.uniform(0.2, 0.2 + size, size=(3, n_cluster))
    xr = _uniform_positions(rng, n_rest, box)
    x = np.ascontiguousarray(np.concatenate([xc, xr], axis=1))
    n = n_cluster + n_rest
    v = _velocities(rng, n)
    return System(box=box, x=x, v=v, tag=np.arange(n, dtype=np.uint32),
                  type=np.zeros(n, dtype=np.uint8), seed=seed, name="clustered")
