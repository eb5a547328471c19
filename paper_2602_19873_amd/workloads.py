"""Seeded synthetic particle systems.

This module only draws inputs. It holds none of the neighbour-list or SPH
arithmetic, so both the GPU path and the CPU oracle can be fed from it.

Every array is drawn in float64 with numpy's PCG64 generator and cast to
float32 once. Seeds are ``SEED_BASE + config_id`` for the single-system
workloads and ``SEED_BASE * 100 + k`` for system ``k`` of a batch.

Workloads (the paper's benchmarks are synthetic: a near-uniform 4M-atom
Lennard-Jones box with ~200 list neighbours, Sec. III-B, and an Evrard
sphere whose density falls off as 1/r, Sec. IV):

* ``uniform_global``   N uniform points in [0,1)^3, one radius r_c for all.
* ``uniform_varied``   as above, radii r_c * U(0.8, 1.2).
* ``evrard_sphere``    density proportional to 1/r inside the unit sphere.
* ``plummer``          Plummer sphere (scale radius a), truncated at 10 a.
* ``batch_systems``    64 systems of log-uniform size in [1e4, 1e6], half
                        uniform cubes and half Plummer spheres.
* ``lj_lattice``       the Lennard-Jones benchmark box: a jittered simple
                        cubic lattice of n_side^3 atoms in [0,1)^3 with
                        rock-salt charges, list radius for ~200 neighbours
                        and interaction cutoff for ~150.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 260219873

UNIT_BOX = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
SPHERE_BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def radius_for_neighbours(n: int, target: float = 200.0, volume: float = 1.0) -> float:
    """Radius whose sphere holds ``target`` particles at mean density n/volume."""
    return (3.0 * target * volume / (4.0 * math.pi * max(n, 1))) ** (1.0 / 3.0)


@dataclass
class ParticleSystem:
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    h: np.ndarray
    m: np.ndarray | None
    box: tuple
    meta: dict = field(default_factory=dict)
    q: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def uniform_global(n: int, seed: int, target: float = 200.0) -> ParticleSystem:
    rng = np.random.default_rng(seed)
    pos = rng.random((3, n))
    rc = radius_for_neighbours(n, target)
    h = np.full(n, rc)
    return ParticleSystem("uniform_global", _f32(pos[0]), _f32(pos[1]), _f32(pos[2]),
                          _f32(h), None, UNIT_BOX, {"r_c": rc, "seed": seed})


def uniform_varied(n: int, seed: int, target: float = 200.0,
                   lo: float = 0.8, hi: float = 1.2) -> ParticleSystem:
    rng = np.random.default_rng(seed)
    pos = rng.random((3, n))
    rc = radius_for_neighbours(n, target)
    h = rc * rng.uniform(lo, hi, n)
    return ParticleSystem("uniform_varied", _f32(pos[0]), _f32(pos[1]), _f32(pos[2]),
                          _f32(h), None, UNIT_BOX, {"r_c": rc, "seed": seed})


def _isotropic(rng, r):
    n = r.shape[0]
    cz = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * math.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return r * s * np.cos(phi), r * s * np.sin(phi), r * cz


def evrard_sphere(n: int, seed: int, target: float = 100.0, seed_h: str = "global") -> ParticleSystem:
    """Unit sphere with number density n(r) = N / (2 pi r): r = sqrt(u).

    ``seed_h='global'`` gives every particle the mean-density radius
    (the plain starting guess); ``'analytic'`` uses the local density.
    """
    rng = np.random.default_rng(seed)
    r = np.sqrt(rng.random(n))
    x, y, z = _isotropic(rng, r)
    if seed_h == "analytic":
        dens = n / (2.0 * math.pi * np.maximum(r, n ** -0.5))
        h = (3.0 * target / (4.0 * math.pi * dens)) ** (1.0 / 3.0)
    else:
        h = np.full(n, radius_for_neighbours(n, target, 4.0 * math.pi / 3.0))
    return ParticleSystem("evrard_sphere", _f32(x), _f32(y), _f32(z), _f32(h), None,
                          SPHERE_BOX, {"seed": seed, "target": target})


def plummer(n: int, seed: int, a: float = 0.1, target: float = 150.0) -> ParticleSystem:
    rng = np.random.default_rng(seed)
    r = np.empty(n)
    filled = 0
    while filled < n:
        u = rng.random(n - filled)
        u = u[u > 0.0]
        rr = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        rr = rr[rr <= 10.0 * a]
        k = min(rr.shape[0], n - filled)
        r[filled:filled + k] = rr[:k]
        filled += k
    x, y, z = _isotropic(rng, r)
    vol = (2.0 * 10.0 * a) ** 3
    h = np.full(n, radius_for_neighbours(n, target, vol))
    return ParticleSystem("plummer", _f32(x), _f32(y), _f32(z), _f32(h), None,
                          SPHERE_BOX, {"seed": seed, "a": a, "target": target})


def batch_systems(count: int = 64, target: float = 150.0, lo: float = 1e4, hi: float = 1e6):
    systems = []
    for k in range(count):
        rng = np.random.default_rng(SEED_BASE * 100 + k)
        nk = int(round(10.0 ** rng.uniform(math.log10(lo), math.log10(hi))))
        seed = SEED_BASE * 100 + 1000 + k
        if k % 2 == 0:
            s = uniform_global(nk, seed, target)
        else:
            s = plummer(nk, seed, target=target)
        systems.append(s)
    return systems


def lj_lattice(n_side: int, seed: int, jitter: float = 0.2, list_target: float = 200.0,
               cut_target: float = 150.0) -> ParticleSystem:
    """Near-uniform atoms for the Lennard-Jones benchmark (Sec. III: about 200
    neighbours inside the list cutoff, 150 inside the interaction cutoff).

    Atom (i, j, k) sits at ((i, j, k) + 1/2 + U(-jitter, jitter)^3) a with
    a = 1/n_side, so no two atoms come closer than (1 - 2 jitter) a. Charges
    alternate +-1/2 with the parity of i + j + k (rock salt, neutral for even
    n_side). sigma = 0.9 a (reduced density 0.729), eps = 1, Coulomb prefactor
    4 a (a charge pair at distance a has energy of order eps). h is the list
    radius for every atom; meta holds the pass parameters."""
    rng = np.random.default_rng(seed)
    a = 1.0 / n_side
    g = np.indices((n_side,) * 3).reshape(3, -1).astype(np.float64)
    pos = (g + 0.5 + rng.uniform(-jitter, jitter, g.shape)) * a
    n = pos.shape[1]
    q = np.where(g.sum(axis=0).astype(np.int64) % 2 == 0, 0.5, -0.5)
    r_list = radius_for_neighbours(n, list_target)
    r_cut = radius_for_neighbours(n, cut_target)
    return ParticleSystem("lj_lattice", _f32(pos[0]), _f32(pos[1]), _f32(pos[2]), _f32(np.full(n, r_list)), None,
                          UNIT_BOX, {"seed": seed, "r_list": r_list, "r_cut": r_cut, "eps": 1.0, "sigma": 0.9 * a,
                                     "coulomb": 4.0 * a, "spacing": a},
                          q=_f32(q))


# Named single-system workloads at their full sizes.
CONFIGS = {
    "uniform_32k": dict(kind="uniform_global", n=32768, seed=SEED_BASE + 1),
    "uniform_2m_varied": dict(kind="uniform_varied", n=2097152, seed=SEED_BASE + 2),
    "evrard_8m": dict(kind="evrard_sphere", n=8388608, seed=SEED_BASE + 3),
    "lj_4m": dict(kind="lj_lattice", n=160 ** 3, seed=SEED_BASE + 6),
}


def make(kind: str, n: int, seed: int, **kw) -> ParticleSystem:
    if kind == "lj_lattice":
        return lj_lattice(int(round(n ** (1.0 / 3.0))), seed, **kw)
    fn = {"uniform_global": uniform_global, "uniform_varied": uniform_varied,
          "evrard_sphere": evrard_sphere, "plummer": plummer}[kind]
    return fn(n, seed, **kw)


def make_config(name: str, n: int | None = None) -> ParticleSystem:
    c = dict(CONFIGS[name])
    kind = c.pop("kind")
    nn = c.pop("n") if n is None else (c.pop("n") and n)
    return make(kind, nn, c.pop("seed"))
