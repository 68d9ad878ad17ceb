"""Seeded synthetic inputs for the short-range Lennard-Jones MD path.

This module only draws starting configurations (lattice sites, random
displacements, Maxwell velocities, random-walk chains, replica batches).  It
holds none of the method's arithmetic: no pair terms, no neighbour search and
no integration.  Both the FP64 oracle and the GPU library are fed from here,
so that the two sides see bit-identical inputs.

Workloads follow the paper's evaluation setup (Sec. 4, "Performance
evaluation"): LJ units with m = eps = sigma = 1, density 0.8442, cutoff 2.5,
skin 0.3, time step 0.005; a bead-spring polymer melt at density 0.85 with a
purely repulsive LJ cutoff 2^(1/6) and skin 0.4, with linear chains or, as
in the paper, rings of 200 beads.  The paper starts the LJ
fluid from a "cubic lattice"; the workloads here use the FCC lattice (four
sites per cubic unit cell), which is the usual reading for rho = 0.8442.

All random draws use NumPy's PCG64 through ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Config", "fcc_lattice", "maxwell_velocities", "jitter", "lj_fluid",
    "random_walk_chains", "lattice_chains", "ring_cycle", "lattice_rings", "lj_slab",
    "lj_sphere", "replica_batch", "retyped", "CONFIGS",
]

# Basis of the FCC conventional cubic cell, in units of the lattice constant.
_FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def fcc_lattice(m, rho, mz=None, my=None):
    """Perfect FCC crystal of m x my x mz cubic unit cells at number density rho.

    Returns (pos[N,3] float64, box[3] float64) with N = 4 m my mz; sites are
    ordered unit cell by unit cell (x fastest), four basis sites per cell.
    The lattice constant is a = (4/rho)^(1/3).
    """
    my = m if my is None else my
    mz = m if mz is None else mz
    a = (4.0 / rho) ** (1.0 / 3.0)
    iz, iy, ix = np.meshgrid(np.arange(mz), np.arange(my), np.arange(m),
                             indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pos = (cells[:, None, :] + _FCC_BASIS[None, :, :]).reshape(-1, 3) * a
    box = np.array([m * a, my * a, mz * a], dtype=np.float64)
    return pos, box


def maxwell_velocities(n, temperature, mass=1.0, seed=0):
    """Gaussian velocities N(0, sqrt(T/m)) per component, zero total momentum,
    rescaled so that sum m v^2 = (3n - 3) T exactly (3n - 3 degrees of freedom).
    """
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, math.sqrt(temperature / mass), size=(n, 3))
    v -= v.mean(axis=0, keepdims=True)
    s2 = mass * float(np.sum(v * v))
    if n > 1 and s2 > 0.0:
        v *= math.sqrt((3 * n - 3) * temperature / s2)
    return v


def jitter(pos, amplitude, seed=0):
    """Uniform random displacement in [-amplitude, amplitude] per component."""
    rng = np.random.default_rng(seed)
    return pos + rng.uniform(-amplitude, amplitude, size=pos.shape)


@dataclasses.dataclass
class Config:
    """One synthetic workload (possibly many replicas).

    pos, vel: [N,3] float64, replicas concatenated; box: [R,3];
    natoms: [R] atoms per replica; types: [N] int32 in [0, ntypes);
    eps, sig: [ntypes, ntypes] symmetric tables; mass: [ntypes].
    bonds: optional [Nb,2] int32 pairs of atom ids (global numbering).
    """
    name: str
    pos: np.ndarray
    vel: np.ndarray
    box: np.ndarray
    natoms: np.ndarray
    types: np.ndarray
    ntypes: int
    eps: np.ndarray
    sig: np.ndarray
    mass: np.ndarray
    rc: float
    skin: float
    dt: float
    temperature: float
    steps: int
    shift: int = 1
    bonds: np.ndarray | None = None
    angles: np.ndarray | None = None

    @property
    def n(self):
        return int(self.pos.shape[0])

    @property
    def nrep(self):
        return int(self.natoms.shape[0])

    def atom_off(self):
        return np.concatenate([[0], np.cumsum(self.natoms)]).astype(np.int64)


def lj_fluid(m, rho=0.8442, temperature=0.72, seed=1, rc=2.5, skin=0.3,
             dt=0.005, steps=100, jitter_amp=0.0, name=None):
    """Single-type LJ fluid started from an FCC crystal of m^3 unit cells.

    m = 10 gives the 4000-atom parity workload; m = 64 gives 1,048,576 atoms.
    ``jitter_amp`` > 0 displaces sites uniformly (used to get non-zero
    forces on a snapshot without running any dynamics).
    """
    pos, box = fcc_lattice(m, rho)
    if jitter_amp > 0.0:
        pos = jitter(pos, jitter_amp, seed=seed + 1000)
    n = pos.shape[0]
    vel = maxwell_velocities(n, temperature, 1.0, seed=seed)
    one = np.ones((1, 1))
    return Config(name or f"lj_fcc{m}", pos, vel, box[None, :].copy(),
                  np.array([n], dtype=np.int64), np.zeros(n, np.int32), 1,
                  one.copy(), one.copy(), np.ones(1), rc, skin, dt,
                  temperature, steps)


def random_walk_chains(nchains, length, rho=0.85, bond=0.97, seed=3,
                       temperature=1.0, dt=0.005, steps=1000):
    """Linear bead-spring chains grown as random walks with fixed step length.

    Chain starts are uniform in a cubic box sized for density rho; each next
    bead sits at distance ``bond`` in a uniformly random direction.  Beads
    may overlap: an untimed force-capped warm-up is needed before dynamics.
    Positions are returned unwrapped (the library wraps them).
    """
    rng = np.random.default_rng(seed)
    n = nchains * length
    L = (n / rho) ** (1.0 / 3.0)
    start = rng.uniform(0.0, L, size=(nchains, 1, 3))
    d = rng.normal(size=(nchains, length - 1, 3))
    d *= bond / np.linalg.norm(d, axis=2, keepdims=True)
    pos = np.concatenate([start, start + np.cumsum(d, axis=1)], axis=1).reshape(n, 3)
    vel = maxwell_velocities(n, temperature, 1.0, seed=seed + 1)
    first = (np.arange(nchains)[:, None] * length + np.arange(length - 1)[None, :]).ravel()
    bonds = np.stack([first, first + 1], axis=1).astype(np.int32)
    one = np.ones((1, 1))
    wca = 2.0 ** (1.0 / 6.0)
    return Config(f"kg_melt_{nchains}x{length}", pos, vel,
                  np.array([[L, L, L]]), np.array([n], dtype=np.int64),
                  np.zeros(n, np.int32), 1, one.copy(), one.copy(), np.ones(1),
                  wca, 0.4, dt, temperature, steps, shift=1, bonds=bonds)


def lattice_chains(shape, length, rho=0.85, seed=3, temperature=1.0, dt=0.005,
                   steps=1000):
    """Linear chains laid along a serpentine (boustrophedon) path through a
    simple-cubic lattice of shape (mx, my, mz) with spacing (1/rho)^(1/3):
    consecutive path sites are lattice neighbours, so every bond has the
    lattice spacing and no two beads overlap (no warm-up needed).  The path
    is cut into chains of ``length`` beads (mx my mz must be a multiple)."""
    mx, my, mz = shape
    n = mx * my * mz
    assert n % length == 0
    a = (1.0 / rho) ** (1.0 / 3.0)
    sites = []
    for z in range(mz):
        ys = range(my) if z % 2 == 0 else range(my - 1, -1, -1)
        for k, y in enumerate(ys):
            row = (z * my + k) % 2 == 0
            xs = range(mx) if row else range(mx - 1, -1, -1)
            sites.extend((x, y, z) for x in xs)
    pos = (np.array(sites, dtype=np.float64) + 0.5) * a
    vel = maxwell_velocities(n, temperature, 1.0, seed=seed)
    nch = n // length
    first = (np.arange(nch)[:, None] * length + np.arange(length - 1)[None, :]).ravel()
    bonds = np.stack([first, first + 1], axis=1).astype(np.int32)
    one = np.ones((1, 1))
    return Config(f"kg_lattice_{nch}x{length}", pos, vel,
                  np.array([[mx * a, my * a, mz * a]]), np.array([n], dtype=np.int64),
                  np.zeros(n, np.int32), 1, one.copy(), one.copy(), np.ones(1),
                  2.0 ** (1.0 / 6.0), 0.4, dt, temperature, steps, shift=1, bonds=bonds)


def ring_cycle(ny, nz):
    """A closed path through the 2 x ny x nz block of lattice sites (x, y, z)
    that steps between lattice neighbours only (ny even): a boustrophedon over
    the (y, z) layer at x = 0 from (0, 0, 0) to (0, 0, nz - 1) (rows along y,
    one row per z), then the same path backwards in the layer x = 1, which
    ends next to the start."""
    assert nz % 2 == 0
    layer = []
    for z in range(nz):
        ys = range(ny) if z % 2 == 0 else range(ny - 1, -1, -1)
        layer.extend((y, z) for y in ys)
    return [(0, y, z) for y, z in layer] + [(1, y, z) for y, z in reversed(layer)]


def lattice_rings(shape, block=(2, 10, 10), rho=0.85, seed=7, temperature=1.0, dt=0.005,
                  steps=1000):
    """Ring polymers on a simple-cubic lattice of shape (mx, my, mz) with
    spacing (1/rho)^(1/3): the lattice is cut into blocks of 2 x by x bz
    sites and each block holds one ring along ``ring_cycle`` (2 by bz beads,
    every bond one lattice spacing, no two beads overlapping).  Returns the
    ring bonds (closing bond included) and one angle triple per bead with the
    bead in the middle."""
    mx, my, mz = shape
    bx, by, bz = block
    assert bx == 2 and mx % bx == 0 and my % by == 0 and mz % bz == 0
    cyc = np.array(ring_cycle(by, bz), dtype=np.int64)
    length = cyc.shape[0]
    a = (1.0 / rho) ** (1.0 / 3.0)
    corners = np.stack(np.meshgrid(np.arange(0, mx, bx), np.arange(0, my, by),
                                   np.arange(0, mz, bz), indexing="ij"), axis=-1).reshape(-1, 3)
    sites = (corners[:, None, :] + cyc[None, :, :]).reshape(-1, 3)
    n = sites.shape[0]
    pos = (sites.astype(np.float64) + 0.5) * a
    vel = maxwell_velocities(n, temperature, 1.0, seed=seed)
    nring = corners.shape[0]
    k = np.arange(length)
    base = (np.arange(nring) * length)[:, None]
    me = (base + k[None, :]).ravel()
    nxt = (base + (k[None, :] + 1) % length).ravel()
    prv = (base + (k[None, :] - 1) % length).ravel()
    bonds = np.stack([me, nxt], axis=1).astype(np.int32)
    angles = np.stack([prv, me, nxt], axis=1).astype(np.int32)
    one = np.ones((1, 1))
    return Config(f"ring_melt_{nring}x{length}", pos, vel,
                  np.array([[mx * a, my * a, mz * a]]), np.array([n], dtype=np.int64),
                  np.zeros(n, np.int32), 1, one.copy(), one.copy(), np.ones(1),
                  2.0 ** (1.0 / 6.0), 0.4, dt, temperature, steps, shift=1, bonds=bonds,
                  angles=angles)


def lj_slab(m=50, rho=0.8, temperature=0.85, seed=4, dt=0.005, steps=1000):
    """FCC slab of m^3 unit cells at density rho, centred in z in a box whose
    z edge is three times the slab thickness (vacuum on both sides)."""
    pos, box = fcc_lattice(m, rho)
    L = box[0]
    pos = pos.copy()
    pos[:, 2] += L  # middle third of [0, 3L)
    n = pos.shape[0]
    vel = maxwell_velocities(n, temperature, 1.0, seed=seed)
    one = np.ones((1, 1))
    return Config(f"lj_slab{m}", pos, vel, np.array([[L, L, 3.0 * L]]),
                  np.array([n], dtype=np.int64), np.zeros(n, np.int32), 1,
                  one.copy(), one.copy(), np.ones(1), 2.5, 0.3, dt,
                  temperature, steps)


def lj_sphere(n_target=2_580_000, box=271.0, rho=0.8442, temperature=0.1, seed=6, dt=0.005,
              steps=100):
    """LJ liquid filling a sphere at the centre of a cubic box, vacuum around
    it (the paper's spatially inhomogeneous case, Sec. 4.2): FCC sites at
    density rho within radius R = (3 n_target / (4 pi rho))^(1/3) of the box
    centre, so N is n_target up to the lattice's discreteness."""
    R = (3.0 * n_target / (4.0 * math.pi * rho)) ** (1.0 / 3.0)
    a = (4.0 / rho) ** (1.0 / 3.0)
    m = int(math.ceil(2.0 * R / a)) + 1
    sites, _ = fcc_lattice(m, rho)
    sites = sites - 0.5 * m * a          # lattice centred on the origin
    keep = np.einsum("ij,ij->i", sites, sites) < R * R
    pos = np.ascontiguousarray(sites[keep] + 0.5 * box)
    n = pos.shape[0]
    vel = maxwell_velocities(n, temperature, 1.0, seed=seed)
    one = np.ones((1, 1))
    return Config(f"lj_sphere{n}", pos, vel, np.array([[box, box, box]]),
                  np.array([n], dtype=np.int64), np.zeros(n, np.int32), 1,
                  one.copy(), one.copy(), np.ones(1), 2.5, 0.3, dt,
                  temperature, steps)


def replica_batch(nrep=256, nmin=500, nmax=20000, rho=0.8442, temperature=1.0,
                  seed=5, param_seed=None, dt=0.005, steps=100):
    """Independent two-type LJ replicas of uneven sizes.

    Sizes are uniform integers in [nmin, nmax].  Replica r is a random subset
    of n_r sites of an FCC lattice of m = ceil((n_r/4)^(1/3)) unit cells scaled
    to the cubic box of edge (n_r/rho)^(1/3).  Types are 0/1 with probability
    1/2; one symmetric 2x2 (eps, sigma) table shared by all replicas has
    entries uniform in [0.8, 1.2].
    """
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=nrep)
    pos_l, vel_l, box_l, typ_l = [], [], [], []
    for r, nr in enumerate(sizes):
        nr = int(nr)
        m = int(math.ceil((nr / 4.0) ** (1.0 / 3.0) - 1e-12))
        L = (nr / rho) ** (1.0 / 3.0)
        sites, _ = fcc_lattice(m, 4.0 / 1.0)  # unit lattice constant
        sites = sites * (L / m)
        pick = np.sort(rng.choice(sites.shape[0], size=nr, replace=False))
        pos_l.append(sites[pick])
        vel_l.append(maxwell_velocities(nr, temperature, 1.0,
                                        seed=seed * 100003 + r))
        box_l.append([L, L, L])
        typ_l.append(rng.integers(0, 2, size=nr).astype(np.int32))
    prng = np.random.default_rng(seed + 7 if param_seed is None else param_seed)
    eps = np.empty((2, 2))
    sig = np.empty((2, 2))
    e = prng.uniform(0.8, 1.2, size=3)
    s = prng.uniform(0.8, 1.2, size=3)
    eps[0, 0], eps[1, 1], eps[0, 1] = e
    sig[0, 0], sig[1, 1], sig[0, 1] = s
    eps[1, 0] = eps[0, 1]
    sig[1, 0] = sig[0, 1]
    return Config(f"replicas{nrep}", np.concatenate(pos_l), np.concatenate(vel_l),
                  np.array(box_l, dtype=np.float64), sizes.astype(np.int64),
                  np.concatenate(typ_l), 2, eps, sig, np.ones(2), 2.5, 0.3, dt,
                  temperature, steps)


def retyped(cfg, ntypes, seed=0):
    """The same configuration with atom types drawn uniformly from
    [0, ntypes) and one symmetric (eps, sigma) table with entries uniform in
    [0.8, 1.2]."""
    rng = np.random.default_rng(seed)
    types = rng.integers(0, ntypes, size=cfg.n).astype(np.int32)
    eps = rng.uniform(0.8, 1.2, size=(ntypes, ntypes))
    sig = rng.uniform(0.8, 1.2, size=(ntypes, ntypes))
    eps = np.triu(eps) + np.triu(eps, 1).T
    sig = np.triu(sig) + np.triu(sig, 1).T
    return dataclasses.replace(cfg, name=f"{cfg.name}_t{ntypes}", types=types, ntypes=ntypes,
                               eps=eps, sig=sig, mass=np.ones(ntypes))


# The five workloads, by name.  Each entry builds its Config on demand.
CONFIGS = {
    "lj4000": lambda: lj_fluid(10, temperature=0.72, seed=1, steps=100,
                               name="lj_fcc10_n4000"),
    "lj1m": lambda: lj_fluid(64, temperature=1.0, seed=2, steps=1000,
                             name="lj_fcc64_n1048576"),
    "kg_melt": lambda: lattice_chains((80, 80, 128), 200, seed=3),
    "kg_melt_random_walk": lambda: random_walk_chains(4096, 200, seed=3),
    "ring_melt": lambda: lattice_rings((80, 80, 50), seed=7),
    "lj_slab": lambda: lj_slab(50, seed=4),
    "lj_sphere": lambda: lj_sphere(seed=6),
    "replicas": lambda: replica_batch(256, seed=5),
}
