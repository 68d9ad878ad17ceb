"""CPU checks of the synthetic workload generators (shapes, densities and
geometry of the inputs; no arithmetic of the method)."""
import math

import numpy as np
import pytest

import md_inputs


def test_sphere_geometry_and_density():
    # the inhomogeneous sphere (paper Sec. 4.2): FCC sites at rho within R of
    # the box centre, vacuum elsewhere
    cfg = md_inputs.lj_sphere(20000, 60.0, seed=3)
    rho = 0.8442
    R = (3.0 * 20000 / (4.0 * math.pi * rho)) ** (1.0 / 3.0)
    r = np.linalg.norm(cfg.pos - 30.0, axis=1)
    assert abs(cfg.n - 20000) < 0.02 * 20000
    assert r.max() < R and np.all(cfg.pos > 0.0) and np.all(cfg.pos < 60.0)
    inner = R - 3.0
    dens = np.count_nonzero(r < inner) / (4.0 / 3.0 * math.pi * inner ** 3)
    assert abs(dens - rho) < 0.03 * rho
    v = cfg.vel
    assert np.allclose(v.mean(axis=0), 0.0, atol=1e-12)
    assert abs(np.sum(v * v) / (3 * cfg.n - 3) - 0.1) < 1e-12


def test_sphere_workload_size():
    # the benchmark workload: 2.58 million atoms, 15.4% of a 271 sigma box
    cfg = md_inputs.CONFIGS["lj_sphere"]()
    assert cfg.n == 2580188 and cfg.box.tolist() == [[271.0, 271.0, 271.0]]
    frac = cfg.n / 0.8442 / 271.0 ** 3
    assert abs(frac - 0.154) < 0.002


def test_ring_melt_geometry():
    cfg = md_inputs.CONFIGS["ring_melt"]()
    a = (1.0 / 0.85) ** (1.0 / 3.0)
    assert cfg.n == 320_000 and cfg.bonds.shape == (320_000, 2)
    assert cfg.angles.shape == (320_000, 3)
    assert cfg.n / np.prod(cfg.box[0]) == pytest.approx(0.85, rel=1e-12)
    # every bond, the closing one included, is one lattice spacing long
    d = cfg.pos[cfg.bonds[:, 0]] - cfg.pos[cfg.bonds[:, 1]]
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), a, rtol=1e-12)
    # rings of 200: bead k of ring r bonds to bead k+1 mod 200 of the same ring
    ring = cfg.bonds // 200
    assert np.array_equal(ring[:, 0], ring[:, 1])
    assert np.array_equal(cfg.bonds[:, 1] % 200, (cfg.bonds[:, 0] % 200 + 1) % 200)
    # each bead is the middle of exactly one triple, between its two partners
    assert np.array_equal(np.sort(cfg.angles[:, 1]), np.arange(cfg.n))
    nxt = np.empty(cfg.n, np.int64)
    nxt[cfg.bonds[:, 0]] = cfg.bonds[:, 1]
    assert np.array_equal(cfg.angles[:, 2], nxt[cfg.angles[:, 1]])
    assert np.array_equal(nxt[cfg.angles[:, 0]], cfg.angles[:, 1])
    # one bead per lattice site
    sites = np.round(cfg.pos / a - 0.5).astype(np.int64)
    key = (sites[:, 0] * 80 + sites[:, 1]) * 50 + sites[:, 2]
    assert np.unique(key).shape[0] == cfg.n
