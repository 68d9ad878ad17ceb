"""Plain FP64 CPU oracle for short-range Lennard-Jones MD -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the GPU library and its binding)
never imports or calls it, and the two share no code: the arithmetic lives in
``orc.c`` (plain C, double precision, no fast-math), compiled with gcc into
``liborc.so`` and called here through ctypes with NumPy arrays.

Each wrapper cites the passage of arXiv 2109.10876 it follows (see the header
of ``orc.c``).  Arrays are per-atom ``[N,3]`` float64 positions/forces and
``[N]`` int32 types; ``box`` is the three edges of the orthorhombic periodic
box.

Parity pins of this oracle (closed forms, lattice shell counts, invariants,
brute force on tiny boxes, finite differences, generator known-answer
vectors) live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

_CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra"]


_LIB_OMP = os.path.join(_HERE, "liborc_omp.so")


def build(force=False, omp=False):
    """Compile orc.c into liborc.so with gcc (plain -O2, no fast-math).

    omp=True builds the timing-only liborc_omp.so instead (-fopenmp with
    ORC_OMP: the pair search and the pair force sum on all threads, per-pair
    arithmetic unchanged), used only for the all-core CPU baseline."""
    lib = _LIB_OMP if omp else _LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(_SRC):
        return lib
    tmp = lib + ".tmp"
    extra = ["-fopenmp", "-DORC_OMP"] if omp else []
    subprocess.run(["gcc", *_CFLAGS, *extra, _SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, lib)
    return lib


_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_U32 = ctypes.POINTER(ctypes.c_uint32)


_lib_omp = None


def _load(omp=False):
    global _lib, _lib_omp
    if omp:
        if _lib_omp is None:
            _lib_omp = _declare(ctypes.CDLL(build(omp=True)))
        return _lib_omp
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _declare(lib):
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.orc_min_image.restype = dbl
    lib.orc_min_image.argtypes = [dbl, dbl]
    lib.orc_lj_pair.restype = ctypes.c_int
    lib.orc_lj_pair.argtypes = [dbl, dbl, dbl, dbl, i32, _D, _D]
    for f in (lib.orc_pairs_brute, lib.orc_pairs_cells):
        f.restype = i64
        f.argtypes = [i32, _D, _D, _D, _D, dbl, _I, _I, i64]
    lib.orc_lj_forces_pairs.restype = None
    lib.orc_lj_forces_pairs.argtypes = [i32, _D, _D, _D, _I, i32, _D, _D, _D, dbl, i32,
                                        i64, _I, _I, _D, _D, _D, _D, _D]
    lib.orc_lj_forces_brute.restype = None
    lib.orc_lj_forces_brute.argtypes = [i32, _D, _D, _D, _I, i32, _D, _D, _D, dbl, i32,
                                        _D, _D, _D, _D, _D]
    lib.orc_lj_force_one.restype = None
    lib.orc_lj_force_one.argtypes = [i32, i32, _D, _D, _D, _I, i32, _D, _D, _D, dbl, i32,
                                     _D, _D, _D]
    lib.orc_lj_forces.restype = i64
    lib.orc_lj_forces.argtypes = [i32, _D, _D, _D, _I, i32, _D, _D, _D, dbl, i32,
                                  _D, _D, _D, _D, _D]
    lib.orc_lj_vjp_pairs.restype = None
    lib.orc_lj_vjp_pairs.argtypes = [i32, _D, _D, _D, _I, i32, _D, _D, _D, dbl, i32,
                                     i64, _I, _I, _D, _D, _D, dbl, _D, _D, _D, _D, _D]
    lib.orc_md_run.restype = i32
    lib.orc_md_run.argtypes = [i32, _D, _D, _D, _D, _D, _D, _I, i32, _D, _D, _D, _D,
                               dbl, i32, dbl, dbl, i32, _U8, _D, _D, _D, _D, _D, _D]
    lib.orc_philox4x32_10.restype = None
    lib.orc_philox4x32_10.argtypes = [_U32, _U32, _U32]
    lib.orc_gauss3.restype = None
    lib.orc_gauss3.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _D]
    lib.orc_langevin.restype = None
    lib.orc_langevin.argtypes = [i32, _D, _D, _D, _I, _D, _I, dbl, dbl, dbl,
                                 ctypes.c_uint64, ctypes.c_uint64, _D, _D, _D]
    lib.orc_fene_pair.restype = ctypes.c_int
    lib.orc_fene_pair.argtypes = [dbl, dbl, dbl, _D, _D]
    lib.orc_fene_forces.restype = i64
    lib.orc_fene_forces.argtypes = [i32, _D, _D, _D, _D, i64, _I, _I, dbl, dbl,
                                    _D, _D, _D, _D, _D]
    lib.orc_angle_triple.restype = ctypes.c_int
    lib.orc_angle_triple.argtypes = [_D, _D, dbl, _D, _D, _D]
    lib.orc_angle_forces.restype = i64
    lib.orc_angle_forces.argtypes = [i32, _D, _D, _D, _D, i64, _I, _I, _I, dbl,
                                     _D, _D, _D, _D, _D]
    lib.orc_md_run_ext.restype = i64
    lib.orc_md_run_ext.argtypes = [i32, _D, _D, _D, _D, _D, _D, _I, i32, _D, _D, _D, _D, dbl,
                                   i32, dbl, dbl, i32, i64, _I, _I, dbl, dbl, i64, _I, _I, _I,
                                   dbl, dbl, dbl, ctypes.c_uint64, ctypes.c_uint64, _U8, _D,
                                   _D, _D, _D, _D]
    return lib


def _d(a):
    return a.ctypes.data_as(_D)


def _i(a):
    return a.ctypes.data_as(_I) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _planes(pos):
    pos = _f64(pos)
    return (np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
            np.ascontiguousarray(pos[:, 2]))


def _tables(eps, sig):
    eps = _f64(np.atleast_2d(eps))
    sig = _f64(np.atleast_2d(sig))
    return eps.ravel().copy(), sig.ravel().copy(), int(eps.shape[0])


def _types(types, n):
    if types is None:
        return None
    t = np.ascontiguousarray(types, dtype=np.int32)
    assert t.shape == (n,)
    return t


# ------------------------------------------------------------------ wrappers

def min_image(d, L):
    """Minimum-image reduction d - L rint(d/L) (periodic box, Sec. 2.1.3)."""
    return _load().orc_min_image(float(d), float(L))


def lj_pair(r2, eps=1.0, sig=1.0, rc=2.5, shift=0):
    """Eq. lj at squared distance r2: returns (U, fr) with fr = -U'(r)/r;
    zero outside the cutoff; shift=1 lowers U by U(rc)."""
    u = ctypes.c_double()
    fr = ctypes.c_double()
    _load().orc_lj_pair(float(r2), float(eps), float(sig), float(rc), int(shift),
                        ctypes.byref(u), ctypes.byref(fr))
    return u.value, fr.value


def _pairs(fn, pos, box, rcut):
    lib = _load()
    x, y, z = _planes(pos)
    n = x.shape[0]
    L = _f64(box).ravel().copy()
    cap = max(64, n * 32)
    while True:
        pi = np.empty(cap, np.int32)
        pj = np.empty(cap, np.int32)
        cnt = getattr(lib, fn)(n, _d(x), _d(y), _d(z), _d(L), float(rcut), _i(pi), _i(pj), cap)
        if cnt < 0:
            raise ValueError(f"{fn}: box too small for rcut={rcut} (code {cnt})")
        if cnt <= cap:
            return np.stack([pi[:cnt], pj[:cnt]], axis=1)
        cap = int(cnt)


def pairs_brute(pos, box, rcut):
    """All unordered pairs (i<j) within rcut (minimum image), by testing every
    pair; [P,2] int32, lexicographic order."""
    return _pairs("orc_pairs_brute", pos, box, rcut)


def pairs_cells(pos, box, rcut):
    """Same pair set through the cell list with the 27-cell stencil
    (Sec. 2.1.2); identical output to pairs_brute."""
    return _pairs("orc_pairs_cells", pos, box, rcut)


def lj_forces_pairs(pos, box, pairs, rc, eps=1.0, sig=1.0, types=None, shift=1):
    """Forces [N,3], energy and virial from an explicit pair set (Eq. lj)."""
    lib = _load()
    x, y, z = _planes(pos)
    n = x.shape[0]
    e_t, s_t, nt = _tables(eps, sig)
    t = _types(types, n)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32)
    pi = np.ascontiguousarray(pairs[:, 0])
    pj = np.ascontiguousarray(pairs[:, 1])
    fx, fy, fz = (np.zeros(n) for _ in range(3))
    e = ctypes.c_double()
    w = ctypes.c_double()
    lib.orc_lj_forces_pairs(n, _d(x), _d(y), _d(z), _i(t), nt, _d(e_t), _d(s_t),
                            _d(_f64(box).ravel().copy()), float(rc), int(shift),
                            pairs.shape[0], _i(pi), _i(pj), _d(fx), _d(fy), _d(fz),
                            ctypes.byref(e), ctypes.byref(w))
    return np.stack([fx, fy, fz], axis=1), e.value, w.value


def lj_forces_brute(pos, box, rc, eps=1.0, sig=1.0, types=None, shift=1):
    """Forces by the O(N^2) definition: for each i, sum over all j != i."""
    lib = _load()
    x, y, z = _planes(pos)
    n = x.shape[0]
    e_t, s_t, nt = _tables(eps, sig)
    t = _types(types, n)
    fx, fy, fz = (np.zeros(n) for _ in range(3))
    e = ctypes.c_double()
    w = ctypes.c_double()
    lib.orc_lj_forces_brute(n, _d(x), _d(y), _d(z), _i(t), nt, _d(e_t), _d(s_t),
                            _d(_f64(box).ravel().copy()), float(rc), int(shift),
                            _d(fx), _d(fy), _d(fz), ctypes.byref(e), ctypes.byref(w))
    return np.stack([fx, fy, fz], axis=1), e.value, w.value


def lj_forces(pos, box, rc, eps=1.0, sig=1.0, types=None, shift=1):
    """Forces, energy, virial over the exact pair set inside rc (cell list)."""
    lib = _load()
    x, y, z = _planes(pos)
    n = x.shape[0]
    e_t, s_t, nt = _tables(eps, sig)
    t = _types(types, n)
    fx, fy, fz = (np.zeros(n) for _ in range(3))
    e = ctypes.c_double()
    w = ctypes.c_double()
    np_ = lib.orc_lj_forces(n, _d(x), _d(y), _d(z), _i(t), nt, _d(e_t), _d(s_t),
                            _d(_f64(box).ravel().copy()), float(rc), int(shift),
                            _d(fx), _d(fy), _d(fz), ctypes.byref(e), ctypes.byref(w))
    if np_ < 0:
        raise ValueError(f"orc_lj_forces failed ({np_})")
    return np.stack([fx, fy, fz], axis=1), e.value, w.value


def lj_force_one(i, pos, box, rc, eps=1.0, sig=1.0, types=None, shift=1, planes=None):
    """Force on atom i by an O(N) loop, plus i's half share of E and W."""
    lib = _load()
    x, y, z = planes if planes is not None else _planes(pos)
    n = x.shape[0]
    e_t, s_t, nt = _tables(eps, sig)
    t = _types(types, n)
    f = np.zeros(3)
    e = ctypes.c_double()
    w = ctypes.c_double()
    lib.orc_lj_force_one(int(i), n, _d(x), _d(y), _d(z), _i(t), nt, _d(e_t), _d(s_t),
                         _d(_f64(box).ravel().copy()), float(rc), int(shift), _d(f),
                         ctypes.byref(e), ctypes.byref(w))
    return f, e.value, w.value


def lj_vjp(pos, box, rc, G, gE, eps=1.0, sig=1.0, types=None, shift=1, pairs=None):
    """Vector-Jacobian product of (F, E) from Eq. lj: returns (gx[N,3],
    geps[nt,nt], gsig[nt,nt]) for upstream G = dL/dF [N,3] and gE = dL/dE."""
    lib = _load()
    if pairs is None:
        pairs = pairs_cells(pos, box, rc)
    x, y, z = _planes(pos)
    n = x.shape[0]
    e_t, s_t, nt = _tables(eps, sig)
    t = _types(types, n)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32)
    pi = np.ascontiguousarray(pairs[:, 0])
    pj = np.ascontiguousarray(pairs[:, 1])
    gfx, gfy, gfz = _planes(G)
    gx, gy, gz = (np.zeros(n) for _ in range(3))
    geps = np.zeros(nt * nt)
    gsig = np.zeros(nt * nt)
    lib.orc_lj_vjp_pairs(n, _d(x), _d(y), _d(z), _i(t), nt, _d(e_t), _d(s_t),
                         _d(_f64(box).ravel().copy()), float(rc), int(shift),
                         pairs.shape[0], _i(pi), _i(pj), _d(gfx), _d(gfy), _d(gfz),
                         float(gE), _d(gx), _d(gy), _d(gz), _d(geps), _d(gsig))
    return np.stack([gx, gy, gz], axis=1), geps.reshape(nt, nt), gsig.reshape(nt, nt)


def md_run(pos, vel, box, rc, skin, dt, steps, eps=1.0, sig=1.0, types=None,
           mass=None, shift=1, omp=False):
    """NVE velocity Verlet (Sec. 2.1, Fig. 1) with the skin rebuild test
    recorded per step.  Returns a dict with final unwrapped positions,
    velocities and forces, per-step rebuild flags and energy series.
    omp=True runs the timing-only all-thread build (CPU baseline only)."""
    lib = _load(omp)
    x, y, z = (p.copy() for p in _planes(pos))
    vx, vy, vz = (p.copy() for p in _planes(vel))
    n = x.shape[0]
    e_t, s_t, nt = _tables(eps, sig)
    t = _types(types, n)
    m = _f64(np.ones(nt) if mass is None else mass).ravel().copy()
    reb = np.zeros(max(steps, 1), np.uint8)
    ep, ek, vi = (np.zeros(steps + 1) for _ in range(3))
    fx, fy, fz = (np.zeros(n) for _ in range(3))
    rc_ = lib.orc_md_run(n, _d(x), _d(y), _d(z), _d(vx), _d(vy), _d(vz), _i(t), nt, _d(m),
                         _d(e_t), _d(s_t), _d(_f64(box).ravel().copy()), float(rc),
                         int(shift), float(skin), float(dt), int(steps),
                         reb.ctypes.data_as(_U8), _d(ep), _d(ek), _d(vi),
                         _d(fx), _d(fy), _d(fz))
    if rc_ != 0:
        raise ValueError(f"orc_md_run failed ({rc_})")
    return {
        "pos": np.stack([x, y, z], axis=1), "vel": np.stack([vx, vy, vz], axis=1),
        "force": np.stack([fx, fy, fz], axis=1), "rebuild": reb[:steps].astype(bool),
        "epot": ep, "ekin": ek, "virial": vi,
    }


def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC 2011): 4 words out."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    _load().orc_philox4x32_10(c.ctypes.data_as(_U32), k.ctypes.data_as(_U32),
                              out.ctypes.data_as(_U32))
    return out


def gauss3(seed, step, atom_id):
    """Three N(0,1) deviates for (seed, step, atom id) via Philox + Box-Muller."""
    g = np.zeros(3)
    _load().orc_gauss3(int(seed), int(step), int(atom_id), _d(g))
    return g


def langevin_forces(vel, ids, gamma, temperature, dt, seed, step, types=None,
                    mass=None, force=None):
    """Adds -gamma m v + sqrt(2 gamma m T/dt) xi to ``force`` (copied)."""
    lib = _load()
    vx, vy, vz = _planes(vel)
    n = vx.shape[0]
    t = _types(types, n)
    m = _f64(np.ones(1) if mass is None else mass).ravel().copy()
    f = np.zeros((n, 3)) if force is None else _f64(force)
    fx, fy, fz = (p.copy() for p in _planes(f))
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    lib.orc_langevin(n, _d(vx), _d(vy), _d(vz), _i(t), _d(m), _i(ids), float(gamma),
                     float(temperature), float(dt), int(seed), int(step),
                     _d(fx), _d(fy), _d(fz))
    return np.stack([fx, fy, fz], axis=1)


def fene_pair(r2, K=30.0, R0=1.5):
    """FENE bond at squared distance r2: (U, fr, intact)."""
    u = ctypes.c_double()
    fr = ctypes.c_double()
    ok = _load().orc_fene_pair(float(r2), float(K), float(R0), ctypes.byref(u),
                               ctypes.byref(fr))
    return u.value, fr.value, bool(ok)


def fene_forces(pos, box, bonds, K=30.0, R0=1.5):
    """FENE forces [N,3], energy, virial and broken-bond count for bonds
    given as atom-index pairs [Nb,2]."""
    lib = _load()
    x, y, z = _planes(pos)
    n = x.shape[0]
    bonds = np.ascontiguousarray(bonds, dtype=np.int32)
    bi = np.ascontiguousarray(bonds[:, 0])
    bj = np.ascontiguousarray(bonds[:, 1])
    fx, fy, fz = (np.zeros(n) for _ in range(3))
    e = ctypes.c_double(0.0)
    w = ctypes.c_double(0.0)
    broken = lib.orc_fene_forces(n, _d(x), _d(y), _d(z), _d(_f64(box).ravel().copy()),
                                 bonds.shape[0], _i(bi), _i(bj), float(K), float(R0),
                                 _d(fx), _d(fy), _d(fz), ctypes.byref(e), ctypes.byref(w))
    return np.stack([fx, fy, fz], axis=1), e.value, w.value, int(broken)


def angle_triple(d1, d2, K=1.5):
    """Cosine angle term of one triple from its two bond vectors d1 = x_a - x_b,
    d2 = x_c - x_b: (U, F_a, F_c, ok); F_b = -F_a - F_c."""
    d1 = _f64(d1).ravel().copy()
    d2 = _f64(d2).ravel().copy()
    fa, fc = np.zeros(3), np.zeros(3)
    u = ctypes.c_double()
    ok = _load().orc_angle_triple(_d(d1), _d(d2), float(K), ctypes.byref(u), _d(fa), _d(fc))
    return u.value, fa, fc, bool(ok)


def _triples(angles):
    angles = np.ascontiguousarray(np.asarray(angles).reshape(-1, 3), dtype=np.int32)
    return tuple(np.ascontiguousarray(angles[:, k]) for k in range(3))


def angle_forces(pos, box, angles, K=1.5):
    """Angle forces [N,3], energy, virial and degenerate-triple count for
    triples given as atom indices [Na,3] (middle bead in column 1)."""
    lib = _load()
    x, y, z = _planes(pos)
    n = x.shape[0]
    ia, ib, ic = _triples(angles)
    fx, fy, fz = (np.zeros(n) for _ in range(3))
    e = ctypes.c_double(0.0)
    w = ctypes.c_double(0.0)
    bad = lib.orc_angle_forces(n, _d(x), _d(y), _d(z), _d(_f64(box).ravel().copy()),
                               ia.shape[0], _i(ia), _i(ib), _i(ic), float(K),
                               _d(fx), _d(fy), _d(fz), ctypes.byref(e), ctypes.byref(w))
    return np.stack([fx, fy, fz], axis=1), e.value, w.value, int(bad)


def md_run_ext(pos, vel, box, rc, skin, dt, steps, eps=1.0, sig=1.0, types=None, mass=None,
               shift=1, bonds=None, K=30.0, R0=1.5, angles=None, Ka=1.5, gamma=0.0,
               temperature=1.0, seed=0, step0=0):
    """Velocity Verlet with LJ, optional FENE bonds ([Nb,2] atom indices),
    optional cosine angle terms ([Na,3] atom indices, middle bead in column 1)
    and optional Langevin thermostat (noise counter step0 for the initial
    forces, step0 + 1 + s for step s).  Returns final state, rebuild flags,
    energies and the number of broken-bond and degenerate-angle events."""
    lib = _load()
    x, y, z = (p.copy() for p in _planes(pos))
    vx, vy, vz = (p.copy() for p in _planes(vel))
    n = x.shape[0]
    e_t, s_t, nt = _tables(eps, sig)
    t = _types(types, n)
    m = _f64(np.ones(nt) if mass is None else mass).ravel().copy()
    if bonds is None:
        bonds = np.zeros((0, 2), np.int32)
    bonds = np.ascontiguousarray(bonds, dtype=np.int32)
    bi = np.ascontiguousarray(bonds[:, 0])
    bj = np.ascontiguousarray(bonds[:, 1])
    ia, ib, ic = _triples(np.zeros((0, 3), np.int32) if angles is None else angles)
    reb = np.zeros(max(steps, 1), np.uint8)
    ep, ek = np.zeros(steps + 1), np.zeros(steps + 1)
    fx, fy, fz = (np.zeros(n) for _ in range(3))
    r = lib.orc_md_run_ext(n, _d(x), _d(y), _d(z), _d(vx), _d(vy), _d(vz), _i(t), nt, _d(m),
                           _d(e_t), _d(s_t), _d(_f64(box).ravel().copy()), float(rc), int(shift),
                           float(skin), float(dt), int(steps), bonds.shape[0], _i(bi), _i(bj),
                           float(K), float(R0), ia.shape[0], _i(ia), _i(ib), _i(ic), float(Ka),
                           float(gamma), float(temperature), int(seed),
                           int(step0), reb.ctypes.data_as(_U8), _d(ep), _d(ek), _d(fx), _d(fy),
                           _d(fz))
    if r < 0:
        raise ValueError(f"orc_md_run_ext failed ({r})")
    return {
        "pos": np.stack([x, y, z], axis=1), "vel": np.stack([vx, vy, vz], axis=1),
        "force": np.stack([fx, fy, fz], axis=1), "rebuild": reb[:steps].astype(bool),
        "epot": ep, "ekin": ek, "broken": int(r),
    }
