"""GPU parity of the polymer melts and the systems in vacuum: purely
repulsive LJ (the LJ kernel with rc = 2^(1/6), energy shifted), FENE bonds,
the cosine angle term of the ring melt (tables keyed by id or by index, the
one-pass bonded call), the Langevin thermostat in each of its placements
(own call, half kick, fused force call), the occupied-tile launch and the
two-stage tile sums, against the FP64 oracle (same Philox noise stream),
including the full-size sphere, slab, ring melt and replica batch."""
import numpy as np
import pytest

import md_inputs
import oracle

pytestmark = pytest.mark.gpu


def _system(cfg, langevin=None, **kw):
    from paper_2109_10876_amd import MDSystem
    return MDSystem(cfg.natoms, cfg.box, cfg.pos, cfg.vel, cfg.types, cfg.eps, cfg.sig,
                    cfg.mass, rc=cfg.rc, skin=cfg.skin, dt=cfg.dt, shift=cfg.shift,
                    bonds=cfg.bonds, angles=cfg.angles, langevin=langevin, **kw)


def test_langevin_noise_matches_oracle():
    import torch
    print("case: langevin noise", flush=True)
    cfg = md_inputs.lj_fluid(6, temperature=1.0, seed=3)
    s = _system(cfg, langevin=(0.5, 1.3, 12345, 77))
    s.setup()
    s.fx.zero_(); s.fy.zero_(); s.fz.zero_()
    s.noise_step.fill_(77)
    s.langevin()
    torch.cuda.synchronize()
    assert int(s.noise_step.item()) == 78
    got = s.forces_np()
    ref = oracle.langevin_forces(s.velocities(), np.arange(cfg.n), 0.5, 1.3, cfg.dt, 12345, 77)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_fene_and_wca_forces_match_oracle():
    print("case: fene + wca forces", flush=True)
    cfg = md_inputs.lattice_chains((8, 8, 10), 40, seed=4)
    cfg.pos = md_inputs.jitter(cfg.pos, 0.05, seed=9)
    s = _system(cfg)
    s.setup()
    s.ensure_list()
    f_lj, e_lj, w_lj = oracle.lj_forces(cfg.pos, cfg.box[0], cfg.rc, shift=1)
    f_b, e_b, w_b, broken = oracle.fene_forces(cfg.pos, cfg.box[0], cfg.bonds)
    assert broken == 0
    np.testing.assert_allclose(s.forces_np(), f_lj + f_b, rtol=0, atol=1e-9)
    assert float(s.energy[0]) == pytest.approx(e_lj, rel=1e-12)
    assert float(s.energy_bond[0]) == pytest.approx(e_b, rel=1e-12)
    assert float(s.virial_bond[0]) == pytest.approx(w_b, rel=1e-12)


def test_broken_bond_raises_the_flag():
    import torch
    from paper_2109_10876_amd import _abi as abi
    print("case: broken bond", flush=True)
    cfg = md_inputs.lattice_chains((6, 6, 10), 20, seed=4)
    cfg.pos = cfg.pos.copy()
    cfg.pos[1] = cfg.pos[0] + np.array([1.6, 0.0, 0.0])     # bond 0-1 beyond R0
    s = _system(cfg)
    s.sort(gated=False)
    s.build(gated=False)
    s.forces()
    s.fene()
    torch.cuda.synchronize()
    assert int(s.status.item()) & abi.MD_F_BOND_BROKEN


@pytest.mark.parametrize("mode", ["full", "tile"])
def test_melt_trajectory_with_thermostat_matches_oracle(mode):
    print(f"case: melt trajectory {mode}", flush=True)
    cfg = md_inputs.lattice_chains((8, 8, 10), 40, seed=6, temperature=1.0)
    steps = 60
    s = _system(cfg, langevin=(0.5, 1.0, 2024, 0), mode=mode)
    s.setup()
    flags, ep = [], []
    for t in range(steps):
        s.step_body(first=(t == 0))
        flags.append(int(s.gate[0].item()))
        ep.append(float(s.energy[0]) + float(s.energy_bond[0]))
    s.vv(2)
    assert s.ensure_list() == 0
    ref = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, cfg.dt, steps,
                            bonds=cfg.bonds, gamma=0.5, temperature=1.0, seed=2024, step0=0)
    assert ref["broken"] == 0
    assert flags == list(ref["rebuild"].astype(int))
    assert np.abs(s.positions() - ref["pos"]).max() < 1e-9
    assert np.abs(s.velocities() - ref["vel"]).max() < 1e-8
    np.testing.assert_allclose(ep, ref["epot"][1:], rtol=1e-10)
    assert float(s.ke[0]) == pytest.approx(ref["ekin"][-1], rel=1e-10)


def test_graphed_melt_matches_eager():
    print("case: melt graph vs eager", flush=True)
    cfg = md_inputs.lattice_chains((8, 8, 10), 40, seed=6, temperature=1.0)
    a = _system(cfg, langevin=(0.5, 1.0, 5, 0))
    a.setup()
    a.run(23, check_every=0)
    b = _system(cfg, langevin=(0.5, 1.0, 5, 0))
    b.setup()
    b.run_graphed(23, k=4)
    a.ensure_list()
    b.ensure_list()
    assert np.array_equal(a.positions(), b.positions())
    assert int(a.noise_step.item()) == int(b.noise_step.item()) == 24


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_slab_forces_sampled(prec):
    # LJ slab: FCC 20^3 x 4 at density 0.8 in the middle third of the box along z
    print(f"case: slab {prec}", flush=True)
    cfg = md_inputs.lj_slab(20, seed=8)
    cfg.pos = md_inputs.jitter(cfg.pos, 0.08, seed=10)
    s = _system(cfg, prec=prec)
    s.setup()
    s.ensure_list()
    f = s.forces_np()
    rng = np.random.default_rng(2)
    smp = rng.choice(cfg.n, 64, replace=False)
    planes = tuple(np.ascontiguousarray(cfg.pos[:, k]) for k in range(3))
    ref = np.array([oracle.lj_force_one(i, None, cfg.box[0], cfg.rc, planes=planes)[0]
                    for i in smp])
    err = np.linalg.norm(f[smp] - ref) / np.linalg.norm(ref)
    assert err < (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec,mode", [("fp64", "tile"), ("mixed", "tile"), ("fp64", "full")])
def test_sphere_forces_sampled(prec, mode):
    # LJ liquid sphere in vacuum (the paper's inhomogeneous case, scaled down):
    # ~1900 atoms at density 0.8442 in a 30 sigma box, most cells and tiles empty
    print(f"case: sphere {prec} {mode}", flush=True)
    cfg = md_inputs.lj_sphere(2000, 30.0, seed=9)
    cfg.pos = md_inputs.jitter(cfg.pos, 0.08, seed=11)
    s = _system(cfg, prec=prec, mode=mode)
    s.setup()
    assert s.ensure_list() == 0
    f = s.forces_np()
    rng = np.random.default_rng(3)
    smp = rng.choice(cfg.n, 64, replace=False)
    planes = tuple(np.ascontiguousarray(cfg.pos[:, k]) for k in range(3))
    ref = np.array([oracle.lj_force_one(i, None, cfg.box[0], cfg.rc, planes=planes)[0]
                    for i in smp])
    err = np.linalg.norm(f[smp] - ref) / np.linalg.norm(ref)
    assert err < (1e-12 if prec == "fp64" else 1e-5)
    # a surface atom has fewer neighbours than one in the bulk
    cnt = s.count.cpu().numpy()[np.argsort(s.id.cpu().numpy())]
    r = np.linalg.norm(cfg.pos - 15.0, axis=1)
    assert cnt[r > r.max() - 1.0].mean() < 0.8 * cnt[r < r.max() - 5.0].mean()


def _rings(shape, seed, jit=0.05):
    # rings of 32 on 2 x 4 x 4 blocks, jittered and moved by a random offset
    # so that rings cross the periodic faces
    cfg = md_inputs.lattice_rings(shape, block=(2, 4, 4), seed=seed)
    rng = np.random.default_rng(seed)
    cfg.pos = md_inputs.jitter(cfg.pos, jit, seed=seed + 1) + rng.uniform(0, 3.0, size=3)
    return cfg


@pytest.mark.parametrize("mode", ["full", "tile"])
def test_ring_melt_forces_match_oracle(mode):
    print(f"case: ring melt forces {mode}", flush=True)
    cfg = _rings((8, 8, 8), 21)
    s = _system(cfg, mode=mode)
    s.setup()
    assert s.ensure_list() == 0
    f_lj, e_lj, _ = oracle.lj_forces(cfg.pos, cfg.box[0], cfg.rc, shift=1)
    f_b, e_b, _, broken = oracle.fene_forces(cfg.pos, cfg.box[0], cfg.bonds)
    f_a, e_a, w_a, bad = oracle.angle_forces(cfg.pos, cfg.box[0], cfg.angles)
    assert broken == 0 and bad == 0
    np.testing.assert_allclose(s.forces_np(), f_lj + f_b + f_a, rtol=0, atol=1e-9)
    assert float(s.energy_angle[0]) == pytest.approx(e_a, rel=1e-12)
    assert abs(float(s.virial_angle[0])) < 1e-9 and abs(w_a) < 1e-9
    # the angle term alone, after zeroing the forces: each atom's own share
    s.fx.zero_(); s.fy.zero_(); s.fz.zero_()
    s.angle()
    np.testing.assert_allclose(s.forces_np(), f_a, rtol=0, atol=1e-12)


def test_degenerate_angle_raises_the_flag():
    import torch
    from paper_2109_10876_amd import _abi as abi
    print("case: degenerate angle", flush=True)
    cfg = md_inputs.lattice_rings((4, 8, 8), block=(2, 4, 4), seed=22)
    s = _system(cfg)
    s.sort(gated=False)
    s.status.zero_()
    s.angle()
    torch.cuda.synchronize()
    assert int(s.status.item()) == 0
    # put bead 1 on top of bead 0: the triples around them lose a bond vector
    cfg.pos = cfg.pos.copy()
    cfg.pos[1] = cfg.pos[0]
    s = _system(cfg)
    s.sort(gated=False)
    s.status.zero_()
    s.angle()
    torch.cuda.synchronize()
    assert int(s.status.item()) & abi.MD_F_NONFINITE


@pytest.mark.parametrize("mode", ["full", "tile"])
def test_ring_melt_trajectory_with_thermostat_matches_oracle(mode):
    print(f"case: ring melt trajectory {mode}", flush=True)
    cfg = _rings((8, 8, 8), 23, jit=0.02)
    steps = 60
    s = _system(cfg, langevin=(0.5, 1.0, 99, 0), mode=mode)
    s.setup()
    flags, ep = [], []
    for t in range(steps):
        s.step_body(first=(t == 0))
        flags.append(int(s.gate[0].item()))
        ep.append(float(s.energy[0]) + float(s.energy_bond[0]) + float(s.energy_angle[0]))
    s.vv(2)
    assert s.ensure_list() == 0
    ref = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, cfg.dt, steps,
                            bonds=cfg.bonds, angles=cfg.angles, gamma=0.5, temperature=1.0,
                            seed=99, step0=0)
    assert ref["broken"] == 0
    assert flags == list(ref["rebuild"].astype(int))
    assert np.abs(s.positions() - ref["pos"]).max() < 1e-9
    assert np.abs(s.velocities() - ref["vel"]).max() < 1e-8
    np.testing.assert_allclose(ep, ref["epot"][1:], rtol=1e-10)


def test_ring_melt_full_size_after_graphed_steps():
    # the 320,000-bead ring melt in the benchmark's form (tile lists, FP32
    # pair math, graphed steps with the thermostat): after 100 steps every
    # force on the current positions against the oracle
    import torch
    print("case: ring melt 320k", flush=True)
    cfg = md_inputs.CONFIGS["ring_melt"]()
    s = _system(cfg, langevin=(0.5, 1.0, 7), mode="tile", prec="mixed")
    s.setup()
    s.run_graphed(100, k=25)
    assert s.ensure_list() == 0
    s.forces()
    s.fene()
    s.angle()
    torch.cuda.synchronize()
    pos = s.positions()
    f_lj, _, _ = oracle.lj_forces(pos, cfg.box[0], cfg.rc, shift=1)
    f_b, _, _, broken = oracle.fene_forces(pos, cfg.box[0], cfg.bonds)
    f_a, e_a, _, bad = oracle.angle_forces(pos, cfg.box[0], cfg.angles)
    assert broken == 0 and bad == 0
    ref = f_lj + f_b + f_a
    got = s.forces_np()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5
    # the bonded terms are FP64 on both sides
    assert float(s.energy_angle[0]) == pytest.approx(e_a, rel=1e-11)


def test_bonded_tables_by_index_match_by_id():
    # tables re-keyed to the cell-sorted order after each re-sort give the
    # same per-atom sums in the same slot order: identical trajectories
    print("case: bonded tables by index vs by id", flush=True)
    cfg = _rings((8, 8, 8), 31)
    a = _system(cfg, langevin=(0.5, 1.0, 3, 0), bonded_order="index")
    b = _system(cfg, langevin=(0.5, 1.0, 3, 0), bonded_order="id")
    for s in (a, b):
        s.setup()
        s.run_graphed(40, k=8)
        assert s.ensure_list() == 0
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.forces_np(), b.forces_np())
    assert float(a.energy_angle[0]) == pytest.approx(float(b.energy_angle[0]), rel=1e-12)
    assert float(a.energy_bond[0]) == pytest.approx(float(b.energy_bond[0]), rel=1e-12)
    # the re-keyed tables name current indices: the partners of atom i are
    # the atoms whose ids the id-keyed table lists for id[i]
    ids = a.id.cpu().numpy()
    where = np.empty_like(ids)
    where[ids] = np.arange(ids.shape[0])
    bp = a.bond_partner.cpu().numpy()
    np.testing.assert_array_equal(a.bond_partner_ix.cpu().numpy(), where[bp[:, ids]])
    tri = a.angle_tri.cpu().numpy()
    np.testing.assert_array_equal(a.angle_tri_ix.cpu().numpy(), where[tri[:, ids]])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fused_step_with_thermostat_matches_oracle(prec):
    # pure LJ on tile lists with the Langevin thermostat: md_lj_forces_vv adds
    # the thermostat force inside the force kernel; the trajectory and the
    # rebuild schedule against the oracle's (same Philox noise)
    print(f"case: fused step with thermostat {prec}", flush=True)
    cfg = md_inputs.lj_fluid(8, temperature=1.0, seed=41)
    steps = 60 if prec == "fp64" else 20   # mixed: the short-horizon bar
    s = _system(cfg, langevin=(1.0, 0.85, 77, 5), mode="tile", prec=prec)
    assert s.fuse and s.thermo is not None
    s.setup()
    s.run(steps, check_every=0)
    assert s.ensure_list() == 0
    assert int(s.noise_step.item()) == 5 + 1 + steps
    ref = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, cfg.dt, steps,
                            gamma=1.0, temperature=0.85, seed=77, step0=5)
    tol = 1e-9 if prec == "fp64" else 1e-6
    assert np.abs(s.positions() - ref["pos"]).max() < tol
    assert np.abs(s.velocities() - ref["vel"]).max() < 10 * tol


def test_fused_step_with_thermostat_equals_split_calls_and_graphs():
    # the fused call (eager and graphed) against md_lj_forces + md_langevin +
    # md_vv_step: the same trajectory up to rounding of the thermostat sum
    import torch
    print("case: fused thermostat vs split, graphed", flush=True)
    cfg = md_inputs.lj_fluid(8, temperature=1.0, seed=42)
    lv = (0.7, 1.1, 99, 0)
    a = _system(cfg, langevin=lv, mode="tile", prec="fp64")
    b = _system(cfg, langevin=lv, mode="tile", prec="fp64", fuse=False)
    c = _system(cfg, langevin=lv, mode="tile", prec="fp64")
    assert a.fuse and not b.fuse
    for s in (a, b, c):
        s.setup()
    a.run(37, check_every=0)
    b.run(37, check_every=0)
    c.run_graphed(37, k=6)
    for s in (a, b, c):
        assert s.ensure_list() == 0
        assert int(s.noise_step.item()) == 38
    assert np.abs(a.positions() - b.positions()).max() < 1e-10
    assert np.abs(a.velocities() - b.velocities()).max() < 1e-9
    assert np.array_equal(a.positions(), c.positions())
    torch.cuda.synchronize()


def test_sums_over_many_tiles_of_one_replica():
    # a sparse droplet in a large box: one replica of more than 16384 tiles,
    # whose energy, virial, kinetic energy and gate are summed in two stages
    print("case: two-stage tile sums", flush=True)
    cfg = md_inputs.lj_sphere(20000, 120.0, seed=12)
    cfg.pos = md_inputs.jitter(cfg.pos, 0.05, seed=13)
    s = _system(cfg, prec="fp64", mode="tile", tile_rows=(1, 1), tile_cells=1)
    assert s.R == 1 and s.nlist.n_tiles >= 16384
    s.setup()
    assert s.ensure_list() == 0
    f_ref, e_ref, w_ref = oracle.lj_forces(cfg.pos, cfg.box[0], cfg.rc, shift=1)
    assert float(s.energy[0]) == pytest.approx(e_ref, rel=1e-10)
    assert float(s.virial[0]) == pytest.approx(w_ref, rel=1e-10)
    # the fused call's kinetic energy and gate against the split calls'
    b = _system(cfg, prec="fp64", mode="tile", tile_rows=(1, 1), tile_cells=1, fuse=False)
    b.setup()
    for x in (s, b):
        x.run(12, check_every=0)
        assert x.ensure_list() == 0
    assert np.array_equal(s.positions(), b.positions())
    assert float(s.ke[0]) == pytest.approx(float(b.ke[0]), rel=1e-12)
    assert float(s.energy[0]) == pytest.approx(float(b.energy[0]), rel=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_occupied_tile_list_on_a_droplet(prec):
    # a droplet in vacuum: the build lists the tiles that have home atoms and
    # the force kernels give workgroups to those only; forces, energies and a
    # thermostatted fused trajectory equal the every-tile launch bit for bit
    print(f"case: occupied-tile list {prec}", flush=True)
    cfg = md_inputs.lj_sphere(2000, 30.0, seed=9)
    cfg.pos = md_inputs.jitter(cfg.pos, 0.08, seed=11)
    a = _system(cfg, prec=prec, mode="tile", langevin=(1.0, 0.5, 21, 0))
    b = _system(cfg, prec=prec, mode="tile", langevin=(1.0, 0.5, 21, 0), sparse_tiles=False)
    assert a.sparse_tiles and not b.sparse_tiles and a.fuse and b.fuse
    for s in (a, b):
        s.setup()
        assert s.ensure_list() == 0
    # the list: the tiles with home atoms, ascending
    act = a.tile_active.cpu().numpy()
    occupied = [t for t, (home, _) in enumerate(a.tile_slot_table()) if len(home)]
    assert 0 < act[0] < a.n_tiles // 2
    assert list(act[1:1 + act[0]]) == occupied
    assert np.array_equal(a.forces_np(), b.forces_np())
    assert float(a.energy[0]) == pytest.approx(float(b.energy[0]), rel=1e-12)
    assert float(a.virial[0]) == pytest.approx(float(b.virial[0]), rel=1e-12)
    for s in (a, b):
        s.run_graphed(30, k=5)
        assert s.ensure_list() == 0
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.velocities(), b.velocities())
    assert float(a.ke[0]) == pytest.approx(float(b.ke[0]), rel=1e-12)


def _sampled_force_error(s, cfg, n_sample, seed, types=None):
    # forces on the current positions (thermostat excluded) against O(N)
    # oracle loops for sampled atoms of replica 0 .. R-1
    import torch
    s.forces()
    torch.cuda.synchronize()
    f = s.forces_np()
    pos = s.positions()
    off = cfg.atom_off()
    rng = np.random.default_rng(seed)
    got, ref = [], []
    for r in range(cfg.nrep):
        a, b = off[r], off[r + 1]
        planes = tuple(np.ascontiguousarray(pos[a:b, k]) for k in range(3))
        t = None if types is None else np.ascontiguousarray(types[a:b])
        for i in rng.choice(b - a, n_sample, replace=False):
            ref.append(oracle.lj_force_one(int(i), None, cfg.box[r], cfg.rc, cfg.eps, cfg.sig,
                                           t, shift=cfg.shift, planes=planes)[0])
            got.append(f[a + i])
    got, ref = np.array(got), np.array(ref)
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["lj_sphere", "lj_slab"])
def test_inhomogeneous_full_size_after_graphed_steps(name):
    # the paper's sphere (2.58 M atoms) and the slab (500,000) in the
    # benchmark's form: tile lists 3 x 2 x 2 with 2048 slots, the occupied-tile
    # launch, the thermostat fused into the force call, FP32-mixed, graphed
    print(f"case: {name} full size", flush=True)
    from paper_2109_10876_amd import _abi as abi
    lib = abi.load()
    lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, 2048)
    try:
        cfg = md_inputs.CONFIGS[name]()
        lang = {"lj_sphere": (1.0, 0.1, 6), "lj_slab": (1.0, 0.85, 4)}[name]
        s = _system(cfg, langevin=lang, mode="tile", prec="mixed", tile_rows=(2, 2),
                    tile_cells=3)
        assert s.sparse_tiles and s.fuse
        s.setup()
        s.run_graphed(50, k=25)
        assert s.ensure_list() == 0
        err = _sampled_force_error(s, cfg, 64, seed=5)
        print(f"  sampled e_F = {err:.3e}", flush=True)
        assert err < 1e-5
    finally:
        lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, 0)


def test_replica_batch_full_size_after_graphed_steps():
    # the 256 uneven two-type replicas (2.62 M atoms) in the benchmark's form:
    # typed tile lists of 2 x 2 rows with 2048 slots and each replica's own
    # width along x, FP32-mixed, graphed; sampled atoms of every replica
    # against the oracle
    print("case: replicas full size", flush=True)
    from paper_2109_10876_amd import _abi as abi
    lib = abi.load()
    lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, 2048)
    try:
        cfg = md_inputs.CONFIGS["replicas"]()
        s = _system(cfg, mode="tile", prec="mixed", tile_rows=(2, 2))
        assert s.nlist.tile_types == 2 and not s.sparse_tiles
        assert s.h_tile_m is not None and len(set(s.h_tile_m.tolist())) > 1
        s.setup()
        s.run_graphed(30, k=10)
        assert s.ensure_list() == 0
        err = _sampled_force_error(s, cfg, 2, seed=6, types=cfg.types)
        print(f"  sampled e_F = {err:.3e}", flush=True)
        assert err < 1e-5
    finally:
        lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, 0)


def test_replica_batch_adjoint_full_size_in_the_benchmarked_form():
    # the force-matching adjoint of the 256-replica batch as the benchmark
    # times it: typed tile lists with per-replica widths, FP32-mixed (the
    # upstream G staged in FP32, the pair term in FP32, FP64 sums), after
    # graphed steps; dL/dx of eight replicas of every tile width against the
    # oracle's adjoint of each replica alone, within the mixed bound 1e-5
    import torch
    print("case: replicas adjoint full size", flush=True)
    from paper_2109_10876_amd import _abi as abi
    lib = abi.load()
    lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, 2048)
    try:
        cfg = md_inputs.CONFIGS["replicas"]()
        s = _system(cfg, mode="tile", prec="mixed", tile_rows=(2, 2))
        s.setup()
        s.run_graphed(20, k=10)
        assert s.ensure_list() == 0
        rng = np.random.default_rng(8)
        G = rng.normal(size=(cfg.n, 3))
        gE = rng.normal(size=s.R)
        ids = s.id.cpu().numpy()
        d = s.dev
        gfx, gfy, gfz = (torch.tensor(G[ids, k].copy(), device=d) for k in range(3))
        gx = torch.zeros(3 * cfg.n, dtype=torch.float64, device=d)
        ge = torch.zeros(cfg.ntypes ** 2, dtype=torch.float64, device=d)
        gs = torch.zeros(cfg.ntypes ** 2, dtype=torch.float64, device=d)
        s.vjp(gfx, gfy, gfz, torch.tensor(gE, device=d), gx, ge, gs)
        torch.cuda.synchronize()
        got = np.empty((cfg.n, 3))
        got[ids] = gx.cpu().numpy().reshape(3, cfg.n).T
        pos = s.positions()
        off = cfg.atom_off()
        picks = []
        for m in sorted(set(s.h_tile_m.tolist())):
            picks += [int(r) for r in np.nonzero(s.h_tile_m == m)[0][:3]]
        for r in picks[:8]:
            a, b = off[r], off[r + 1]
            ref, _, _ = oracle.lj_vjp(pos[a:b], cfg.box[r], cfg.rc, G[a:b], float(gE[r]),
                                      cfg.eps, cfg.sig, cfg.types[a:b], shift=cfg.shift)
            err = np.linalg.norm(got[a:b] - ref) / np.linalg.norm(ref)
            print(f"  replica {r} width {s.h_tile_m[r]} N={b - a}: e = {err:.3e}", flush=True)
            assert err < 1e-5
    finally:
        lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, 0)


def test_bonded_forces_equal_the_separate_calls():
    # md_bonded_forces (FENE and angles in one pass) against md_fene_forces
    # then md_angle_forces on the same state: forces and energies bit for bit
    import torch
    print("case: combined bonded call", flush=True)
    cfg = _rings((8, 8, 8), 41, jit=0.05)
    s = _system(cfg)
    s.setup()
    s.run(20, check_every=0)
    assert s.ensure_list() == 0
    out = []
    for combined in (True, False):
        s.forces()
        if combined:
            s.bonded()
        else:
            s.fene()
            s.angle()
        torch.cuda.synchronize()
        out.append((s.forces_np(), float(s.energy_bond[0]), float(s.virial_bond[0]),
                    float(s.energy_angle[0]), float(s.virial_angle[0])))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1:] == out[1][1:]


def test_half_kick_with_thermostat_equals_langevin_then_half_kick():
    # md_vv_step with the thermostat against md_langevin followed by the plain
    # md_vv_step, from the same state and noise counter (phases 3 and 2)
    import torch
    print("case: half kick with thermostat", flush=True)
    cfg = md_inputs.lattice_chains((8, 8, 10), 40, seed=6, temperature=1.0)
    for phase in (3, 2):
        out = []
        for inside in (True, False):
            s = _system(cfg, langevin=(0.5, 1.2, 77, 3))
            assert s.vv_thermo
            s.setup()
            s.run(5, check_every=0)
            s.forces()
            s.fene()
            if inside:
                s.vv(phase)
            else:
                s.langevin()
                s.vv_thermo = False
                s.vv(phase)
            torch.cuda.synchronize()
            out.append((s.positions(), s.velocities(), s.forces_np(), float(s.ke[0]),
                        int(s.noise_step.item())))
        a, b = out
        assert a[4] == b[4]
        np.testing.assert_allclose(a[2], b[2], rtol=1e-14, atol=1e-12)
        np.testing.assert_allclose(a[1], b[1], rtol=1e-14, atol=1e-14)
        np.testing.assert_allclose(a[0], b[0], rtol=1e-15, atol=1e-14)
        assert a[3] == pytest.approx(b[3], rel=1e-14)


# ---------------------------------------------------- the melts as benchmarked
# The benchmark times both melts on global full lists with FP32 pair math and
# the thermostat force added by the half kick, replayed from captured graphs.
# Bounds: forces normwise 1e-5 (the mixed path's target); the WCA energy
# relative 1e-6; the bonded terms run in FP64 on both sides (1e-11).

MELT_LANGEVIN = {"kg_melt": (0.5, 1.0, 3), "ring_melt": (0.5, 1.0, 7)}


@pytest.mark.parametrize("name", ["kg_melt", "ring_melt"])
def test_melt_full_size_in_the_benchmarked_form(name):
    import torch
    from paper_2109_10876_amd import _abi as abi
    cfg = md_inputs.CONFIGS[name]()
    print(f"case: {name} N={cfg.n} full list, mixed, thermostat in the half kick, "
          f"50 graphed steps", flush=True)
    s = _system(cfg, langevin=MELT_LANGEVIN[name], mode="full", prec="mixed")
    assert s.mode == abi.MD_FULL and not s.fuse and s.vv_thermo
    s.setup()
    s.run_checked(50, k=24)
    assert s.ensure_list() == 0
    # every force on the current positions (LJ, then the bonded terms added)
    s.forces()
    if cfg.angles is not None:
        s.bonded()
    else:
        s.fene()
    torch.cuda.synchronize()
    pos = s.positions()
    f_lj, e_lj, _ = oracle.lj_forces(pos, cfg.box[0], cfg.rc, shift=1)
    f_b, e_b, w_b, broken = oracle.fene_forces(pos, cfg.box[0], cfg.bonds)
    ref = f_lj + f_b
    assert broken == 0
    if cfg.angles is not None:
        f_a, e_a, _, bad = oracle.angle_forces(pos, cfg.box[0], cfg.angles)
        assert bad == 0
        ref = ref + f_a
        assert float(s.energy_angle[0]) == pytest.approx(e_a, rel=1e-11)
    got = s.forces_np()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5
    assert float(s.energy[0]) == pytest.approx(e_lj, rel=1e-6)
    assert float(s.energy_bond[0]) == pytest.approx(e_b, rel=1e-11)
    assert float(s.virial_bond[0]) == pytest.approx(w_b, rel=1e-11)


@pytest.mark.parametrize("rings", [False, True])
def test_melt_mixed_trajectory_short_horizon(rings):
    # 20 thermostatted steps of a small melt in the benchmarked form against
    # the oracle's run with the same noise stream: the FP32 pair terms move
    # positions by ~1e-8 over this horizon, held to 1e-6
    cfg = _rings((8, 8, 8), 23, jit=0.02) if rings else \
        md_inputs.lattice_chains((8, 8, 10), 40, seed=6, temperature=1.0)
    print(f"case: melt mixed 20 steps rings={rings}", flush=True)
    s = _system(cfg, langevin=(0.5, 1.0, 41, 0), mode="full", prec="mixed")
    s.setup()
    s.run(20)
    assert s.ensure_list() == 0
    ref = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, cfg.dt, 20,
                            bonds=cfg.bonds, angles=cfg.angles, gamma=0.5, temperature=1.0,
                            seed=41, step0=0)
    assert ref["broken"] == 0
    assert np.abs(s.positions() - ref["pos"]).max() < 1e-6
    assert np.abs(s.velocities() - ref["vel"]).max() < 1e-5
    assert float(s.ke[0]) == pytest.approx(ref["ekin"][-1], rel=1e-6)
    # the potential energy the run leaves (evaluated by its tail)
    e_pot = float(s.energy[0]) + float(s.energy_bond[0]) + \
        (float(s.energy_angle[0]) if rings else 0.0)
    assert e_pot == pytest.approx(ref["epot"][-1], rel=1e-5)


def test_run_energies_are_those_of_the_final_state():
    # a run's repeated steps sum no energies; its tail evaluates them at the
    # final positions without touching the forces or the noise counter: the
    # potential and kinetic energy after 30 graphed FP64 steps equal the
    # oracle's, and the forces and counter equal those of step-by-step calls
    cfg = _rings((8, 8, 8), 23, jit=0.02)
    print("case: run energies of the final state", flush=True)
    a = _system(cfg, langevin=(0.5, 1.0, 57, 0), mode="full")
    a.setup()
    a.run_graphed(30, k=8)
    assert a.ensure_list() == 0
    ref = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, cfg.dt, 30,
                            bonds=cfg.bonds, angles=cfg.angles, gamma=0.5, temperature=1.0,
                            seed=57, step0=0)
    assert ref["broken"] == 0
    assert np.abs(a.positions() - ref["pos"]).max() < 1e-9
    e_pot = float(a.energy[0]) + float(a.energy_bond[0]) + float(a.energy_angle[0])
    assert e_pot == pytest.approx(ref["epot"][-1], rel=1e-10)
    assert float(a.ke[0]) == pytest.approx(ref["ekin"][-1], rel=1e-10)
    b = _system(cfg, langevin=(0.5, 1.0, 57, 0), mode="full")
    b.setup()
    for t in range(30):
        b.step_body(first=(t == 0))
    b.vv(2)
    assert np.array_equal(a.forces_np(), b.forces_np())
    assert int(a.noise_step[0].item()) == int(b.noise_step[0].item())
    assert float(a.energy[0]) == float(b.energy[0])
    assert float(a.energy_bond[0]) == float(b.energy_bond[0])
