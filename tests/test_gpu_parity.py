"""GPU parity: libmd (through its C ABI) against the FP64 oracle.

Tolerances (derivations):
  FP64 path -- same arithmetic, different summation order and a reciprocal
    refined by Newton steps: per-atom force error ~ (terms) x (largest term)
    x 2^-53 ~ 50 x 200 x 1.1e-16 ~ 1e-12; bound 1e-10 absolute, 1e-12
    normwise; energy/virial relative 1e-12 for the 4000-atom cases.  For a
    replica of N_r atoms the energy sums P ~ 27 N_r pair terms of mixed
    sign in a different order on each side: the recursive-summation bound
    P x 2^-53 x sum|U| with sum|U| ~ 2|E| gives ~3e-11 relative at
    N_r = 6000, so larger replicas are held to 1e-10.
  FP32-mixed path -- single-precision reciprocal (1 ulp) and LJ polynomial:
    relative pair-force error ~ 10 x 2^-24 ~ 6e-7, partly cancelling in the
    sum; the required bound is the target's 1e-5 normwise relative force
    error; energy and virial relative 1e-6 where the total is large.  Each
    atom sums its ~40 pair energies (each below ~10 in size) in single
    precision: at most ~40 x 10 x 2^-24 ~ 2.4e-5 per atom, so for replicas
    whose total energy nearly cancels the bound is |dE| <= 1e-5 N_r.
  Integer work (pair sets, counts, rebuild schedule): exact.
"""
import dataclasses

import numpy as np
import pytest

import md_inputs
import oracle

pytestmark = pytest.mark.gpu

RC, SKIN = 2.5, 0.3


def say(msg):
    print(msg, flush=True)


def _system(cfg, **kw):
    from paper_2109_10876_amd import MDSystem
    return MDSystem(cfg.natoms, cfg.box, cfg.pos, cfg.vel, cfg.types, cfg.eps, cfg.sig,
                    cfg.mass, rc=cfg.rc, skin=cfg.skin, dt=cfg.dt, shift=cfg.shift, **kw)


def _err(f, ref):
    return np.linalg.norm(f - ref) / np.linalg.norm(ref)


@pytest.fixture(scope="module")
def c1_snapshot():
    # 4000-atom LJ fluid (FCC 10^3 x 4, rho 0.8442), sites jittered so forces are non-zero
    return md_inputs.lj_fluid(10, temperature=0.72, seed=1, jitter_amp=0.1)


@pytest.mark.parametrize("mode,rows", [("full", None), ("half", None), ("tile", (1, 1)),
                                       ("tile", (2, 1)), ("tile", (2, 2))])
def test_forces_fp64_match_oracle(c1_snapshot, mode, rows):
    cfg = c1_snapshot
    say(f"case: forces fp64 {mode} {rows} N={cfg.n}")
    s = _system(cfg, mode=mode, prec="fp64", **({"tile_rows": rows} if rows else {}))
    s.setup()
    assert s.ensure_list() == 0
    f = s.forces_np()
    ref, e, w = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
    assert np.abs(f - ref).max() < 1e-10
    assert _err(f, ref) < 1e-12
    assert float(s.energy[0]) == pytest.approx(e, rel=1e-12)
    assert float(s.virial[0]) == pytest.approx(w, rel=1e-12)


@pytest.mark.parametrize("mode", ["full", "half", "tile"])
def test_forces_mixed_within_bound(c1_snapshot, mode):
    cfg = c1_snapshot
    say(f"case: forces mixed {mode} N={cfg.n}")
    s = _system(cfg, mode=mode, prec="mixed")
    s.setup()
    f = s.forces_np()
    ref, e, w = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
    err = _err(f, ref)
    say(f"  mixed e_F = {err:.3e}")
    assert err < 1e-5
    assert float(s.energy[0]) == pytest.approx(e, rel=1e-6)
    assert float(s.virial[0]) == pytest.approx(w, rel=1e-6)


@pytest.mark.parametrize("prec,ntypes", [("mixed", 1), ("mixed", 2), ("mixed", 3),
                                          ("fp64", 1)])
def test_cutoff_at_rc_is_decided_as_in_double(prec, ntypes):
    # simple cubic lattice of spacing rc/2: every axis pair sits at rc, moved
    # by a jitter of 1e-9 to either side.  The single-precision path's
    # displacements carry rounding of order 1e-8, and a pair put on the wrong
    # side of rc moves two forces by |F(rc)| (above 0.008 for every type pair
    # here); decided as in double, the forces match the oracle's to the
    # single-precision rounding of the pair terms (~1e-4 at most).
    k = 20
    g = (np.arange(k) + 0.25) * (RC / 2)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = md_inputs.jitter(pos, 1e-9, seed=13)
    n = pos.shape[0]
    cfg = dataclasses.replace(md_inputs.lj_fluid(10), pos=pos, vel=np.zeros_like(pos),
                              box=np.full((1, 3), k * RC / 2), natoms=np.array([n]),
                              types=np.zeros(n, np.int32))
    if ntypes > 1:
        cfg = md_inputs.retyped(cfg, ntypes, seed=31)
    say(f"case: cutoff at rc {prec} ntypes={ntypes}")
    s = _system(cfg, mode="tile", prec=prec)
    s.setup()
    assert s.ensure_list() == 0
    f = s.forces_np()
    ref, _, _ = oracle.lj_forces(cfg.pos, cfg.box[0], RC, cfg.eps, cfg.sig, cfg.types, shift=1)
    # the axis pairs inside rc leave net forces of order |F(rc)|
    assert np.abs(ref).max() > 0.008
    assert np.abs(f - ref).max() < (1e-3 if prec == "mixed" else 1e-10)


def test_full_list_forces_are_deterministic_and_match_half(c1_snapshot):
    cfg = c1_snapshot
    say("case: determinism full vs half")
    a = _system(cfg, mode="full")
    a.setup()
    b = _system(cfg, mode="full")
    b.setup()
    assert np.array_equal(a.forces_np(), b.forces_np())
    h = _system(cfg, mode="half")
    h.setup()
    assert np.abs(h.forces_np() - a.forces_np()).max() < 1e-10


@pytest.mark.parametrize("mode", ["full", "half"])
def test_pair_batch_and_gather_source_do_not_change_results(c1_snapshot, mode):
    from paper_2109_10876_amd import _abi as abi
    cfg = c1_snapshot
    say(f"case: batch/gather variants {mode}")
    lib = abi.load()
    ref = None
    try:
        for p4 in (True, False):
            s = _system(cfg, mode=mode, pos4=p4)
            s.setup()
            for batch in (1, 2, 4, 8):
                assert lib.md_tune_set(abi.MD_TUNE_PAIR_BATCH, batch) == 0
                s.forces()
                f = s.forces_np()
                if ref is None:
                    ref = f
                elif mode == "full":
                    assert np.array_equal(f, ref)       # same summation order
                else:
                    assert np.abs(f - ref).max() < 1e-10
    finally:
        lib.md_tune_set(abi.MD_TUNE_PAIR_BATCH, 4)


def _unordered(pairs):
    p = np.sort(pairs, axis=1)
    return set(map(tuple, np.unique(p, axis=0)))


@pytest.mark.parametrize("mode,rows", [("full", None), ("half", None), ("tile", (1, 1)),
                                       ("tile", (2, 2))])
def test_verlet_list_is_the_skin_pair_set(c1_snapshot, mode, rows):
    cfg = c1_snapshot
    say(f"case: list set {mode} {rows}")
    s = _system(cfg, mode=mode, **({"tile_rows": rows} if rows else {}))
    s.setup()
    pairs, codes = s.list_pairs()
    # each unordered pair exactly twice (full) or once (half)
    p = np.sort(pairs, axis=1)
    _, mult = np.unique(p, axis=0, return_counts=True)
    assert np.all(mult == (1 if mode == "half" else 2))
    got = _unordered(pairs)
    rl = RC + SKIN
    ref = oracle.pairs_cells(cfg.pos, cfg.box[0], rl)
    exp = set(map(tuple, ref))
    # the set is unique up to pairs within rounding of the Verlet radius
    diff = got.symmetric_difference(exp)
    for i, j in diff:
        d = cfg.pos[i] - cfg.pos[j]
        d -= cfg.box[0] * np.rint(d / cfg.box[0])
        assert abs(np.dot(d, d) - rl * rl) < 1e-10
    assert len(diff) <= 2


@pytest.mark.parametrize("mode,rows", [("full", None), ("half", None), ("tile", (1, 1)),
                                       ("tile", (2, 2))])
def test_pairs_at_the_verlet_radius_are_decided_in_fp64(mode, rows):
    # simple cubic lattice of spacing rl/2: every axis pair sits at rl, moved by
    # a jitter of 1e-7 to either side, far inside a single-precision distance
    # test's rounding and far outside double precision's
    rl = RC + SKIN
    k = 20
    g = (np.arange(k) + 0.25) * (rl / 2)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = md_inputs.jitter(pos, 1e-7, seed=11)
    cfg = md_inputs.lj_fluid(10)
    n = pos.shape[0]
    cfg = dataclasses.replace(cfg, pos=pos, vel=np.zeros_like(pos),
                              box=np.full((1, 3), k * rl / 2), natoms=np.array([n]),
                              types=np.zeros(n, np.int32))
    say(f"case: pairs at the Verlet radius {mode} {rows}")
    s = _system(cfg, mode=mode, **({"tile_rows": rows} if rows else {}))
    s.setup()
    pairs, _ = s.list_pairs()
    exp = set(map(tuple, oracle.pairs_cells(cfg.pos, cfg.box[0], rl)))
    # 26 lattice neighbours inside rl per atom, and about half of the six on it
    assert 26 * n // 2 + n < len(exp) < 29 * n // 2 + n // 2
    # as for the skin pair set, only pairs within rounding of rl may differ
    # (a tile list keeps pairs up to rl^2 (1 + 2^-40))
    diff = _unordered(pairs).symmetric_difference(exp)
    for i, j in diff:
        d = cfg.pos[i] - cfg.pos[j]
        d -= cfg.box[0] * np.rint(d / cfg.box[0])
        assert abs(np.dot(d, d) - rl * rl) < 1e-10
    assert len(diff) <= 2


def test_fcc_lattice_exact_counts():
    cfg = md_inputs.lj_fluid(10, temperature=0.72, seed=1)
    say("case: fcc counts")
    for mode, per in (("full", 78), ("half", 39), ("tile", 78)):
        s = _system(cfg, mode=mode)
        s.setup()
        cnt = s.count.cpu().numpy()
        if mode != "half":
            assert np.all(cnt == per)
        else:
            assert cnt.sum() == per * cfg.n
        assert np.abs(s.forces_np()).max() < 1e-10


@pytest.mark.parametrize("mode,rows", [("full", None), ("tile", (1, 1)), ("tile", (2, 2))])
def test_trajectory_matches_oracle_100_steps(mode, rows):
    # the 4000-atom parity workload: T = 0.72, 100 NVE steps, FP64
    cfg = md_inputs.lj_fluid(10, temperature=0.72, seed=1)
    say(f"case: trajectory 100 steps fp64 {mode} {rows}")
    s = _system(cfg, mode=mode, prec="fp64", **({"tile_rows": rows} if rows else {}))
    s.setup()
    flags, ek, ep = [], [], []
    for t in range(cfg.steps):
        s.step_body(first=(t == 0))
        flags.append(int(s.gate[0].item()))
        ep.append(float(s.energy[0]))
        if t > 0:
            ek.append(float(s.ke[0]))
    s.vv(2)
    ek.append(float(s.ke[0]))
    assert s.ensure_list() == 0
    ref = oracle.md_run(cfg.pos, cfg.vel, cfg.box[0], RC, SKIN, cfg.dt, cfg.steps)
    assert flags == list(ref["rebuild"].astype(int))
    assert sum(flags) >= 1
    assert np.abs(s.positions() - ref["pos"]).max() < 1e-9
    assert np.abs(s.velocities() - ref["vel"]).max() < 1e-9
    np.testing.assert_allclose(ep, ref["epot"][1:], rtol=1e-10)
    np.testing.assert_allclose(ek, ref["ekin"][1:], rtol=1e-10)


def test_graph_replays_match_eager_steps():
    cfg = md_inputs.lj_fluid(8, temperature=1.5, seed=21)
    say("case: graph replay vs eager")
    a = _system(cfg)
    a.setup()
    a.run(36, check_every=0)
    b = _system(cfg)
    b.setup()
    b.run_graphed(36, k=5)      # 7 replays with eager work between them
    b.ensure_list()
    a.ensure_list()
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.forces_np(), b.forces_np())
    assert float(a.ke[0]) == float(b.ke[0])
    # the same captured graph again, from a new starting point
    a.run(12, check_every=0)
    b.run_graphed(12, k=5)
    a.ensure_list()
    b.ensure_list()
    assert np.array_equal(a.positions(), b.positions())


def test_mixed_trajectory_short_horizon():
    cfg = md_inputs.lj_fluid(10, temperature=0.72, seed=1)
    say("case: trajectory 20 steps mixed")
    s = _system(cfg, mode="full", prec="mixed")
    s.setup()
    s.run(20)
    s.ensure_list()
    ref = oracle.md_run(cfg.pos, cfg.vel, cfg.box[0], RC, SKIN, cfg.dt, 20)
    assert np.abs(s.positions() - ref["pos"]).max() < 1e-6
    assert float(s.ke[0]) == pytest.approx(ref["ekin"][-1], rel=1e-6)


def test_contains_all_pairs_within_cutoff_along_a_trajectory():
    cfg = md_inputs.lj_fluid(8, temperature=1.5, seed=9)
    say("case: containment along trajectory")
    s = _system(cfg, mode="half")
    s.setup()
    for chunk in range(4):
        s.run(15, check_every=0)
        s.ensure_list()
        pos = s.positions()
        need = set(map(tuple, oracle.pairs_cells(pos, cfg.box[0], RC)))
        assert need <= _unordered(s.list_pairs()[0])


def test_neighbour_overflow_is_flagged_then_recovered(c1_snapshot):
    from paper_2109_10876_amd import _abi as abi
    cfg = c1_snapshot
    say("case: overflow")
    s = _system(cfg, mode="full", max_nbr=10)
    s.sort(gated=False)
    s.build(gated=False)
    import torch
    torch.cuda.synchronize()
    assert int(s.status.item()) & abi.MD_F_NBR_OVERFLOW
    assert int(s.need.item()) == int(s.count.max().item()) > 10
    s.ensure_list()
    assert s.max_nbr >= int(s.count.max().item())
    s.forces()
    ref, _, _ = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
    assert np.abs(s.forces_np() - ref).max() < 1e-10


def _midrun_overflow_case(mode):
    # the 4000-atom fluid from its perfect FCC sites: exactly 78 neighbours
    # within rc + skin at t = 0, so max_nbr = 80 fits at set-up; the vibrating
    # lattice needs more, so the list first overflows at a rebuild during
    # the run
    cfg = md_inputs.lj_fluid(10, temperature=0.72, seed=1)
    s = _system(cfg, mode=mode, prec="fp64", max_nbr=80)
    s.setup()
    assert s.max_nbr == 80 and s.recoveries == []
    return cfg, s


@pytest.mark.parametrize("mode,graphed", [("full", False), ("tile", False), ("tile", True)])
def test_overflow_first_seen_mid_run_is_recovered(mode, graphed):
    # run() goes back to the state saved at the last check, grows the list
    # and runs those steps again (run_checked: from the start of the run);
    # the trajectory then equals the oracle's, which never uses a list
    cfg, s = _midrun_overflow_case(mode)
    say(f"case: mid-run overflow {mode} graphed={graphed}")
    if graphed:
        s.run_checked(cfg.steps, k=10)
    else:
        s.run(cfg.steps, check_every=10)
    assert s.ensure_list() == 0
    assert s.recoveries and s.max_nbr > 80
    if not graphed:
        assert s.recoveries[0]["step"] > 0
    ref = oracle.md_run(cfg.pos, cfg.vel, cfg.box[0], RC, SKIN, cfg.dt, cfg.steps)
    assert np.abs(s.positions() - ref["pos"]).max() < 1e-9
    assert np.abs(s.velocities() - ref["vel"]).max() < 1e-9
    assert float(s.energy[0]) == pytest.approx(ref["epot"][-1], rel=1e-10)
    assert float(s.ke[0]) == pytest.approx(ref["ekin"][-1], rel=1e-10)


@pytest.mark.parametrize("mode", ["full", "tile"])
def test_overflow_after_an_unchecked_run_raises(mode):
    # without checks the steps after the overflow used a truncated list:
    # reading the status afterwards raises and leaves the flag set
    from paper_2109_10876_amd import _abi as abi
    cfg, s = _midrun_overflow_case(mode)
    say(f"case: unchecked overflow raises {mode}")
    s.run(cfg.steps, check_every=0)
    with pytest.raises(abi.ListOverflowError):
        s.ensure_list()
    assert int(s.status.item()) & abi.MD_F_NBR_OVERFLOW


def test_small_boxes_with_two_cells_per_dimension():
    # replicas of 500 atoms: box 8.398 gives 2 cells of edge >= 2.8 per dimension
    cfg = md_inputs.replica_batch(nrep=5, nmin=500, nmax=700, seed=11)
    say("case: small replicas")
    for mode in ("full", "half"):
        s = _system(cfg, mode=mode)
        s.setup()
        f = s.forces_np()
        off = cfg.atom_off()
        for r in range(cfg.nrep):
            a, b = off[r], off[r + 1]
            ref, e, w = oracle.lj_forces(cfg.pos[a:b], cfg.box[r], RC, cfg.eps, cfg.sig,
                                         cfg.types[a:b], 1)
            assert np.abs(f[a:b] - ref).max() < 1e-9
            assert float(s.energy[r]) == pytest.approx(e, rel=1e-12)
            assert float(s.virial[r]) == pytest.approx(w, rel=1e-12)


@pytest.mark.parametrize("mode,prec", [("full", "fp64"), ("half", "fp64"), ("tile", "fp64"),
                                       ("full", "mixed"), ("tile", "mixed")])
def test_one_pair_and_an_isolated_atom(mode, prec):
    # the smallest system the method has: two atoms 1.2 apart (one pair inside
    # rc, across a cell boundary) and one atom beyond rc + skin of both, in a
    # box of two cells per side; the isolated atom's list is empty and its
    # force exactly zero, and the pair's forces are equal and opposite
    pos = np.array([[3.4, 1.0, 1.0], [4.6, 1.0, 1.0], [5.5, 5.5, 5.5]])
    cfg = dataclasses.replace(md_inputs.lj_fluid(10), pos=pos, vel=np.zeros_like(pos),
                              box=np.full((1, 3), 8.0), natoms=np.array([3]),
                              types=np.zeros(3, np.int32))
    say(f"case: one pair and an isolated atom {mode} {prec}")
    s = _system(cfg, mode=mode, prec=prec)
    s.setup()
    assert s.ensure_list() == 0
    pairs, _ = s.list_pairs()
    assert _unordered(pairs) == {(0, 1)}
    f = s.forces_np()
    ref, e, w = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
    assert np.all(f[2] == 0.0)
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert np.abs(f - ref).max() <= tol * np.abs(ref).max()
    assert float(s.energy[0]) == pytest.approx(e, rel=tol)
    assert float(s.virial[0]) == pytest.approx(w, rel=tol)


def test_batch_equals_each_replica_alone():
    cfg = md_inputs.replica_batch(nrep=6, nmin=500, nmax=5000, seed=12)
    say("case: batch vs single")
    s = _system(cfg)
    s.setup()
    s.run(10)
    s.ensure_list()
    pos_b, f_b = s.positions(), s.forces_np()
    off = cfg.atom_off()
    for r in (0, 3, 5):
        a, b = off[r], off[r + 1]
        one = md_inputs.Config("one", cfg.pos[a:b], cfg.vel[a:b], cfg.box[r:r + 1],
                               cfg.natoms[r:r + 1], cfg.types[a:b], 2, cfg.eps, cfg.sig,
                               cfg.mass, RC, SKIN, cfg.dt, 1.0, 10)
        t = _system(one)
        t.setup()
        t.run(10)
        t.ensure_list()
        assert np.array_equal(t.positions(), pos_b[a:b])
        assert np.array_equal(t.forces_np(), f_b[a:b])
        assert float(t.ke[0]) == float(s.ke[r])


@pytest.mark.parametrize("prec,mode", [("fp64", "full"), ("mixed", "full"), ("fp64", "tile"),
                                       ("mixed", "tile")])
def test_vjp_matches_oracle(prec, mode):
    import torch
    cfg = md_inputs.replica_batch(nrep=3, nmin=900, nmax=2500, seed=13)
    say(f"case: vjp {prec} {mode}")
    s = _system(cfg, mode=mode, prec=prec)
    s.setup()
    rng = np.random.default_rng(0)
    G = rng.normal(size=(cfg.n, 3))
    gE = rng.normal(size=cfg.nrep)
    ids = s.id.cpu().numpy()
    d = s.dev
    Gs = G[ids]
    gfx, gfy, gfz = (torch.tensor(Gs[:, k].copy(), device=d) for k in range(3))
    gx = torch.zeros(3 * cfg.n, dtype=torch.float64, device=d)
    geps = torch.zeros(4, dtype=torch.float64, device=d)
    gsig = torch.zeros(4, dtype=torch.float64, device=d)
    s.vjp(gfx, gfy, gfz, torch.tensor(gE, device=d), gx, geps, gsig)
    torch.cuda.synchronize()
    gxs = gx.cpu().numpy().reshape(3, cfg.n).T
    got = np.empty_like(gxs)
    got[ids] = gxs
    off = cfg.atom_off()
    ge_ref = np.zeros((2, 2))
    gs_ref = np.zeros((2, 2))
    tol = 1e-11 if prec == "fp64" else 1e-5
    for r in range(cfg.nrep):
        a, b = off[r], off[r + 1]
        gx_r, ge_r, gs_r = oracle.lj_vjp(cfg.pos[a:b], cfg.box[r], RC, G[a:b], gE[r], cfg.eps,
                                         cfg.sig, cfg.types[a:b], 1)
        assert _err(got[a:b], gx_r) < tol
        ge_ref += ge_r
        gs_ref += gs_r
    np.testing.assert_allclose(geps.cpu().numpy().reshape(2, 2), ge_ref, rtol=tol * 10)
    np.testing.assert_allclose(gsig.cpu().numpy().reshape(2, 2), gs_ref, rtol=tol * 10)


@pytest.fixture(scope="module")
def lj1m_jittered():
    # the 1,048,576-atom workload jittered so forces are non-zero, with the
    # oracle's forces, energy and virial of all atoms (its cell-list path)
    cfg = md_inputs.lj_fluid(64, temperature=1.0, seed=2, jitter_amp=0.1)
    ref = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
    return cfg, ref


@pytest.mark.parametrize("prec,mode,rows", [("mixed", "full", None), ("fp64", "full", None),
                                            ("mixed", "tile", (1, 1)), ("fp64", "tile", (2, 2)),
                                            ("mixed", "tile", (2, 1))])
def test_full_size_sampled_forces(lj1m_jittered, prec, mode, rows):
    # the 1,048,576-atom workload, in the configuration the benchmark times:
    # every atom's force, the energy and the virial against the oracle's cell
    # path, and 48 sampled atoms against its O(N) single-atom loop
    cfg, (f_ref, e_ref, w_ref) = lj1m_jittered
    say(f"case: 1M {prec} {mode} {rows}")
    s = _system(cfg, mode=mode, prec=prec, **({"tile_rows": rows} if rows else {}))
    s.setup()
    s.ensure_list()
    f = s.forces_np()
    err_all = _err(f, f_ref)
    e_rel = abs(float(s.energy[0]) - e_ref) / abs(e_ref)
    w_rel = abs(float(s.virial[0]) - w_ref) / abs(w_ref)
    say(f"  all atoms e_F = {err_all:.3e}, E rel {e_rel:.3e}, W rel {w_rel:.3e}")
    assert err_all < (1e-12 if prec == "fp64" else 1e-5)
    assert e_rel < (1e-11 if prec == "fp64" else 1e-6)
    assert w_rel < (1e-11 if prec == "fp64" else 1e-6)
    planes = tuple(np.ascontiguousarray(cfg.pos[:, k]) for k in range(3))
    rng = np.random.default_rng(1)
    sample = rng.choice(cfg.n, 48, replace=False)
    ref = np.array([oracle.lj_force_one(i, None, cfg.box[0], RC, planes=planes)[0]
                    for i in sample])
    err = _err(f[sample], ref)
    say(f"  sampled e_F = {err:.3e}")
    assert err < (1e-12 if prec == "fp64" else 1e-5)
    # the list at t=0 holds every pair within rc + skin: FCC-perturbed counts
    cnt = s.count.cpu().numpy()
    assert cnt.min() > 40 and cnt.max() < s.max_nbr


@pytest.mark.parametrize("m,rows", [(1, (1, 1)), (2, (1, 1)), (3, (1, 1)), (1, (2, 2)),
                                    (2, (2, 1)), (3, (1, 2))])
def test_tile_lists_in_two_cell_boxes(m, rows):
    # 256 atoms in a 6.72 box: two cells per dimension, so every staged row
    # wraps on both sides and holds cells twice under different images
    cfg = md_inputs.lj_fluid(4, temperature=1.0, seed=17, jitter_amp=0.1)
    say(f"case: tile two-cell box m={m} rows={rows}")
    s = _system(cfg, mode="tile", tile_cells=m, tile_rows=rows)
    s.setup()
    assert s.ensure_list() == 0
    ref, e, w = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
    assert np.abs(s.forces_np() - ref).max() < 1e-10
    assert float(s.energy[0]) == pytest.approx(e, rel=1e-12)
    got = _unordered(s.list_pairs()[0])
    exp = set(map(tuple, oracle.pairs_cells(cfg.pos, cfg.box[0], RC + SKIN)))
    assert got == exp


def test_tile_overflow_is_flagged_and_recovered():
    from paper_2109_10876_amd import _abi as abi
    import torch
    # 87,808 atoms, 16 cells per row of ~21.4 atoms: a 16-cell tile stages
    # 9 rows x 18 cells x 21.4 ~ 3470 atoms > 3072 slots
    cfg = md_inputs.lj_fluid(28, temperature=1.0, seed=19, jitter_amp=0.1)
    say("case: tile overflow")
    s = _system(cfg, mode="tile", tile_cells=16)
    s.sort(gated=False)
    s.build(gated=False)
    torch.cuda.synchronize()
    assert int(s.status.item()) & abi.MD_F_TILE_OVERFLOW
    assert int(s.tile_need.item()) > abi.MD_TILE_SLOTS
    s.ensure_list()
    assert s.tile_cells < 16
    s.forces()
    f = s.forces_np()
    planes = tuple(np.ascontiguousarray(cfg.pos[:, k]) for k in range(3))
    for i in np.random.default_rng(0).choice(cfg.n, 24, replace=False):
        ref = oracle.lj_force_one(i, None, cfg.box[0], RC, planes=planes)[0]
        assert np.abs(f[i] - ref).max() < 1e-10


def test_tile_graph_replays_match_eager():
    cfg = md_inputs.lj_fluid(8, temperature=1.5, seed=23)
    say("case: tile graph vs eager")
    a = _system(cfg, mode="tile")
    a.setup()
    a.run(30, check_every=0)
    b = _system(cfg, mode="tile")
    b.setup()
    b.run_graphed(30, k=4)
    a.ensure_list()
    b.ensure_list()
    assert np.array_equal(a.positions(), b.positions())
    f = _system(cfg, mode="full")
    f.setup()
    f.run(30, check_every=0)
    f.ensure_list()
    assert np.abs(f.positions() - a.positions()).max() < 1e-10


@pytest.mark.parametrize("tb,slots,rows", [(256, 2048, (2, 2)), (256, 1536, (2, 1)),
                                           (256, 1536, (1, 1)), (128, 0, (2, 1)),
                                           (64, 0, (1, 1))])
def test_tile_shapes_match_oracle(c1_snapshot, tb, slots, rows):
    # every workgroup shape (threads x staged capacity) gives the oracle's
    # forces and the skin pair set; tile size chosen automatically per shape.
    # (5 cells of ~32 atoms per side: 2 x 2 rows would stage ~1536 atoms even
    # for one-cell tiles, which the 1536-slot shape cannot hold)
    from paper_2109_10876_amd import _abi as abi
    lib = abi.load()
    cfg = c1_snapshot
    say(f"case: tile shape tb={tb} slots={slots} rows={rows}")
    assert lib.md_tune_set(abi.MD_TUNE_TILE_THREADS, tb) == 0
    assert lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, slots) == 0
    try:
        s = _system(cfg, mode="tile", prec="fp64", tile_rows=rows)
        assert 1 <= s.tile_cells <= lib.md_tile_max_cells()
        s.setup()
        assert s.ensure_list() == 0
        ref, e, w = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
        assert np.abs(s.forces_np() - ref).max() < 1e-10
        assert float(s.energy[0]) == pytest.approx(e, rel=1e-12)
        assert float(s.virial[0]) == pytest.approx(w, rel=1e-12)
        got = _unordered(s.list_pairs()[0])
        exp = set(map(tuple, oracle.pairs_cells(cfg.pos, cfg.box[0], RC + SKIN)))
        assert got == exp
    finally:
        lib.md_tune_set(abi.MD_TUNE_TILE_THREADS, 256)
        lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, 0)


def test_tile_cells_beyond_the_shape_are_rejected():
    # the 64-thread shape holds at most 8 cells per tile along x: a 9-cell
    # tile is refused on the host before any launch
    from paper_2109_10876_amd import _abi as abi
    lib = abi.load()
    cfg = md_inputs.lj_fluid(16, temperature=1.0, seed=23, jitter_amp=0.05)
    say("case: tile cells beyond the shape")
    assert lib.md_tune_set(abi.MD_TUNE_TILE_THREADS, 64) == 0
    try:
        s = _system(cfg, mode="tile", tile_cells=9)
        s.sort(gated=False)
        with pytest.raises(abi.MDError):
            s.build(gated=False)
    finally:
        lib.md_tune_set(abi.MD_TUNE_TILE_THREADS, 256)


def test_tile_list_padding_and_neighbour_overflow(c1_snapshot):
    # tile lists: entries past the count, up to a multiple of 16, name the pad
    # slot; a too-small max_nbr is flagged, regrown, and forces recover
    from paper_2109_10876_amd import _abi as abi
    import torch
    lib = abi.load()
    cfg = c1_snapshot
    say("case: tile padding and neighbour overflow")
    s = _system(cfg, mode="tile", prec="fp64", max_nbr=16)
    assert s.max_nbr == 16
    s.sort(gated=False)
    s.build(gated=False)
    torch.cuda.synchronize()
    assert int(s.status.item()) & abi.MD_F_NBR_OVERFLOW
    s.ensure_list()
    assert s.max_nbr % 16 == 0 and s.max_nbr >= int(s.count.max().item())
    cnt = s.count.cpu().numpy()
    ent = s.tile_entries()
    pad = 8 * lib.md_tile_capacity()
    for i in range(0, s.N, 97):
        n = int(cnt[i])
        top = (n + 15) // 16 * 16
        assert np.all(ent[i, n:top] == pad)
        assert np.all(ent[i, :n] < pad) and np.all(ent[i, :n] % 8 == 0)
    s.forces()
    ref, e, _ = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
    assert np.abs(s.forces_np() - ref).max() < 1e-10
    assert float(s.energy[0]) == pytest.approx(e, rel=1e-12)


def _crowded_cells():
    # 8 cells of 2.9 per side (Verlet radius 2.8) holding a jittered lattice of
    # 8000 atoms (15.6 per cell), except two cells: cell A = (3, 3, 3) holds a
    # clump of 60 atoms near its low y/z corner and cell B = (3, 2, 2), which
    # lies in A's first stencil row, a clump of 30 atoms near the corner
    # they share.  Every clump atom of A is within the Verlet radius of the
    # other 89, so the list build holds over 80 entries of one home atom after
    # its first three candidate chunks while the stencil still has over 192
    # candidates left: the wave's entry buffer is flushed mid-list.
    L, nc = 23.2, 8
    w = L / nc
    rng = np.random.default_rng(23)
    g = (np.arange(20) + 0.5) * (L / 20)
    bg = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    bg = bg + rng.uniform(-0.1, 0.1, bg.shape)
    cell = np.floor(bg / w).astype(int)
    keep = ~(np.all(cell == (3, 3, 3), 1) | np.all(cell == (3, 2, 2), 1))
    a = np.stack(np.meshgrid(*(np.arange(4),) * 3, indexing="ij"), -1).reshape(-1, 3)[:60]
    a = np.array([3 * w + 0.05, 3 * w + 0.05, 3 * w + 0.05]) + 0.3 * a
    b = np.stack(np.meshgrid(*(np.arange(4),) * 3, indexing="ij"), -1).reshape(-1, 3)[:30]
    b = np.array([3 * w + 0.05, 3 * w - 0.7, 3 * w - 0.7]) + np.array([0.3, 0.2, 0.2]) * b
    clumps = np.concatenate([a, b]) + rng.uniform(-0.01, 0.01, (90, 3))
    pos = np.mod(np.concatenate([bg[keep], clumps]), L)
    n = pos.shape[0]
    cfg = md_inputs.Config("crowded_cells", pos, np.zeros((n, 3)), np.full((1, 3), L),
                           np.array([n]), np.zeros(n, np.int32), 1, np.ones((1, 1)),
                           np.ones((1, 1)), np.ones(1), RC, SKIN, 0.005, 1.0, 1)
    # the construction does what it is for (checked on the host)
    c = np.floor(pos / w).astype(int)
    in_a = np.all(c == (3, 3, 3), 1)
    assert in_a.sum() == 60 and np.all(c == (3, 2, 2), 1).sum() == 30
    d = np.abs(c - np.array([3, 3, 3]))
    assert 384 <= np.all(d <= 1, 1).sum() <= 768
    pa = pos[in_a]
    near = np.linalg.norm(pa[:, None, :] - pos[None, :, :], axis=2) < RC + SKIN
    assert near.sum(1).min() - 1 > 80
    return cfg


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tile_build_flushes_a_crowded_cells_entries(prec):
    cfg = _crowded_cells()
    say(f"case: tile build of crowded cells {prec} N={cfg.n}")
    s = _system(cfg, mode="tile", prec=prec)
    s.setup()
    s.ensure_list()
    got = _unordered(s.list_pairs()[0])
    rl = RC + SKIN
    exp = set(map(tuple, oracle.pairs_cells(cfg.pos, cfg.box[0], rl)))
    # the set is unique up to pairs within rounding of the Verlet radius
    for i, j in got.symmetric_difference(exp):
        d = cfg.pos[i] - cfg.pos[j]
        d -= cfg.box[0] * np.rint(d / cfg.box[0])
        assert abs(np.dot(d, d) - rl * rl) < 1e-10
    assert len(got.symmetric_difference(exp)) <= 2
    ref, e, _ = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
    assert _err(s.forces_np(), ref) < (1e-12 if prec == "fp64" else 1e-5)


def _one_type(cfg):
    # the replica batch with every atom of type 0 and a 1 x 1 (eps, sigma)
    return md_inputs.Config(cfg.name + "_1t", cfg.pos, cfg.vel, cfg.box, cfg.natoms,
                            np.zeros_like(cfg.types), 1, np.ones((1, 1)), np.ones((1, 1)),
                            np.ones(1), cfg.rc, cfg.skin, cfg.dt, cfg.temperature, cfg.steps)


@pytest.mark.parametrize("rows", [(1, 1), (2, 2)])
def test_tile_lists_on_a_batch_of_uneven_replicas(rows):
    # five replicas of 500 .. 6000 atoms (boxes of 2 to 4 cells per side),
    # each replica's forces and energy against the oracle on that replica
    cfg = _one_type(md_inputs.replica_batch(nrep=5, nmin=500, nmax=6000, seed=21))
    say(f"case: tile batch of replicas rows={rows}")
    s = _system(cfg, mode="tile", prec="fp64", tile_rows=rows)
    s.setup()
    assert s.ensure_list() == 0
    f = s.forces_np()
    off = cfg.atom_off()
    for r in range(5):
        a, b = off[r], off[r + 1]
        ref, e, w = oracle.lj_forces(cfg.pos[a:b], cfg.box[r], RC, shift=1)
        assert np.abs(f[a:b] - ref).max() < 1e-10
        assert float(s.energy[r]) == pytest.approx(e, rel=1e-10)
        assert float(s.virial[r]) == pytest.approx(w, rel=1e-10)


def test_tile_batch_equals_each_replica_alone():
    cfg = _one_type(md_inputs.replica_batch(nrep=4, nmin=800, nmax=5000, seed=22))
    say("case: tile batch vs single")
    s = _system(cfg, mode="tile", tile_cells=2, tile_rows=(2, 2))
    s.setup()
    s.run(12)
    s.ensure_list()
    pos_b, f_b = s.positions(), s.forces_np()
    off = cfg.atom_off()
    for r in (0, 2, 3):
        a, b = off[r], off[r + 1]
        one = md_inputs.Config("one", cfg.pos[a:b], cfg.vel[a:b], cfg.box[r:r + 1],
                               cfg.natoms[r:r + 1], cfg.types[a:b], 1, cfg.eps, cfg.sig,
                               cfg.mass, RC, SKIN, cfg.dt, 1.0, 12)
        t = _system(one, mode="tile", tile_cells=2, tile_rows=(2, 2))
        t.setup()
        t.run(12)
        t.ensure_list()
        assert np.array_equal(t.positions(), pos_b[a:b])
        assert np.array_equal(t.forces_np(), f_b[a:b])
        assert float(t.ke[0]) == float(s.ke[r])


def test_tile_widths_per_replica_equal_each_replica_alone():
    # replicas of 500 .. 20000 atoms have cells of different occupancy, so the
    # automatic tiling gives each its own width (cells per tile along x); a
    # replica's trajectory and forces in the batch equal, bit for bit, those
    # of the replica alone tiled with that width, and its forces match the
    # oracle
    cfg = _one_type(md_inputs.replica_batch(nrep=6, nmin=500, nmax=20000, seed=23))
    say("case: per-replica tile widths")
    s = _system(cfg, mode="tile", tile_rows=(2, 2))
    assert s.h_tile_m is not None and len(set(s.h_tile_m.tolist())) > 1
    assert s.tile_cells == int(s.h_tile_m.max())
    s.setup()
    s.run(12)
    s.ensure_list()
    pos_b, f_b = s.positions(), s.forces_np()
    off = cfg.atom_off()
    for r in range(6):
        a, b = off[r], off[r + 1]
        one = md_inputs.Config("one", cfg.pos[a:b], cfg.vel[a:b], cfg.box[r:r + 1],
                               cfg.natoms[r:r + 1], cfg.types[a:b], 1, cfg.eps, cfg.sig,
                               cfg.mass, RC, SKIN, cfg.dt, 1.0, 12)
        t = _system(one, mode="tile", tile_cells=int(s.h_tile_m[r]), tile_rows=(2, 2))
        t.setup()
        t.run(12)
        t.ensure_list()
        assert np.array_equal(t.positions(), pos_b[a:b]), r
        assert np.array_equal(t.forces_np(), f_b[a:b]), r
    r = int(np.argmax(s.h_tile_m))
    a, b = off[r], off[r + 1]
    ref, _, _ = oracle.lj_forces(pos_b[a:b], cfg.box[r], RC, shift=1)
    assert _err(f_b[a:b], ref) < 1e-5


def test_tile_overflow_shrinks_only_the_overflowing_replicas_tiles():
    # one replica planned with a whole cell row per tile overflows the staging
    # capacity: the recovery shrinks that replica's tiles only, and the lists
    # then give the oracle's forces
    cfg = _one_type(md_inputs.replica_batch(nrep=4, nmin=3000, nmax=12000, seed=24))
    say("case: per-replica tile overflow")
    s = _system(cfg, mode="tile", tile_rows=(2, 2))
    m = (s.h_tile_m.copy() if s.h_tile_m is not None
         else np.full(s.R, s.tile_cells, dtype=np.int32))
    r = int(np.argmax(cfg.natoms))
    big = m.copy()
    big[r] = int(s.h_ncell[r, 0])
    assert big[r] > m[r]
    s._plan_tiles(big)
    s._set_nlist()
    s.setup()
    assert s.ensure_list() == 0
    assert s.h_tile_m[r] < big[r]
    assert all(s.h_tile_m[k] == big[k] for k in range(s.R) if k != r)
    f = s.forces_np()
    off = cfg.atom_off()
    for k in (r, (r + 1) % s.R):
        a, b = off[k], off[k + 1]
        ref, _, _ = oracle.lj_forces(cfg.pos[a:b], cfg.box[k], RC, shift=1)
        assert np.abs(f[a:b] - ref).max() < 1e-10


@pytest.mark.parametrize("prec,ntypes", [("fp64", 2), ("mixed", 2), ("fp64", 3),
                                          ("mixed", 4)])
def test_typed_tile_lists_on_the_replica_batch(prec, ntypes):
    # several atom types with one symmetric (eps, sigma) table: tile-list
    # entries carry the neighbour's type (two types: constants selected in
    # registers; three or four: read from a table); forces and energy per
    # replica against the oracle, and the pair set against the global list
    cfg = md_inputs.replica_batch(nrep=5, nmin=500, nmax=6000, seed=23)
    if ntypes != 2:
        cfg = md_inputs.retyped(cfg, ntypes, seed=29)
    say(f"case: typed tile batch {prec} ntypes={ntypes}")
    s = _system(cfg, mode="tile", prec=prec, tile_rows=(2, 2))
    assert s.nlist.tile_types == ntypes
    s.setup()
    assert s.ensure_list() == 0
    f = s.forces_np()
    off = cfg.atom_off()
    for r in range(5):
        a, b = off[r], off[r + 1]
        ref, e, w = oracle.lj_forces(cfg.pos[a:b], cfg.box[r], RC, cfg.eps, cfg.sig,
                                     cfg.types[a:b], shift=1)
        if prec == "fp64":
            assert np.abs(f[a:b] - ref).max() < 1e-10
            assert float(s.energy[r]) == pytest.approx(e, rel=1e-10)
            assert float(s.virial[r]) == pytest.approx(w, rel=1e-10)
        else:
            assert _err(f[a:b], ref) < 1e-5
            assert abs(float(s.energy[r]) - e) <= 1e-5 * (b - a)
    g = _system(cfg, mode="full")
    g.setup()
    assert _unordered(s.list_pairs()[0]) == _unordered(g.list_pairs()[0])


def test_typed_tile_list_is_required_for_several_types(c1_snapshot):
    # an untyped tile list with a two-type LJ table (and the reverse) is
    # refused on the host
    from paper_2109_10876_amd import _abi as abi
    cfg = md_inputs.replica_batch(nrep=2, nmin=500, nmax=900, seed=24)
    say("case: typed tile list checks")
    s = _system(cfg, mode="tile")
    s.setup()
    s.nlist.tile_types = 0
    with pytest.raises(abi.MDError):
        s.forces()
    one = _system(c1_snapshot, mode="tile")
    one.setup()
    one.nlist.tile_types = 2
    with pytest.raises(abi.MDError):
        one.forces()


@pytest.mark.parametrize("rows", [(1, 1), (2, 2)])
def test_fused_force_step_trajectory_matches_oracle(rows):
    # md_lj_forces_vv: the forces of step t with its Integrate2 and the
    # Integrate1 of step t + 1 in one call; same schedule, energies and
    # kinetic energies as the oracle's 100 NVE steps
    cfg = md_inputs.lj_fluid(10, temperature=0.72, seed=1)
    say(f"case: fused force+step trajectory {rows}")
    s = _system(cfg, mode="tile", prec="fp64", tile_rows=rows)
    assert s.fuse
    s.setup()
    flags, ek, ep = [], [], []
    s.vv(1)
    flags.append(int(s.gate[0].item()))
    s.sort()
    s.build()
    for t in range(1, cfg.steps):
        s.forces_vv()
        ep.append(float(s.energy[0]))
        ek.append(float(s.ke[0]))
        flags.append(int(s.gate[0].item()))
        s.sort()
        s.build()
    s.forces()
    ep.append(float(s.energy[0]))
    s.vv(2)
    ek.append(float(s.ke[0]))
    assert s.ensure_list() == 0
    ref = oracle.md_run(cfg.pos, cfg.vel, cfg.box[0], RC, SKIN, cfg.dt, cfg.steps)
    assert flags == list(ref["rebuild"].astype(int))
    assert np.abs(s.positions() - ref["pos"]).max() < 1e-9
    assert np.abs(s.velocities() - ref["vel"]).max() < 1e-9
    np.testing.assert_allclose(ep, ref["epot"][1:], rtol=1e-10)
    np.testing.assert_allclose(ek, ref["ekin"][1:], rtol=1e-10)


def test_repeated_fused_steps_set_the_oracles_rebuild_schedule():
    # the repeated steps of a run take the skin test from the force kernel
    # itself, into two gate words used alternately with the position buffers
    # (md_lj_forces_vv's gate_clear): the gate each step's re-sort and list
    # build read is the oracle's rebuild schedule, and the trajectory is the
    # oracle's, eagerly and through graphs
    cfg = md_inputs.lj_fluid(10, temperature=0.72, seed=1)
    say("case: rebuild schedule of repeated fused steps")
    ref = oracle.md_run(cfg.pos, cfg.vel, cfg.box[0], RC, SKIN, cfg.dt, cfg.steps)
    s = _system(cfg, mode="tile", prec="fp64")
    assert s.fuse and len(s._pos) == 2
    s.setup()
    s._head()
    flags = [int(s.step_gate[0].item())]
    for _ in range(1, cfg.steps):
        s._body()
        assert s.step_gate.data_ptr() != s.gate.data_ptr()
        flags.append(int(s.step_gate[0].item()))
    s._tail()
    assert s.ensure_list() == 0
    assert flags == list(ref["rebuild"].astype(int))
    assert sum(flags) >= 2
    assert np.abs(s.positions() - ref["pos"]).max() < 1e-9
    assert float(s.energy[0]) == pytest.approx(ref["epot"][-1], rel=1e-10)
    assert float(s.ke[0]) == pytest.approx(ref["ekin"][-1], rel=1e-10)
    g = _system(cfg, mode="tile", prec="fp64")
    g.setup()
    g.run_graphed(cfg.steps, k=6)
    assert g.ensure_list() == 0
    assert np.array_equal(g.positions(), s.positions())


@pytest.mark.parametrize("prec,batch", [("fp64", 4), ("mixed", 4), ("fp64", 8), ("mixed", 8)])
def test_fused_and_split_steps_are_bitwise_equal(prec, batch):
    # same FMA sequence in one kernel or in md_lj_forces + md_vv_step:
    # positions and velocities equal bit for bit, also through graphs; with
    # a pair batch of 8 the tile kernels take 16 entries per pass
    from paper_2109_10876_amd import _abi as abi
    lib = abi.load()
    assert lib.md_tune_set(abi.MD_TUNE_PAIR_BATCH, batch) == 0
    try:
        _fused_and_split(prec)
    finally:
        lib.md_tune_set(abi.MD_TUNE_PAIR_BATCH, 4)


def _fused_and_split(prec):
    cfg = md_inputs.lj_fluid(8, temperature=1.5, seed=25)
    say(f"case: fused vs split {prec}")
    a = _system(cfg, mode="tile", prec=prec, fuse=False)
    b = _system(cfg, mode="tile", prec=prec)
    c = _system(cfg, mode="tile", prec=prec)
    # with the packed copy kept, the fused call copies the next positions
    # back instead of alternating two buffers
    d = _system(cfg, mode="tile", prec=prec, pos4=True)
    assert not a.fuse and b.fuse and d.fuse
    assert len(b._pos) == 2 and len(d._pos) == 1
    for x in (a, b, c, d):
        x.setup()
    a.run(40, check_every=0)
    b.run(40, check_every=0)
    c.run_graphed(40, k=5)
    d.run(40, check_every=0)
    for x in (a, b, c, d):
        assert x.ensure_list() == 0
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.velocities(), b.velocities())
    assert np.array_equal(b.positions(), c.positions())
    assert np.array_equal(b.positions(), d.positions())
    assert np.array_equal(a.forces_np(), b.forces_np())
    assert float(b.ke[0]) == pytest.approx(float(a.ke[0]), rel=1e-12)


@pytest.mark.parametrize("prec,ntypes", [("fp64", 2), ("mixed", 2), ("mixed", 3)])
def test_fused_and_split_steps_are_bitwise_equal_with_types(prec, ntypes):
    # several atom types (typed tile lists, per-type masses): the fused call
    # and md_lj_forces + md_vv_step give the same trajectory bit for bit, on
    # a batch of uneven replicas, eagerly and through graphs; the forces and
    # energies of the final state match the oracle's
    cfg = md_inputs.retyped(md_inputs.replica_batch(nrep=3, nmin=500, nmax=3000, seed=27),
                            ntypes, seed=33)
    cfg = dataclasses.replace(cfg, mass=np.linspace(1.0, 2.0, ntypes))
    say(f"case: fused vs split with {ntypes} types {prec}")
    a = _system(cfg, mode="tile", prec=prec, fuse=False, tile_rows=(2, 2))
    b = _system(cfg, mode="tile", prec=prec, tile_rows=(2, 2))
    c = _system(cfg, mode="tile", prec=prec, tile_rows=(2, 2))
    assert not a.fuse and b.fuse and c.fuse
    for x in (a, b, c):
        x.setup()
    a.run(30, check_every=0)
    b.run(30, check_every=0)
    c.run_graphed(30, k=6)
    for x in (a, b, c):
        assert x.ensure_list() == 0
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.velocities(), b.velocities())
    assert np.array_equal(b.positions(), c.positions())
    assert np.array_equal(a.forces_np(), b.forces_np())
    f = b.forces_np()
    pos = b.positions()
    off = cfg.atom_off()
    for r in range(cfg.nrep):
        lo, hi = off[r], off[r + 1]
        ref, e, _ = oracle.lj_forces(pos[lo:hi], cfg.box[r], RC, cfg.eps, cfg.sig,
                                     cfg.types[lo:hi], shift=1)
        if prec == "fp64":
            assert np.abs(f[lo:hi] - ref).max() < 1e-9
            assert float(b.energy[r]) == pytest.approx(e, rel=1e-10)
        else:
            assert _err(f[lo:hi], ref) < 1e-5
            assert abs(float(b.energy[r]) - e) <= 1e-5 * (hi - lo)


def test_kernel_timing_records_eager_pair_kernels_only(c1_snapshot):
    import ctypes
    from paper_2109_10876_amd import _abi as abi
    lib = abi.load()
    say("case: kernel timing")
    s = _system(c1_snapshot, mode="tile", prec="fp64")
    s.setup()
    ms, n = ctypes.c_double(), ctypes.c_int32()
    assert lib.md_kernel_timing_start(3) == 0
    s.capture(2)   # launches under stream capture are not timed
    for _ in range(4):
        s.forces()  # four eager launches, the first three timed
    assert lib.md_kernel_timing_read(ctypes.byref(ms), ctypes.byref(n)) == 0
    assert n.value == 3 and 0.0 < ms.value < 100.0



@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tile_vjp_equals_global_vjp_one_type(prec):
    # the same adjoint over a tile-local and a global-index list of one type
    import torch
    cfg = md_inputs.lj_fluid(8, temperature=1.0, seed=21, jitter_amp=0.05)
    say(f"case: tile vs global vjp {prec}")
    rng = np.random.default_rng(4)
    G = rng.normal(size=(cfg.n, 3))
    out = {}
    for mode in ("full", "tile"):
        s = _system(cfg, mode=mode, prec=prec)
        s.setup()
        assert s.ensure_list() == 0
        ids = s.id.cpu().numpy()
        d = s.dev
        gfx, gfy, gfz = (torch.tensor(G[ids, k].copy(), device=d) for k in range(3))
        gx = torch.zeros(3 * cfg.n, dtype=torch.float64, device=d)
        ge = torch.zeros(1, dtype=torch.float64, device=d)
        gs = torch.zeros(1, dtype=torch.float64, device=d)
        s.vjp(gfx, gfy, gfz, torch.tensor([0.7], device=d, dtype=torch.float64), gx, ge, gs)
        torch.cuda.synchronize()
        gxs = gx.cpu().numpy().reshape(3, cfg.n).T
        got = np.empty_like(gxs)
        got[ids] = gxs
        out[mode] = (got, float(ge.item()), float(gs.item()))
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert _err(out["tile"][0], out["full"][0]) < tol
    assert out["tile"][1] == pytest.approx(out["full"][1], rel=tol * 10)
    assert out["tile"][2] == pytest.approx(out["full"][2], rel=tol * 10)
    gx_r, ge_r, gs_r = oracle.lj_vjp(cfg.pos, cfg.box[0], RC, G, 0.7, shift=1)
    assert _err(out["tile"][0], gx_r) < (1e-11 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("mode,prec", [("full", "fp64"), ("tile", "mixed"), ("half", "fp64")])
def test_coincident_atoms_raise_the_nonfinite_flag(mode, prec):
    # two atoms at one position: the pair term is not finite, the force call
    # says so in the status word (nothing is clamped silently)
    import torch
    from paper_2109_10876_amd import _abi as abi
    cfg = md_inputs.lj_fluid(6, temperature=1.0, seed=8)
    cfg.pos = cfg.pos.copy()
    say(f"case: coincident atoms {mode} {prec}")
    clean = _system(cfg, mode=mode, prec=prec)
    clean.setup()
    assert not (clean.ensure_list() & abi.MD_F_NONFINITE)
    cfg.pos[1] = cfg.pos[0]
    s = _system(cfg, mode=mode, prec=prec)
    s.sort(gated=False)
    s.build(gated=False)
    s.forces()
    torch.cuda.synchronize()
    assert int(s.status.item()) & abi.MD_F_NONFINITE
