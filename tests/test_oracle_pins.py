"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against closed forms of Eq. lj (Sec. 2.1.1),
crystal geometry, conservation laws of Newton's equations (Sec. 2.1),
brute force on tiny boxes, finite differences, or published generator
vectors -- never against a retyped copy of its own formulas.
"""
import math
import os

import numpy as np
import pytest

import md_inputs
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RC, SKIN = 2.5, 0.3


# ---------------------------------------------------------------- Eq. lj

@pytest.mark.parametrize("eps,sig", [(1.0, 1.0), (0.8, 1.2), (1.7, 0.9)])
def test_lj_closed_forms(eps, sig):
    # U(sigma) = 0 and the force magnitude there is 24 eps / sigma
    u, fr = oracle.lj_pair(sig * sig, eps, sig, rc=10.0, shift=0)
    assert abs(u) < 1e-14 * eps
    assert math.isclose(fr * sig, 24.0 * eps / sig, rel_tol=1e-14)
    # minimum at r = 2^(1/6) sigma: U = -eps, zero force
    rm2 = 2.0 ** (1.0 / 3.0) * sig * sig
    u, fr = oracle.lj_pair(rm2, eps, sig, rc=10.0, shift=0)
    assert math.isclose(u, -eps, rel_tol=1e-14)
    assert abs(fr) < 1e-13 * eps
    # attractive beyond the minimum, repulsive inside it
    assert oracle.lj_pair(1.2 * rm2, eps, sig, 10.0, 0)[1] < 0.0
    assert oracle.lj_pair(0.9 * rm2, eps, sig, 10.0, 0)[1] > 0.0


def test_lj_value_at_cutoff():
    # U(2.5) = 4 (2.5^-12 - 2.5^-6) = -0.016316891136... (exact decimal expansion)
    u, _ = oracle.lj_pair(RC * RC - 1e-13, 1.0, 1.0, rc=RC, shift=0)
    assert abs(u - (-0.016316891136)) < 1e-11
    # strict cutoff: r = rc and beyond contribute nothing
    assert oracle.lj_pair(RC * RC, rc=RC, shift=0) == (0.0, 0.0)
    assert oracle.lj_pair(7.0, rc=RC, shift=0) == (0.0, 0.0)
    # energy shift makes U continuous at rc and leaves the force unchanged
    us, frs = oracle.lj_pair(RC * RC - 1e-13, rc=RC, shift=1)
    u0, fr0 = oracle.lj_pair(RC * RC - 1e-13, rc=RC, shift=0)
    assert abs(us) < 1e-12
    assert frs == fr0
    assert math.isclose(u0 - us, -0.016316891136007795, rel_tol=1e-12)


def test_lj_force_is_minus_gradient_of_energy():
    # fr = -U'(r)/r, checked by central differences of U in r
    for r in (0.95, 1.1, 1.5, 2.2):
        h = 1e-6
        up, _ = oracle.lj_pair((r + h) ** 2, 1.3, 1.05, RC, 0)
        um, _ = oracle.lj_pair((r - h) ** 2, 1.3, 1.05, RC, 0)
        _, fr = oracle.lj_pair(r * r, 1.3, 1.05, RC, 0)
        assert math.isclose(fr * r, -(up - um) / (2 * h), rel_tol=1e-7)


def test_min_image():
    assert oracle.min_image(0.4, 1.0) == pytest.approx(0.4)
    assert oracle.min_image(0.6, 1.0) == pytest.approx(-0.4)
    assert oracle.min_image(-0.7, 1.0) == pytest.approx(0.3)
    assert oracle.min_image(3.2, 1.0) == pytest.approx(0.2)


def test_two_atoms_across_the_boundary():
    # atoms at x = 0.3 and x = L - 0.7 are 1.0 apart through the periodic face
    L = np.array([10.0, 11.0, 12.0])
    pos = np.array([[0.3, 5.0, 6.0], [L[0] - 0.7, 5.0, 6.0]])
    f, e, w = oracle.lj_forces_brute(pos, L, RC, shift=0)
    u, fr = oracle.lj_pair(1.0, rc=RC, shift=0)
    assert e == pytest.approx(u, rel=1e-14)
    # d = x0 - x1 reduced = +1.0, so atom 0 is pushed in +x by 24
    assert f[0, 0] == pytest.approx(fr * 1.0, rel=1e-14)
    assert f[0, 0] == pytest.approx(24.0, rel=1e-14)
    assert f[1, 0] == pytest.approx(-24.0, rel=1e-14)
    assert w == pytest.approx(fr * 1.0, rel=1e-14)


# --------------------------------------------------------- pair sets, FCC

def _fcc_shells():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fcc_shells.txt"))
            if l.strip() and not l.startswith("#")]
    return [(float(a), int(b)) for a, b in rows]


@pytest.mark.parametrize("rcut,half", [(2.5, 27), (2.8, 39)])
def test_fcc_pair_counts(rcut, half):
    # FCC at rho = 0.8442: a = 1.67960; shells (r^2/a^2, n) from the fixture.
    pos, box = md_inputs.fcc_lattice(5, 0.8442)
    a = (4 / 0.8442) ** (1 / 3)
    expect = sum(n for s, n in _fcc_shells() if s * a * a < rcut * rcut)
    assert expect == 2 * half
    pairs = oracle.pairs_cells(pos, box, rcut)
    assert pairs.shape[0] == half * pos.shape[0]
    counts = np.bincount(pairs.ravel(), minlength=pos.shape[0])
    assert np.all(counts == 2 * half)


def test_fcc_lattice_forces_vanish_and_energy_matches_shell_sum():
    pos, box = md_inputs.fcc_lattice(5, 0.8442)
    a = (4 / 0.8442) ** (1 / 3)
    for shift in (0, 1):
        f, e, w = oracle.lj_forces(pos, box, RC, shift=shift)
        assert np.abs(f).max() < 1e-11
        shell = sum(n * oracle.lj_pair(s * a * a, rc=RC, shift=shift)[0]
                    for s, n in _fcc_shells() if s * a * a < RC * RC)
        assert e / pos.shape[0] == pytest.approx(0.5 * shell, rel=1e-11)
    # lattice energy per atom, unshifted: -6.773368 (four-shell sum by hand)
    f, e, w = oracle.lj_forces(pos, box, RC, shift=0)
    assert e / pos.shape[0] == pytest.approx(-6.773368, abs=2e-6)


@pytest.mark.parametrize("seed", range(6))
def test_cell_list_equals_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    # boxes with 1, 2, 3 and more cells per dimension, non-cubic
    L = rng.uniform(2 * 2.8 + 0.05, 14.0, size=3)
    n = int(rng.integers(2, 180))
    pos = rng.uniform(-0.3, 1.3, size=(n, 3)) * L  # some atoms outside [0, L)
    for rcut in (RC, RC + SKIN, 1.1):
        if rcut >= 0.5 * L.min():
            continue
        pb = oracle.pairs_brute(pos, L, rcut)
        pc = oracle.pairs_cells(pos, L, rcut)
        assert np.array_equal(pb, pc)


def test_cell_list_rejects_small_box():
    pos = np.zeros((2, 3))
    with pytest.raises(ValueError):
        oracle.pairs_cells(pos, np.array([5.0, 8.0, 8.0]), 2.8)


# ------------------------------------------------------- forces, invariants

def _snapshot(m=4, amp=0.12, seed=0):
    pos, box = md_inputs.fcc_lattice(m, 0.8442)
    return md_inputs.jitter(pos, amp, seed=seed), box


def test_forces_cells_equal_brute_definition():
    pos, box = _snapshot(m=4)
    f1, e1, w1 = oracle.lj_forces(pos, box, RC)
    f2, e2, w2 = oracle.lj_forces_brute(pos, box, RC)
    # same partner order per atom -> identical per-atom sums
    assert np.array_equal(f1, f2)
    assert e1 == pytest.approx(e2, rel=1e-13)
    assert w1 == pytest.approx(w2, rel=1e-13)


@pytest.mark.parametrize("shift", [0, 1])
@pytest.mark.parametrize("typed", [False, True])
def test_force_one_equals_brute_rows_and_shares_sum_to_totals(shift, typed):
    # The single-atom loop (the reference of every sampled full-size check)
    # against the plainest definition, Eq. lj summed over all j != i: row i
    # bit for bit, and the half shares of E and W summed over i give E and W.
    pos, box = _snapshot(m=4, seed=11)
    n = pos.shape[0]
    kw = {}
    if typed:
        rng = np.random.default_rng(4)
        kw = dict(types=rng.integers(0, 2, n).astype(np.int32),
                  eps=np.array([[1.0, 0.87], [0.87, 1.15]]),
                  sig=np.array([[1.0, 1.08], [1.08, 0.93]]))
    f, e, w = oracle.lj_forces_brute(pos, box, RC, shift=shift, **kw)
    planes = tuple(np.ascontiguousarray(pos[:, k]) for k in range(3))
    es = ws = 0.0
    for i in range(n):
        fi, ei, wi = oracle.lj_force_one(i, pos, box, RC, shift=shift, planes=planes, **kw)
        assert np.array_equal(fi, f[i]), i
        es += ei
        ws += wi
    assert es == pytest.approx(e, rel=1e-13)
    assert ws == pytest.approx(w, rel=1e-13)
    # the forces are not trivially zero on this snapshot
    assert np.abs(f).max() > 1.0


def test_newton_third_law_and_translation_invariance():
    pos, box = _snapshot(m=4, seed=3)
    f, e, w = oracle.lj_forces(pos, box, RC)
    assert np.abs(f.sum(axis=0)).max() < 1e-10 * np.abs(f).max()
    f2, e2, w2 = oracle.lj_forces(pos + np.array([0.37, -1.91, 5.3]), box, RC)
    np.testing.assert_allclose(f2, f, rtol=0, atol=1e-10)
    assert e2 == pytest.approx(e, rel=1e-12)


def test_force_is_minus_gradient_of_total_energy():
    pos, box = _snapshot(m=4, seed=5)
    f, _, _ = oracle.lj_forces(pos, box, RC, shift=1)
    rng = np.random.default_rng(9)
    h = 1e-6
    for i in rng.choice(pos.shape[0], 6, replace=False):
        for d in range(3):
            p, m = pos.copy(), pos.copy()
            p[i, d] += h
            m[i, d] -= h
            ep = oracle.lj_forces(p, box, RC, shift=1)[1]
            em = oracle.lj_forces(m, box, RC, shift=1)[1]
            assert f[i, d] == pytest.approx(-(ep - em) / (2 * h), rel=1e-6, abs=1e-6)


def test_virial_is_minus_volume_derivative():
    # W = -dU/dlambda at lambda = 1 for r -> lambda r (positions and box)
    pos, box = _snapshot(m=4, amp=0.05, seed=7)
    _, _, w = oracle.lj_forces(pos, box, RC, shift=0)
    h = 1e-6
    ep = oracle.lj_forces(pos * (1 + h), box * (1 + h), RC, shift=0)[1]
    em = oracle.lj_forces(pos * (1 - h), box * (1 - h), RC, shift=0)[1]
    assert w == pytest.approx(-(ep - em) / (2 * h), rel=1e-6)


# ------------------------------------------------------ velocity Verlet

def _small_md(m=4, T=0.72, seed=11):
    pos, box = md_inputs.fcc_lattice(m, 0.8442)
    pos = md_inputs.jitter(pos, 0.05, seed=seed)
    vel = md_inputs.maxwell_velocities(pos.shape[0], T, seed=seed)
    return pos, vel, box


def test_skin_rule_keeps_the_list_valid_and_a_skipped_rebuild_is_caught():
    # the rebuild rule (rebuild once an atom moved more than skin/2): while it
    # has not fired, every pair within rc is in the list built with rc + skin;
    # a list kept past the point where it fires misses pairs, which the
    # containment check the GPU tests use then reports
    pos, vel, box = _small_md(T=1.5, seed=3)
    lst = set(map(tuple, oracle.pairs_cells(pos, box, RC + SKIN)))
    r = oracle.md_run(pos, vel, box, RC, SKIN, 0.005, 60)
    first = int(np.argmax(r["rebuild"])) if r["rebuild"].any() else None
    assert first is not None and first > 0
    ok = oracle.md_run(pos, vel, box, RC, SKIN, 0.005, first)
    assert set(map(tuple, oracle.pairs_cells(ok["pos"], box, RC))) <= lst
    late = oracle.md_run(pos, vel, box, RC, SKIN, 0.005, 60)
    assert not set(map(tuple, oracle.pairs_cells(late["pos"], box, RC))) <= lst


def test_vv_time_reversible():
    pos, vel, box = _small_md()
    a = oracle.md_run(pos, vel, box, RC, SKIN, 0.005, 40)
    b = oracle.md_run(a["pos"], -a["vel"], box, RC, SKIN, 0.005, 40)
    np.testing.assert_allclose(b["pos"], pos, rtol=0, atol=1e-9)
    np.testing.assert_allclose(-b["vel"], vel, rtol=0, atol=1e-9)


def test_vv_momentum_and_energy():
    pos, vel, box = _small_md()
    r = oracle.md_run(pos, vel, box, RC, SKIN, 0.005, 60)
    assert np.abs(r["vel"].sum(axis=0)).max() < 1e-11
    etot = r["epot"] + r["ekin"]
    assert np.abs(etot - etot[0]).max() < 2e-3 * abs(etot[0]) / pos.shape[0] * 50


def test_vv_energy_error_scales_as_dt_squared():
    pos, vel, box = _small_md(T=1.0)
    fl = []
    for dt, steps in ((0.004, 100), (0.002, 200)):
        r = oracle.md_run(pos, vel, box, RC, SKIN, dt, steps)
        etot = r["epot"] + r["ekin"]
        fl.append(np.sqrt(np.mean((etot - etot.mean()) ** 2)))
    assert 3.0 < fl[0] / fl[1] < 5.2


def test_rebuild_schedule_closed_form():
    # two far-apart atoms moving freely at speed 0.7: displacement after s
    # steps is 0.0035 s; the skin/2 = 0.15 test first fires at s = 43, then
    # 43 steps after each rebuild.
    box = np.array([20.0, 20.0, 20.0])
    pos = np.array([[1.0, 1.0, 1.0], [10.0, 10.0, 10.0]])
    vel = np.array([[0.7, 0.0, 0.0], [0.0, -0.7, 0.0]])
    r = oracle.md_run(pos, vel, box, RC, SKIN, 0.005, 130)
    assert list(np.nonzero(r["rebuild"])[0]) == [42, 85, 128]
    np.testing.assert_allclose(r["pos"][0], [1.0 + 130 * 0.0035, 1.0, 1.0], atol=1e-12)


# ------------------------------------------------------------------- VJP

def _vjp_case(seed=0, nt=2):
    rng = np.random.default_rng(seed)
    pos, box = _snapshot(m=3, amp=0.1, seed=seed)
    n = pos.shape[0]
    types = rng.integers(0, nt, n).astype(np.int32)
    eps = rng.uniform(0.8, 1.2, (nt, nt))
    sig = rng.uniform(0.8, 1.2, (nt, nt))
    eps = 0.5 * (eps + eps.T)
    sig = 0.5 * (sig + sig.T)
    G = rng.normal(size=(n, 3))
    return pos, box, types, eps, sig, G


def _loss(pos, box, types, eps, sig, G, gE, shift):
    f, e, _ = oracle.lj_forces(pos, box, RC, eps, sig, types, shift)
    return float(np.sum(G * f) + gE * e)


@pytest.mark.parametrize("shift", [0, 1])
def test_vjp_positions_by_finite_differences(shift):
    pos, box, types, eps, sig, G = _vjp_case(1)
    gE = 0.7
    gx, _, _ = oracle.lj_vjp(pos, box, RC, G, gE, eps, sig, types, shift)
    rng = np.random.default_rng(2)
    v = rng.normal(size=pos.shape)
    h = 1e-6
    fd = (_loss(pos + h * v, box, types, eps, sig, G, gE, shift)
          - _loss(pos - h * v, box, types, eps, sig, G, gE, shift)) / (2 * h)
    assert np.sum(gx * v) == pytest.approx(fd, rel=2e-6)
    # translation invariance: the position gradient sums to zero
    assert np.abs(gx.sum(axis=0)).max() < 1e-9 * np.abs(gx).max()


@pytest.mark.parametrize("shift", [0, 1])
def test_vjp_parameters_by_finite_differences(shift):
    pos, box, types, eps, sig, G = _vjp_case(3)
    gE = -1.3
    _, geps, gsig = oracle.lj_vjp(pos, box, RC, G, gE, eps, sig, types, shift)
    h = 1e-6
    for a, b in ((0, 0), (0, 1), (1, 1)):
        for tab, grad in ((eps, geps), (sig, gsig)):
            p, m = tab.copy(), tab.copy()
            p[a, b] += h
            m[a, b] -= h
            if a != b:
                p[b, a] += h
                m[b, a] -= h
            if tab is eps:
                lp = _loss(pos, box, types, p, sig, G, gE, shift)
                lm = _loss(pos, box, types, m, sig, G, gE, shift)
            else:
                lp = _loss(pos, box, types, eps, p, G, gE, shift)
                lm = _loss(pos, box, types, eps, m, G, gE, shift)
            assert grad[a, b] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-6)
            assert grad[a, b] == grad[b, a]


def test_vjp_energy_only_is_minus_force():
    pos, box, types, eps, sig, _ = _vjp_case(4)
    gE = 2.5
    gx, _, _ = oracle.lj_vjp(pos, box, RC, np.zeros_like(pos), gE, eps, sig, types, 1)
    f, _, _ = oracle.lj_forces(pos, box, RC, eps, sig, types, 1)
    np.testing.assert_allclose(gx, -gE * f, rtol=1e-12, atol=1e-12)


def test_vjp_force_jacobian_is_symmetric():
    # F = -grad E, so dF/dx is minus the Hessian and symmetric: with the
    # position VJP gx(u) = u^T dF/dx, u . gx(v) = v . gx(u) for any u, v
    pos, box, types, eps, sig, u = _vjp_case(6)
    v = np.random.default_rng(7).normal(size=pos.shape)
    gu, _, _ = oracle.lj_vjp(pos, box, RC, u, 0.0, eps, sig, types, 1)
    gv, _, _ = oracle.lj_vjp(pos, box, RC, v, 0.0, eps, sig, types, 1)
    a, b = float(np.sum(v * gu)), float(np.sum(u * gv))
    assert a == pytest.approx(b, rel=1e-11)


def test_vjp_eps_homogeneity_and_sigma_euler():
    pos, box, types, eps, sig, G = _vjp_case(5)
    gE = 0.9
    f, e, w = oracle.lj_forces(pos, box, RC, eps, sig, types, 1)
    _, geps, _ = oracle.lj_vjp(pos, box, RC, G, gE, eps, sig, types, 1)
    # F and (shifted) E are linear in eps: sum over unique pairs eps dL/deps = L
    uniq = [(0, 0), (0, 1), (1, 1)]
    lhs = sum(eps[a, b] * geps[a, b] for a, b in uniq)
    assert lhs == pytest.approx(np.sum(G * f) + gE * e, rel=1e-11)
    # unshifted energy depends on sigma/r only: sum sigma dE/dsigma = W
    _, e0, w0 = oracle.lj_forces(pos, box, RC, eps, sig, types, 0)
    _, _, gsig = oracle.lj_vjp(pos, box, RC, np.zeros_like(pos), 1.0, eps, sig, types, 0)
    assert sum(sig[a, b] * gsig[a, b] for a, b in uniq) == pytest.approx(w0, rel=1e-11)


# ---------------------------------------------- generator, thermostat, FENE

def test_philox_known_answers():
    for line in open(os.path.join(GOLDEN, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        out = oracle.philox4x32_10(w[0:4], w[4:6])
        assert list(out) == w[6:10]


def test_gaussian_deviates_statistics():
    g = np.array([oracle.gauss3(7, s, i) for s in range(40) for i in range(250)]).ravel()
    assert abs(g.mean()) < 0.03
    assert abs(g.var() - 1.0) < 0.04
    assert abs(np.mean(np.abs(g) < 1.0) - 0.682689) < 0.015
    # deterministic in (seed, step, id), different across each of them
    assert np.array_equal(oracle.gauss3(7, 3, 5), oracle.gauss3(7, 3, 5))
    assert not np.array_equal(oracle.gauss3(7, 3, 5), oracle.gauss3(8, 3, 5))
    assert not np.array_equal(oracle.gauss3(7, 3, 5), oracle.gauss3(7, 4, 5))
    assert not np.array_equal(oracle.gauss3(7, 3, 5), oracle.gauss3(7, 3, 6))


def test_langevin_limits():
    rng = np.random.default_rng(0)
    v = rng.normal(size=(3000, 3))
    ids = np.arange(3000)
    f = oracle.langevin_forces(v, ids, 0.5, 0.0, 0.005, 1, 0)
    np.testing.assert_allclose(f, -0.5 * v, rtol=1e-15)
    f0 = oracle.langevin_forces(v, ids, 0.0, 1.0, 0.005, 1, 0)
    np.testing.assert_array_equal(f0, np.zeros_like(v))
    gamma, T, dt = 0.5, 1.0, 0.005
    f = oracle.langevin_forces(v, ids, gamma, T, dt, 1, 0)
    xi = (f + gamma * v) / math.sqrt(2 * gamma * T / dt)
    assert abs(xi.var() - 1.0) < 0.06


def test_fene_closed_form_and_bond_balance():
    K, R0 = 30.0, 1.5
    u, fr, ok = oracle.fene_pair(0.5 * R0 * R0, K, R0)
    assert ok
    assert u == pytest.approx(-0.5 * K * R0 * R0 * math.log(0.5), rel=1e-14)
    assert fr == pytest.approx(-2.0 * K, rel=1e-14)
    assert not oracle.fene_pair(R0 * R0, K, R0)[2]
    assert not oracle.fene_pair(1.1 * R0 * R0, K, R0)[2]
    # purely repulsive LJ (rc = 2^(1/6)) plus FENE balance at r = 0.96090
    wca = 2.0 ** (1.0 / 6.0)

    def net(r):
        return oracle.lj_pair(r * r, 1.0, 1.0, wca, 1)[1] + oracle.fene_pair(r * r, K, R0)[1]

    lo, hi = 0.9, 1.0
    assert net(lo) > 0 > net(hi)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if net(mid) > 0 else (lo, mid)
    assert abs(lo - 0.96090) < 5e-5


def test_fene_forces_sum_and_broken_count():
    box = np.array([10.0, 10.0, 10.0])
    pos = np.array([[0.2, 5, 5], [9.4, 5, 5], [9.4, 6.0, 5], [3, 3, 3], [3, 3, 4.6]])
    bonds = np.array([[0, 1], [1, 2], [3, 4]])
    f, e, w, broken = oracle.fene_forces(pos, box, bonds)
    assert broken == 1  # 1.6 > R0
    assert np.abs(f.sum(axis=0)).max() < 1e-12
    u1, fr1, _ = oracle.fene_pair(0.8 ** 2)
    u2, fr2, _ = oracle.fene_pair(1.0)
    assert e == pytest.approx(u1 + u2, rel=1e-14)
    # bond 0-1 crosses the x face: d = x0 - x1 = +0.8, attractive pulls 0 to -x
    assert f[0, 0] == pytest.approx(fr1 * 0.8, rel=1e-14)


# ------------------------------------------------------ cosine angle term

def test_angle_closed_forms():
    K = 1.5
    # straight triple: U = K (1 + cos pi) = 0, no force
    u, fa, fc, ok = oracle.angle_triple([1.1, 0, 0], [-0.9, 0, 0], K)
    assert ok and u == pytest.approx(0.0, abs=1e-15)
    assert np.abs(fa).max() < 1e-15 and np.abs(fc).max() < 1e-15
    # right angle, a on +x at r1 and c on +y at r2: U = K; -grad U opens the
    # angle: F_a = -(K / r1) y, F_c = -(K / r2) x
    r1, r2 = 1.2, 0.9
    u, fa, fc, ok = oracle.angle_triple([r1, 0, 0], [0, r2, 0], K)
    assert u == pytest.approx(K, rel=1e-15)
    np.testing.assert_allclose(fa, [0.0, -K / r1, 0.0], rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(fc, [-K / r2, 0.0, 0.0], rtol=1e-15, atol=1e-16)
    # 120 degrees: cos = -1/2, U = K / 2; |F_a| = K sin(t) / r1
    t = 2.0 * math.pi / 3.0
    u, fa, fc, ok = oracle.angle_triple([r1, 0, 0], [r2 * math.cos(t), r2 * math.sin(t), 0], K)
    assert u == pytest.approx(0.5 * K, rel=1e-14)
    assert np.linalg.norm(fa) == pytest.approx(K * math.sin(t) / r1, rel=1e-14)
    assert np.linalg.norm(fc) == pytest.approx(K * math.sin(t) / r2, rel=1e-14)
    # folded onto itself: U = 2K, a stationary point (no force)
    u, fa, fc, ok = oracle.angle_triple([1.0, 0, 0], [0.7, 0, 0], K)
    assert u == pytest.approx(2.0 * K, rel=1e-15)
    assert np.abs(fa).max() < 1e-15 and np.abs(fc).max() < 1e-15
    # a zero-length bond vector is reported, not evaluated
    assert not oracle.angle_triple([0, 0, 0], [1.0, 0, 0], K)[3]


def test_angle_forces_are_minus_the_gradient_and_conserve_momentum():
    rng = np.random.default_rng(11)
    K, h = 1.5, 1e-6
    for _ in range(20):
        d1 = rng.normal(size=3)
        d2 = rng.normal(size=3)
        u, fa, fc, ok = oracle.angle_triple(d1, d2, K)
        assert ok
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            # moving a shifts d1, moving c shifts d2; moving b shifts both
            ga = (oracle.angle_triple(d1 + e, d2, K)[0] - oracle.angle_triple(d1 - e, d2, K)[0]) / (2 * h)
            gc = (oracle.angle_triple(d1, d2 + e, K)[0] - oracle.angle_triple(d1, d2 - e, K)[0]) / (2 * h)
            gb = (oracle.angle_triple(d1 - e, d2 - e, K)[0]
                  - oracle.angle_triple(d1 + e, d2 + e, K)[0]) / (2 * h)
            assert fa[k] == pytest.approx(-ga, abs=1e-8)
            assert fc[k] == pytest.approx(-gc, abs=1e-8)
            assert -(fa[k] + fc[k]) == pytest.approx(-gb, abs=1e-8)
        # rotation invariance: no torque about the middle bead; the term is
        # scale invariant, so its virial d1.F_a + d2.F_c vanishes
        assert np.abs(np.cross(d1, fa) + np.cross(d2, fc)).max() < 1e-13
        assert abs(d1 @ fa + d2 @ fc) < 1e-13


def test_angle_forces_minimum_image_and_sums():
    box = np.array([6.0, 7.0, 8.0])
    rng = np.random.default_rng(12)
    # three beads of a bent triple whose bonds cross the x and z faces
    base = np.array([[5.6, 3.0, 7.7], [0.3, 3.4, 7.9], [0.6, 4.3, 0.5]])
    tri = np.array([[0, 1, 2]])
    f, e, w, bad = oracle.angle_forces(base, box, tri)
    unwrapped = base + np.array([[0, 0, 0], [6.0, 0, 0], [6.0, 0, 8.0]])
    d1, d2 = unwrapped[0] - unwrapped[1], unwrapped[2] - unwrapped[1]
    u, fa, fc, _ = oracle.angle_triple(d1, d2)
    assert bad == 0 and e == pytest.approx(u, rel=1e-14)
    np.testing.assert_allclose(f[0], fa, rtol=1e-14)
    np.testing.assert_allclose(f[2], fc, rtol=1e-14)
    np.testing.assert_allclose(f[1], -(fa + fc), rtol=1e-14)
    # a ring: total force zero, virial zero, energy = sum of the triples
    cfg = md_inputs.lattice_rings((4, 8, 8), block=(2, 4, 4))
    pos = cfg.pos + rng.normal(scale=0.05, size=cfg.pos.shape)
    f, e, w, bad = oracle.angle_forces(pos, cfg.box[0], cfg.angles)
    assert bad == 0
    assert np.abs(f.sum(axis=0)).max() < 1e-12 and abs(w) < 1e-12
    ref = sum(oracle.angle_triple(pos[a] - pos[b], pos[c] - pos[b])[0] for a, b, c in cfg.angles)
    assert e == pytest.approx(ref, rel=1e-13)


# ------------------------------------------- MD with bonds and a thermostat

def test_md_run_ext_reduces_to_nve_run():
    pos, vel, box = _small_md()
    a = oracle.md_run(pos, vel, box, RC, SKIN, 0.005, 25)
    b = oracle.md_run_ext(pos, vel, box, RC, SKIN, 0.005, 25)
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
    assert np.array_equal(a["rebuild"], b["rebuild"])
    assert np.array_equal(a["epot"], b["epot"]) and np.array_equal(a["ekin"], b["ekin"])


def test_bonded_nve_conserves_energy_with_dt_squared_error():
    # purely repulsive LJ + FENE chains on a lattice path, no thermostat
    cfg = md_inputs.lattice_chains((6, 6, 10), 20, seed=5, temperature=1.0)
    fl = []
    for dt, steps in ((0.004, 100), (0.002, 200)):
        r = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, dt, steps,
                              bonds=cfg.bonds)
        assert r["broken"] == 0
        etot = r["epot"] + r["ekin"]
        fl.append(np.sqrt(np.mean((etot - etot.mean()) ** 2)))
        assert np.abs(r["vel"].sum(axis=0)).max() < 1e-10     # bonds conserve momentum
    assert 3.0 < fl[0] / fl[1] < 5.2


def test_ring_melt_nve_conserves_energy_with_dt_squared_error():
    # purely repulsive LJ + FENE + cosine angle term on rings, no thermostat
    cfg = md_inputs.lattice_rings((4, 8, 8), block=(2, 4, 4), seed=9, temperature=1.0)
    assert cfg.n == 256 and cfg.angles.shape == (256, 3)
    fl = []
    for dt, steps in ((0.004, 100), (0.002, 200)):
        r = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, dt, steps,
                              bonds=cfg.bonds, angles=cfg.angles)
        assert r["broken"] == 0
        etot = r["epot"] + r["ekin"]
        fl.append(np.sqrt(np.mean((etot - etot.mean()) ** 2)))
        assert np.abs(r["vel"].sum(axis=0)).max() < 1e-10
    assert 3.0 < fl[0] / fl[1] < 5.2
    # the angle term is in the potential energy: it starts at K per corner
    r0 = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, 0.004, 0,
                           bonds=cfg.bonds)
    r1 = oracle.md_run_ext(cfg.pos, cfg.vel, cfg.box[0], cfg.rc, cfg.skin, 0.004, 0,
                           bonds=cfg.bonds, angles=cfg.angles)
    corners = sum(1 for a, b, c in cfg.angles
                  if abs((cfg.pos[a] - cfg.pos[b]) @ (cfg.pos[c] - cfg.pos[b])) < 1e-9)
    assert r1["epot"][0] - r0["epot"][0] == pytest.approx(1.5 * corners, rel=1e-12)


def test_broken_bond_is_counted():
    box = np.array([10.0, 10.0, 10.0])
    pos = np.array([[1.0, 1.0, 1.0], [2.6, 1.0, 1.0]])    # 1.6 > R0 = 1.5
    r = oracle.md_run_ext(pos, np.zeros((2, 3)), box, 2 ** (1 / 6), 0.4, 0.001, 1,
                          bonds=np.array([[0, 1]]))
    assert r["broken"] >= 1


def test_langevin_thermostat_reaches_target_temperature():
    pos, box = md_inputs.fcc_lattice(4, 0.8442)
    vel = md_inputs.maxwell_velocities(pos.shape[0], 0.3, seed=2)
    target = 1.2
    r = oracle.md_run_ext(pos, vel, box, RC, SKIN, 0.005, 1600, gamma=1.0,
                          temperature=target, seed=11)
    n = pos.shape[0]
    tkin = 2.0 * r["ekin"][800:] / (3 * n)
    assert abs(tkin.mean() - target) < 0.08 * target


# ------------------------------------------------ all-thread timing build

def test_timing_build_runs_the_same_trajectory():
    # liborc_omp.so (the all-core CPU baseline) splits the pair search and
    # the force sum over threads: same pairs, same per-pair arithmetic, only
    # the summation order of forces, energy and virial differs
    cfg = md_inputs.lj_fluid(8, temperature=1.0, seed=17)
    a = oracle.md_run(cfg.pos, cfg.vel, cfg.box[0], RC, SKIN, cfg.dt, 30)
    b = oracle.md_run(cfg.pos, cfg.vel, cfg.box[0], RC, SKIN, cfg.dt, 30, omp=True)
    assert np.array_equal(a["rebuild"], b["rebuild"]) and a["rebuild"].any()
    assert np.abs(a["pos"] - b["pos"]).max() < 1e-11
    np.testing.assert_allclose(b["epot"], a["epot"], rtol=1e-12)
    np.testing.assert_allclose(b["virial"], a["virial"], rtol=1e-12)
    np.testing.assert_allclose(b["ekin"], a["ekin"], rtol=1e-12)
