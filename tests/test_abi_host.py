"""CPU-side checks of the C ABI: the library loads, exports every function
that include/md.h declares, and validates arguments on the host (no GPU
work is enqueued by any call here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2109_10876_amd import _abi as abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "md.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(md_[a-z_0-9]+)\s*\(",
                                 src, flags=re.M)))


def test_header_and_binding_agree():
    assert set(_declared()) == set(abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.md_abi_version() == abi.MD_ABI_VERSION


def test_header_constants_match_binding():
    src = open(os.path.join(ROOT, "include", "md.h")).read()
    for name in ("MD_ABI_VERSION", "MD_OK", "MD_EINVAL", "MD_EBOX", "MD_ENOWS", "MD_EUNSUPPORTED", "MD_EHIP",
                 "MD_ERANGE", "MD_HALF", "MD_FULL", "MD_FP64", "MD_FP32_MIXED",
                 "MD_UNIT_ATOMS", "MD_IDX_BITS", "MD_MAX_TYPES", "MD_TILE_FULL",
                 "MD_TILE_SLOTS", "MD_TILE_MAX_CELLS", "MD_TILE_MAX_ROWS", "MD_TILE_MAX_TYPES",
                 "MD_TUNE_PAIR_BATCH", "MD_TUNE_TILE_THREADS", "MD_TUNE_TILE_STAGE_PACKED",
                 "MD_TUNE_TILE_SLOTS", "MD_MAX_BONDS", "MD_MAX_ANGLES", "MD_BY_ID",
                 "MD_BY_INDEX", "MD_ESCRATCH"):
        m = re.search(rf"#define\s+{name}\s+(-?\w+)", src)
        assert m, name
        assert int(m.group(1), 0) == getattr(abi, name), name


def test_tile_plan():
    lib = abi.load()
    ncell = np.array([38, 38, 38, 2, 3, 5], np.int32)
    n = lib.md_tile_plan(2, ncell.ctypes.data, 10, None, 1, 1, None, None)
    assert n == 38 * 38 * 4 + 3 * 5 * 1
    rep = np.zeros(n, np.int32)
    off = np.zeros(3, np.int32)
    assert lib.md_tile_plan(2, ncell.ctypes.data, 10, None, 1, 1, rep.ctypes.data,
                            off.ctypes.data) == n
    assert list(off) == [0, 5776, 5791] and rep[5775] == 0 and rep[5776] == 1
    # 2 x 2 rows per tile: 19 x 19 row blocks; odd counts leave a short block
    assert lib.md_tile_plan(2, ncell.ctypes.data, 3, None, 2, 2, None, None) == \
        13 * 19 * 19 + 1 * 2 * 3
    assert lib.md_tile_plan(2, ncell.ctypes.data, 0, None, 1, 1, None, None) == abi.MD_EINVAL
    assert lib.md_tile_plan(2, ncell.ctypes.data, 65, None, 1, 1, None, None) == abi.MD_EINVAL
    assert lib.md_tile_plan(2, ncell.ctypes.data, 4, None, 3, 1, None, None) == abi.MD_EINVAL


def test_tile_plan_per_replica_widths():
    # replica r cut into tiles of m_r cells along x; each m_r in 1 .. tile_cells
    lib = abi.load()
    ncell = np.array([38, 38, 38, 2, 3, 5], np.int32)
    m = np.array([3, 1], np.int32)
    n = lib.md_tile_plan(2, ncell.ctypes.data, 3, m.ctypes.data, 2, 2, None, None)
    assert n == 13 * 19 * 19 + 2 * 2 * 3
    rep = np.zeros(n, np.int32)
    off = np.zeros(3, np.int32)
    assert lib.md_tile_plan(2, ncell.ctypes.data, 3, m.ctypes.data, 2, 2, rep.ctypes.data,
                            off.ctypes.data) == n
    assert list(off) == [0, 13 * 19 * 19, n] and np.all(rep[off[1]:] == 1)
    for bad in ([4, 1], [3, 0]):
        mb = np.array(bad, np.int32)
        assert lib.md_tile_plan(2, ncell.ctypes.data, 3, mb.ctypes.data, 2, 2, None,
                                None) == abi.MD_EINVAL


def test_tuning_knobs():
    lib = abi.load()
    assert lib.md_tune_get(abi.MD_TUNE_PAIR_BATCH) == 4
    for v in (1, 2, 8, 4):
        assert lib.md_tune_set(abi.MD_TUNE_PAIR_BATCH, v) == abi.MD_OK
        assert lib.md_tune_get(abi.MD_TUNE_PAIR_BATCH) == v
    assert lib.md_tune_set(abi.MD_TUNE_PAIR_BATCH, 3) == abi.MD_EINVAL
    assert lib.md_tune_get(abi.MD_TUNE_TILE_THREADS) == 256
    assert lib.md_tile_capacity() == abi.MD_TILE_SLOTS
    assert lib.md_tile_max_cells() == abi.MD_TILE_MAX_CELLS
    for tb, cap, mc in ((64, 1024, 8), (128, 1792, 16), (256, 3072, 64)):
        assert lib.md_tune_set(abi.MD_TUNE_TILE_THREADS, tb) == abi.MD_OK
        assert lib.md_tile_capacity() == cap and lib.md_tile_max_cells() == mc
    # smaller staged capacity at 256 threads (less LDS per workgroup)
    for slots, cap, mc in ((2048, 2048, 16), (1536, 1536, 8), (3072, 3072, 64), (0, 3072, 64)):
        assert lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, slots) == abi.MD_OK
        assert lib.md_tile_capacity() == cap and lib.md_tile_max_cells() == mc
    assert lib.md_tune_set(abi.MD_TUNE_TILE_SLOTS, 1000) == abi.MD_EINVAL
    assert lib.md_tune_get(abi.MD_TUNE_TILE_SLOTS) == 0
    assert lib.md_tune_set(abi.MD_TUNE_TILE_THREADS, 96) == abi.MD_EINVAL
    assert lib.md_tune_set(abi.MD_TUNE_TILE_STAGE_PACKED, 2) == abi.MD_EINVAL
    assert lib.md_tune_set(99, 1) == abi.MD_EINVAL
    assert lib.md_tune_get(99) == abi.MD_EINVAL


def _plan(natoms, box, rc=2.5, skin=0.3):
    lib = abi.load()
    natoms = np.asarray(natoms, np.int32)
    box = np.asarray(box, np.float64).reshape(-1, 3)
    N, C, U = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    code = lib.md_plan_sizes(len(natoms), natoms.ctypes.data, box.ctypes.data, rc, skin,
                             ctypes.byref(N), ctypes.byref(C), ctypes.byref(U))
    return code, N.value, C.value, U.value


def test_plan_single_system():
    # 1,048,576 atoms in a 107.494 box: 38 cells of edge >= 2.8 per dimension
    L = (1048576 / 0.8442) ** (1 / 3)
    code, N, C, U = _plan([1048576], [L, L, L])
    assert code == abi.MD_OK
    assert (N, C, U) == (1048576, 38 ** 3, 4096)


def test_plan_fill_batch():
    lib = abi.load()
    natoms = np.array([500, 257, 3000], np.int32)
    box = np.array([[8.5, 8.5, 8.5], [7.0, 6.0, 5.7], [15.2, 15.2, 15.2]])
    code, N, C, U = _plan(natoms, box)
    assert code == abi.MD_OK and N == 3757 and U == 2 + 2 + 12
    ao, co, uo = (np.zeros(4, np.int32) for _ in range(3))
    nc = np.zeros(9, np.int32)
    ur = np.zeros(U, np.int32)
    assert lib.md_plan_fill(3, natoms.ctypes.data, box.ctypes.data, 2.5, 0.3, ao.ctypes.data,
                            co.ctypes.data, nc.ctypes.data, ur.ctypes.data,
                            uo.ctypes.data) == abi.MD_OK
    assert list(ao) == [0, 500, 757, 3757]
    assert list(nc) == [3, 3, 3, 2, 2, 2, 5, 5, 5]
    assert list(co) == [0, 27, 35, 160] and C == 160
    assert list(uo) == [0, 2, 4, 16]
    assert list(ur) == [0, 0, 1, 1] + [2] * 12


@pytest.mark.parametrize("natoms,box,rc,skin,code", [
    ([100], [5.5, 8, 8], 2.5, 0.3, abi.MD_EBOX),      # L < 2 (rc + skin)
    ([0], [8, 8, 8], 2.5, 0.3, abi.MD_EINVAL),        # empty replica
    ([10], [8, 8, 8], -1.0, 0.3, abi.MD_EINVAL),      # negative cutoff
    ([10], [8, -8, 8], 2.5, 0.3, abi.MD_EINVAL),      # negative box
    ([1 << 26], [500, 500, 500], 2.5, 0.3, abi.MD_ERANGE),
])
def test_plan_rejects(natoms, box, rc, skin, code):
    assert _plan(natoms, box, rc, skin)[0] == code


def test_calls_reject_bad_arguments_without_a_gpu():
    lib = abi.load()
    P = ctypes.byref
    bad = abi.MdBatch()   # R = 0
    atoms, nl, lj = abi.MdAtoms(), abi.MdNlist(), abi.MdLj()
    assert lib.md_cell_sort(P(bad), P(atoms), P(atoms), None, None, 0, None, None, None) == abi.MD_EINVAL
    assert lib.md_verlet_build(P(bad), P(atoms), None, 2.5, 0.3, P(nl), None, None, None, None) == abi.MD_EINVAL
    assert lib.md_lj_forces(P(bad), P(atoms), P(nl), P(lj), 0, 0, None, None, None, 0, None, None) == abi.MD_EINVAL
    assert lib.md_vv_step(P(bad), P(atoms), 1, 0.005, None, 1, 0.3, None, None, None, None, 0,
                          None, None) == abi.MD_EINVAL
    assert lib.md_lj_forces_vjp(P(bad), P(atoms), P(nl), P(lj), 0, None, None, None, None, None,
                                None, None, None, 0, None, None) == abi.MD_EINVAL
    assert lib.md_workspace_bytes(P(bad)) == 0
    # a well-formed batch (fake device pointers) still fails on missing arrays,
    # on bad modes and on a short workspace, before anything is launched
    ok = abi.MdBatch(1, 1000, 27, 4, 8, 8, 8, 8, 8, 8)
    assert lib.md_workspace_bytes(P(ok)) > 0
    nl = abi.MdNlist(7, 64, 1024, 0, 8, 8, 0, 1, 1, 0, None, None, None, None)
    assert lib.md_verlet_build(P(ok), P(atoms), 8, 2.5, 0.3, P(nl), None, None, None, None) == abi.MD_EINVAL
    full = abi.MdAtoms(*([8] * 17))
    nl = abi.MdNlist(abi.MD_HALF, 64, 1000, 0, 8, 8, 0, 1, 1, 0, None, None, None, None)   # ld % 64
    lj1 = abi.MdLj(1, 1, 2.5, 8, 8)
    assert lib.md_lj_forces(P(ok), P(full), P(nl), P(lj1), 0, 0, None, None, 8, 1 << 30, None, None) == abi.MD_EINVAL
    nl = abi.MdNlist(abi.MD_HALF, 64, 1024, 0, 8, 8, 0, 1, 1, 0, None, None, None, None)
    assert lib.md_lj_forces(P(ok), P(full), P(nl), P(lj1), 5, 0, None, None, 8, 1 << 30, None, None) == abi.MD_EINVAL
    assert lib.md_lj_forces(P(ok), P(full), P(nl), P(lj1), 0, 0, None, None, 8, 16, None, None) == abi.MD_ENOWS
    assert lib.md_lj_forces_vjp(P(ok), P(full), P(nl), P(lj1), 0, 8, 8, 8, None, 8, None, None,
                                8, 1 << 30, None, None) == abi.MD_EUNSUPPORTED
    assert lib.md_vv_step(P(ok), P(full), 4, 0.005, 8, 1, 0.3, 8, None, None, 8, 1 << 30, None,
                          None) == abi.MD_EINVAL
    # a thermostat only with the phases that kick with the force, and complete
    th = abi.MdThermostat(0.5, 1.0, 7, 8, 8)
    assert lib.md_vv_step(P(ok), P(full), 1, 0.005, 8, 1, 0.3, 8, None, P(th), 8, 1 << 30, None,
                          None) == abi.MD_EINVAL
    for bad_th in (abi.MdThermostat(0.5, 1.0, 7, None, 8), abi.MdThermostat(0.5, 1.0, 7, 8, None),
                   abi.MdThermostat(-1.0, 1.0, 7, 8, 8), abi.MdThermostat(0.5, -1.0, 7, 8, 8)):
        assert lib.md_vv_step(P(ok), P(full), 3, 0.005, 8, 1, 0.3, 8, None, P(bad_th), 8,
                              1 << 30, None, None) == abi.MD_EINVAL


def test_angle_forces_reject_bad_arguments_without_a_gpu():
    lib = abi.load()
    P = ctypes.byref
    ok = abi.MdBatch(1, 1000, 27, 4, 8, 8, 8, 8, 8, 8)
    full = abi.MdAtoms(*([8] * 17))
    ang = abi.MdAngles(3, 0, 8, 8)
    big = 1 << 30
    assert lib.md_angle_forces(P(abi.MdBatch()), P(full), P(ang), 1.5, None, None, 8, big,
                               None, None) == abi.MD_EINVAL
    assert lib.md_angle_forces(P(ok), P(full), None, 1.5, None, None, 8, big,
                               None, None) == abi.MD_EINVAL
    for m in (0, abi.MD_MAX_ANGLES + 1):
        assert lib.md_angle_forces(P(ok), P(full), P(abi.MdAngles(m, 0, 8, 8)), 1.5, None, None,
                                   8, big, None, None) == abi.MD_EINVAL
    assert lib.md_angle_forces(P(ok), P(full), P(abi.MdAngles(3, 0, 8, None)), 1.5, None, None,
                               8, big, None, None) == abi.MD_EINVAL
    for K in (-1.0, float("inf"), float("nan")):
        assert lib.md_angle_forces(P(ok), P(full), P(ang), K, None, None, 8, big,
                                   None, None) == abi.MD_EINVAL
    assert lib.md_angle_forces(P(ok), P(full), P(ang), 1.5, None, None, 8, 16,
                               None, None) == abi.MD_ENOWS


def test_noalloc_forces_check_arguments_and_scratch_size_without_a_gpu():
    # everything md_lj_forces checks, then the fixed scratch size, all on the
    # host before the scratch array is looked up on a device
    lib = abi.load()
    P = ctypes.byref
    full = abi.MdAtoms(*([8] * 17))
    lj1 = abi.MdLj(1, 1, 2.5, 8, 8)
    nl = abi.MdNlist(abi.MD_FULL, 64, 1024, 0, 8, 8, 0, 1, 1, 0, None, None, None, None)
    assert lib.md_lj_forces_noalloc(P(abi.MdBatch()), P(full), P(nl), P(lj1), 0, 0, None, None,
                                    None, None) == abi.MD_EINVAL
    ok = abi.MdBatch(1, 1000, 27, 4, 8, 8, 8, 8, 8, 8)
    assert lib.md_lj_forces_noalloc(P(ok), P(full), P(nl), P(lj1), 5, 0, None, None, None,
                                    None) == abi.MD_EINVAL
    assert lib.md_lj_forces_noalloc(P(ok), None, P(nl), P(lj1), 0, 0, None, None, None,
                                    None) == abi.MD_EINVAL
    # 32 bytes per work unit (and per tile): 2^18 rows fit, one more does not
    rows = abi.MD_NOALLOC_SCRATCH_BYTES // 32
    n = abi.MD_MAX_ATOMS // 64 * 64   # ld a multiple of 64; two replicas give rows + 1 units
    nlb = abi.MdNlist(abi.MD_FULL, 64, n, 0, 8, 8, 0, 1, 1, 0, None, None, None, None)
    big = abi.MdBatch(2, n, 54, rows + 1, 8, 8, 8, 8, 8, 8)
    assert lib.md_lj_forces_noalloc(P(big), P(full), P(nlb), P(lj1), 0, 0, None, None, None,
                                    None) == abi.MD_ESCRATCH
    # tile lists add one row per tile
    cap = lib.md_tile_capacity()
    nt, nu = rows - 32767, 32768   # tile lists: ld <= 2^23 atoms
    tl = abi.MdNlist(abi.MD_TILE_FULL, 64, 1 << 23, 1, 16, 16, nt, 1, 1, 0, 16, 16, None, 16,
                     cap, 0, 16)
    tb = abi.MdBatch(1, 1 << 23, nt, nu, 8, 8, 8, 8, 8, 8)
    assert lib.md_lj_forces_noalloc(P(tb), P(full), P(tl), P(lj1), 0, 0, None, None, None,
                                    None) == abi.MD_ESCRATCH
    assert "scratch" in abi.strerror(abi.MD_ESCRATCH)


def test_kernel_timing_arguments_and_empty_read():
    # no launch is timed on the host: start and an empty read touch no GPU
    import ctypes
    lib = abi.load()
    assert lib.md_kernel_timing_start(-1) == abi.MD_EINVAL
    assert lib.md_kernel_timing_start(1025) == abi.MD_EINVAL
    assert lib.md_kernel_timing_start(0) == abi.MD_OK
    ms, n = ctypes.c_double(-1.0), ctypes.c_int32(-1)
    assert lib.md_kernel_timing_read(ctypes.byref(ms), ctypes.byref(n)) == abi.MD_OK
    assert n.value == 0 and ms.value == 0.0
    assert lib.md_kernel_timing_read(None, ctypes.byref(n)) == abi.MD_EINVAL


def test_copy_probe_rejects_bad_arguments_without_a_gpu():
    lib = abi.load()
    buf = (ctypes.c_double * 8)()
    p = ctypes.addressof(buf)
    assert lib.md_copy_probe(None, p, 16, None) == abi.MD_EINVAL
    assert lib.md_copy_probe(p, None, 16, None) == abi.MD_EINVAL
    assert lib.md_copy_probe(p, p + 16, 0, None) == abi.MD_EINVAL
    assert lib.md_copy_probe(p, p + 16, 24, None) == abi.MD_EINVAL
    assert lib.md_copy_probe(p + 8, p + 32, 16, None) == abi.MD_EINVAL


def test_tile_list_needs_a_staging_table_of_the_current_capacity():
    # rejected on the host before anything is launched (fake device pointers)
    lib = abi.load()
    P = ctypes.pointer
    ok = abi.MdBatch(1, 1000, 27, 4, 8, 8, 8, 8, 8, 8)
    full = abi.MdAtoms(*([8] * 17))
    cap = lib.md_tile_capacity()

    def nl(src, src_cap):
        return abi.MdNlist(abi.MD_TILE_FULL, 64, 1024, 1, 16, 16, 1, 1, 1, 0, 16, 16, None, 16,
                           src_cap, 0, src)

    for bad in (nl(None, cap), nl(16, cap + 1), nl(16, 0)):
        assert lib.md_verlet_build(P(ok), P(full), 16, 2.5, 0.3, P(bad), None, None, None,
                                   None) == abi.MD_EINVAL
    # the occupied-tile list covers one replica only
    two = abi.MdBatch(2, 1000, 27, 4, 8, 8, 8, 8, 8, 8)
    listed = abi.MdNlist(abi.MD_TILE_FULL, 64, 1024, 1, 16, 16, 1, 1, 1, 0, 16, 16, None, 16,
                         cap, 0, 16, 16)
    lj1 = abi.MdLj(1, 1, 2.5, 8, 8)
    assert lib.md_verlet_build(P(two), P(full), 16, 2.5, 0.3, P(listed), None, None, None,
                               None) == abi.MD_EINVAL
    assert lib.md_lj_forces(P(two), P(full), P(listed), P(lj1), 0, 0, None, None, 8, 1 << 30,
                            None, None) == abi.MD_EINVAL


def test_fused_step_next_position_buffers_are_checked():
    # all three or none, no overlap with the current planes, no packed copy;
    # rejected on the host before anything is launched (fake device pointers)
    lib = abi.load()
    P = ctypes.pointer
    ok = abi.MdBatch(1, 1000, 27, 4, 8, 8, 8, 8, 8, 8)
    cap = lib.md_tile_capacity()
    nl = abi.MdNlist(abi.MD_TILE_FULL, 64, 1024, 1, 16, 16, 1, 1, 1, 0, 16, 16, None, 16,
                     cap, 0, 16)
    lj1 = abi.MdLj(1, 1, 2.5, 8, 8)
    X, Y, Z = 1 << 20, 2 << 20, 3 << 20
    atoms = abi.MdAtoms(X, Y, Z, *([8] * 13), None)
    packed = abi.MdAtoms(X, Y, Z, *([8] * 13), 8)
    far = 16 << 20

    def call(a, xn, yn, zn, thermo=None, gate_clear=None):
        return lib.md_lj_forces_vv(P(ok), P(a), P(nl), P(lj1), 0, 0.005, 8, 1, 0.3, 8,
                                   gate_clear, None, None, None, xn, yn, zn,
                                   P(thermo) if thermo else None, 8, 1 << 30, None, None)

    assert call(atoms, far, None, None) == abi.MD_EINVAL             # not all three
    assert call(atoms, X + 8 * 500, far, far + (1 << 20)) == abi.MD_EINVAL   # overlaps x
    assert call(atoms, far, far + (1 << 20), Z) == abi.MD_EINVAL     # overlaps z
    assert call(packed, far, far + (1 << 20), far + (2 << 20)) == abi.MD_EINVAL  # pos4 set
    # a thermostat needs its counter and masses, gamma >= 0 and T >= 0
    nxt = (far, far + (1 << 20), far + (2 << 20))
    for th in (abi.MdThermostat(0.5, 1.0, 7, None, 8), abi.MdThermostat(0.5, 1.0, 7, 8, None),
               abi.MdThermostat(-0.5, 1.0, 7, 8, 8), abi.MdThermostat(0.5, -1.0, 7, 8, 8),
               abi.MdThermostat(float("nan"), 1.0, 7, 8, 8)):
        assert call(atoms, *nxt, thermo=th) == abi.MD_EINVAL
    # alternating gate words: not overlapping the gate, not with a thermostat
    assert call(atoms, *nxt, gate_clear=8) == abi.MD_EINVAL
    assert call(atoms, *nxt, gate_clear=16 << 10,
                thermo=abi.MdThermostat(0.5, 1.0, 7, 8, 8)) == abi.MD_EINVAL


def test_bonded_tables_check_their_order_without_a_gpu():
    lib = abi.load()
    P = ctypes.byref
    ok = abi.MdBatch(1, 1000, 27, 4, 8, 8, 8, 8, 8, 8)
    full = abi.MdAtoms(*([8] * 17))
    big = 1 << 30
    for order in (-1, 2):
        assert lib.md_fene_forces(P(ok), P(full), P(abi.MdBonds(2, order, 8, 8)), 30.0, 1.5,
                                  None, None, 8, big, None, None) == abi.MD_EINVAL
        assert lib.md_angle_forces(P(ok), P(full), P(abi.MdAngles(3, order, 8, 8)), 1.5, None,
                                   None, 8, big, None, None) == abi.MD_EINVAL
    # tables keyed by id need where[]; keyed by index they do not (short
    # workspace reached instead, before any launch)
    nowhere = abi.MdAtoms(*([8] * 15), None, 8)
    assert lib.md_fene_forces(P(ok), P(nowhere), P(abi.MdBonds(2, abi.MD_BY_ID, 8, 8)), 30.0,
                              1.5, None, None, 8, big, None, None) == abi.MD_EINVAL
    assert lib.md_fene_forces(P(ok), P(nowhere), P(abi.MdBonds(2, abi.MD_BY_INDEX, 8, 8)), 30.0,
                              1.5, None, None, 8, 16, None, None) == abi.MD_ENOWS
    assert lib.md_angle_forces(P(ok), P(nowhere), P(abi.MdAngles(3, abi.MD_BY_ID, 8, 8)), 1.5,
                               None, None, 8, big, None, None) == abi.MD_EINVAL
    assert lib.md_angle_forces(P(ok), P(nowhere), P(abi.MdAngles(3, abi.MD_BY_INDEX, 8, 8)), 1.5,
                               None, None, 8, 16, None, None) == abi.MD_ENOWS
    # the re-index pass: inputs keyed by id, outputs present, counts in range
    bid = abi.MdBonds(2, abi.MD_BY_ID, 8, 8)
    aid = abi.MdAngles(3, abi.MD_BY_ID, 8, 8)
    assert lib.md_bonded_reindex(P(ok), P(full), None, None, None, None, None, None, None,
                                 None) == abi.MD_OK          # nothing to do, nothing launched
    assert lib.md_bonded_reindex(P(ok), P(nowhere), P(bid), 8, 8, None, None, None, None,
                                 None) == abi.MD_EINVAL
    assert lib.md_bonded_reindex(P(ok), P(full), P(abi.MdBonds(2, abi.MD_BY_INDEX, 8, 8)), 8, 8,
                                 None, None, None, None, None) == abi.MD_EINVAL
    assert lib.md_bonded_reindex(P(ok), P(full), P(bid), 8, None, None, None, None, None,
                                 None) == abi.MD_EINVAL
    assert lib.md_bonded_reindex(P(ok), P(full), P(abi.MdBonds(abi.MD_MAX_BONDS + 1, 0, 8, 8)),
                                 8, 8, None, None, None, None, None) == abi.MD_EINVAL
    assert lib.md_bonded_reindex(P(ok), P(full), None, None, None, P(aid), 8, None, None,
                                 None) == abi.MD_EINVAL
    assert lib.md_bonded_reindex(P(ok), P(full), None, None, None,
                                 P(abi.MdAngles(abi.MD_MAX_ANGLES + 1, 0, 8, 8)), 8, 8, None,
                                 None) == abi.MD_EINVAL
    assert lib.md_bonded_reindex(P(abi.MdBatch()), P(full), P(bid), 8, 8, None, None, None, None,
                                 None) == abi.MD_EINVAL
    # the one-pass bonded call: both tables keyed by index
    bix = abi.MdBonds(2, abi.MD_BY_INDEX, 8, 8)
    aix = abi.MdAngles(3, abi.MD_BY_INDEX, 8, 8)

    def bonded(bb, aa, K=30.0, R0=1.5, Ka=1.5, ws_bytes=big):
        return lib.md_bonded_forces(P(ok), P(full), P(bb) if bb else None, K, R0,
                                    P(aa) if aa else None, Ka, None, None, None, None, 8,
                                    ws_bytes, None, None)

    assert bonded(bid, aix) == abi.MD_EINVAL
    assert bonded(bix, aid) == abi.MD_EINVAL
    assert bonded(None, aix) == abi.MD_EINVAL and bonded(bix, None) == abi.MD_EINVAL
    assert bonded(bix, aix, Ka=-1.0) == abi.MD_EINVAL
    assert bonded(bix, aix, Ka=float("inf")) == abi.MD_EINVAL
    assert bonded(bix, aix, R0=0.0) == abi.MD_EINVAL
    assert bonded(bix, aix, ws_bytes=16) == abi.MD_ENOWS
