"""ctypes binding of libmd's C ABI (``include/md.h``).

Argument marshalling only: every step of the MD path runs in the HIP
kernels of ``libmd.so``.  The library must have been built in-tree
(``paper_2109_10876_amd.build.build_library()``); loading fails loudly
otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmd.so")

# Constants mirrored from md.h.
MD_ABI_VERSION = 11
MD_OK = 0
MD_EINVAL = -1
MD_EBOX = -2
MD_ENOWS = -3
MD_EUNSUPPORTED = -4
MD_EHIP = -5
MD_ERANGE = -6
MD_ESCRATCH = -7
MD_NOALLOC_SCRATCH_BYTES = 8 << 20
MD_F_NBR_OVERFLOW = 0x1
MD_F_NONFINITE = 0x2
MD_F_BOND_BROKEN = 0x4
MD_F_TILE_OVERFLOW = 0x8
MD_HALF = 0
MD_FULL = 1
MD_TILE_FULL = 2
MD_BY_ID = 0
MD_BY_INDEX = 1
MD_TILE_SLOTS = 3072
MD_TILE_MAX_CELLS = 64
MD_TILE_MAX_ROWS = 2
MD_TILE_MAX_TYPES = 4
MD_FP64 = 0
MD_FP32_MIXED = 1
MD_UNIT_ATOMS = 256
MD_IDX_BITS = 26
MD_IDX_MASK = 0x03FFFFFF
MD_MAX_ATOMS = 0x03FFFFFF
MD_MAX_TYPES = 8
MD_MAX_BONDS = 4
MD_MAX_ANGLES = 8
MD_TUNE_PAIR_BATCH = 0
MD_TUNE_TILE_THREADS = 1
MD_TUNE_TILE_STAGE_PACKED = 2
MD_TUNE_TILE_SLOTS = 3

EXPORTS = (
    "md_abi_version", "md_strerror", "md_tune_set", "md_tune_get", "md_tile_capacity",
    "md_tile_max_cells", "md_kernel_timing_start", "md_kernel_timing_read", "md_copy_probe",
    "md_plan_sizes",
    "md_plan_fill",
    "md_tile_plan",
    "md_workspace_bytes", "md_cell_sort", "md_verlet_build", "md_lj_forces",
    "md_lj_forces_noalloc",
    "md_vv_step", "md_lj_forces_vv", "md_lj_forces_vjp", "md_fene_forces", "md_angle_forces",
    "md_bonded_forces", "md_bonded_reindex", "md_langevin",
)

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_dbl = ctypes.c_double


class MdBatch(ctypes.Structure):
    _fields_ = [("R", _i32), ("N", _i32), ("C", _i32), ("n_units", _i32),
                ("atom_off", _vp), ("cell_off", _vp), ("ncell", _vp), ("box", _vp),
                ("unit_rep", _vp), ("unit_off", _vp)]


class MdAtoms(ctypes.Structure):
    _fields_ = [(n, _vp) for n in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz",
                                   "xb", "yb", "zb", "type", "id", "img", "where", "pos4")]


class MdNlist(ctypes.Structure):
    _fields_ = [("mode", _i32), ("max_nbr", _i32), ("ld", _i32), ("tile_cells", _i32),
                ("count", _vp), ("idx", _vp), ("n_tiles", _i32), ("tile_py", _i32),
                ("tile_pz", _i32), ("tile_types", _i32),
                ("tile_rep", _vp), ("tile_off", _vp), ("tile_need", _vp), ("cell_start", _vp),
                ("tile_src_cap", _i32), ("_pad", _i32), ("tile_src", _vp),
                ("tile_active", _vp), ("tile_m", _vp), ("tile_todo", _vp)]


class MdLj(ctypes.Structure):
    _fields_ = [("ntypes", _i32), ("shift", _i32), ("rc", _dbl), ("eps", _vp), ("sig", _vp)]


class MdBonds(ctypes.Structure):
    _fields_ = [("max_bonds", _i32), ("order", _i32), ("count", _vp), ("partner", _vp)]


class MdAngles(ctypes.Structure):
    _fields_ = [("max_angles", _i32), ("order", _i32), ("count", _vp), ("tri", _vp)]


class MdThermostat(ctypes.Structure):
    _fields_ = [("gamma", _dbl), ("temperature", _dbl), ("seed", ctypes.c_uint64),
                ("step", _vp), ("mass", _vp)]


class MDError(RuntimeError):
    """A libmd call returned a negative MD_E* code."""

    def __init__(self, fn, code):
        self.code = code
        super().__init__(f"{fn}: {strerror(code)} (code {code})")


class ListOverflowError(RuntimeError):
    """Steps ran on a Verlet list that had overflowed (MD_F_NBR_OVERFLOW or
    MD_F_TILE_OVERFLOW set after a run): their trajectory is not valid."""


_lib = None


def load():
    """Load libmd.so (built in-tree); raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libmd.so not found at {LIB_PATH}; build it first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.md_abi_version.restype = ctypes.c_int
    lib.md_abi_version.argtypes = []
    lib.md_strerror.restype = ctypes.c_char_p
    lib.md_strerror.argtypes = [ctypes.c_int]
    lib.md_tune_set.restype = ctypes.c_int
    lib.md_tune_set.argtypes = [_i32, _i32]
    lib.md_tune_get.restype = ctypes.c_int
    lib.md_tune_get.argtypes = [_i32]
    lib.md_plan_sizes.restype = ctypes.c_int
    lib.md_plan_sizes.argtypes = [_i32, _vp, _vp, _dbl, _dbl, P(_i32), P(_i32), P(_i32)]
    lib.md_plan_fill.restype = ctypes.c_int
    lib.md_plan_fill.argtypes = [_i32, _vp, _vp, _dbl, _dbl, _vp, _vp, _vp, _vp, _vp]
    lib.md_tile_capacity.restype = ctypes.c_int
    lib.md_tile_capacity.argtypes = []
    lib.md_tile_max_cells.restype = ctypes.c_int
    lib.md_tile_max_cells.argtypes = []
    lib.md_kernel_timing_start.restype = ctypes.c_int
    lib.md_kernel_timing_start.argtypes = [_i32]
    lib.md_kernel_timing_read.restype = ctypes.c_int
    lib.md_kernel_timing_read.argtypes = [P(_dbl), P(_i32)]
    lib.md_copy_probe.restype = ctypes.c_int
    lib.md_copy_probe.argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
    lib.md_tile_plan.restype = ctypes.c_int
    lib.md_tile_plan.argtypes = [_i32, _vp, _i32, _vp, _i32, _i32, _vp, _vp]
    lib.md_workspace_bytes.restype = ctypes.c_size_t
    lib.md_workspace_bytes.argtypes = [P(MdBatch)]
    lib.md_cell_sort.restype = ctypes.c_int
    lib.md_cell_sort.argtypes = [P(MdBatch), P(MdAtoms), P(MdAtoms), _vp, _vp, ctypes.c_size_t,
                                 _vp, _vp, _vp]
    lib.md_verlet_build.restype = ctypes.c_int
    lib.md_verlet_build.argtypes = [P(MdBatch), P(MdAtoms), _vp, _dbl, _dbl, P(MdNlist), _vp,
                                    _vp, _vp, _vp]
    lib.md_lj_forces.restype = ctypes.c_int
    lib.md_lj_forces.argtypes = [P(MdBatch), P(MdAtoms), P(MdNlist), P(MdLj), _i32, _i32,
                                 _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
    lib.md_lj_forces_noalloc.restype = ctypes.c_int
    lib.md_lj_forces_noalloc.argtypes = [P(MdBatch), P(MdAtoms), P(MdNlist), P(MdLj), _i32, _i32,
                                         _vp, _vp, _vp, _vp]
    lib.md_vv_step.restype = ctypes.c_int
    lib.md_vv_step.argtypes = [P(MdBatch), P(MdAtoms), _i32, _dbl, _vp, _i32, _dbl, _vp, _vp,
                               P(MdThermostat), _vp, ctypes.c_size_t, _vp, _vp]
    lib.md_lj_forces_vv.restype = ctypes.c_int
    lib.md_lj_forces_vv.argtypes = [P(MdBatch), P(MdAtoms), P(MdNlist), P(MdLj), _i32, _dbl,
                                    _vp, _i32, _dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                    P(MdThermostat), _vp, ctypes.c_size_t, _vp, _vp]
    lib.md_lj_forces_vjp.restype = ctypes.c_int
    lib.md_lj_forces_vjp.argtypes = [P(MdBatch), P(MdAtoms), P(MdNlist), P(MdLj), _i32,
                                     _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                     _vp, _vp]
    lib.md_fene_forces.restype = ctypes.c_int
    lib.md_fene_forces.argtypes = [P(MdBatch), P(MdAtoms), P(MdBonds), _dbl, _dbl, _vp, _vp,
                                   _vp, ctypes.c_size_t, _vp, _vp]
    lib.md_angle_forces.restype = ctypes.c_int
    lib.md_angle_forces.argtypes = [P(MdBatch), P(MdAtoms), P(MdAngles), _dbl, _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp, _vp]
    lib.md_bonded_forces.restype = ctypes.c_int
    lib.md_bonded_forces.argtypes = [P(MdBatch), P(MdAtoms), P(MdBonds), _dbl, _dbl, P(MdAngles),
                                     _dbl, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
    lib.md_bonded_reindex.restype = ctypes.c_int
    lib.md_bonded_reindex.argtypes = [P(MdBatch), P(MdAtoms), P(MdBonds), _vp, _vp, P(MdAngles),
                                      _vp, _vp, _vp, _vp]
    lib.md_langevin.restype = ctypes.c_int
    lib.md_langevin.argtypes = [P(MdBatch), P(MdAtoms), _vp, _i32, _dbl, _dbl, _dbl,
                                ctypes.c_uint64, _vp, _vp, _vp]
    _lib = lib
    return lib


def strerror(code):
    try:
        return load().md_strerror(int(code)).decode()
    except Exception:  # library missing: still give the code back
        return f"md error {code}"


def check(fn, code):
    if code != MD_OK:
        raise MDError(fn, code)
    return code
