"""Device-resident MD state and the step loop, driving libmd through its C ABI.

PyTorch only allocates device memory and supplies the HIP stream; every
step of the path (re-sort, list build, forces, integration, reductions)
runs in libmd's kernels.  The step follows Fig. 1 of the paper:

    Integrate1 -> [skin test -> Resort + Neigh] -> forces -> Integrate2

with the skin test evaluated on the device (a per-replica gate that the
re-sort and list-build kernels read), so a step never waits for the host.
Consecutive steps fuse Integrate2 of one step with Integrate1 of the next.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _abi as abi
from ._abi import check


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _empty_cell_fraction(pos, box, ncell):
    """Host-side launch planning: the fraction of the cells of one box that
    hold no atom."""
    nc = np.asarray(ncell).astype(np.int64)
    c = np.minimum((np.mod(pos, box) * nc / box).astype(np.int64), nc - 1)
    occ = np.unique((c[:, 2] * nc[1] + c[:, 1]) * nc[0] + c[:, 0]).shape[0]
    return 1.0 - occ / float(np.prod(nc))


def _occupied_cell_density(pos, natoms, box, ncell):
    """Host-side launch planning: mean atoms per non-empty cell of the cell
    grid, per replica."""
    nu, off = [], 0
    for r, n in enumerate(np.asarray(natoms).ravel()):
        n = int(n)
        L, nc = box[r], ncell[r].astype(np.int64)
        c = np.minimum((np.mod(pos[off:off + n], L) * nc / L).astype(np.int64), nc - 1)
        cnt = np.bincount((c[:, 2] * nc[1] + c[:, 1]) * nc[0] + c[:, 0])
        nu.append(max(1.0, float(cnt[cnt > 0].mean())))
        off += n
    return np.array(nu)


def _tile_cells_for(nu, nx, cap, tb, py, pz, max_cells):
    """Cells per tile along x for mean occupancy nu and nx cells per row: the
    staged neighbourhood (m + 2)(py + 2)(pz + 2) nu within 92% of the
    staging capacity and about one home atom per thread, then balanced along
    the row (the paper grows its subnodes until the work per core stops
    paying, Sec. 3.3; here the LDS staging bounds the tile)."""
    m = int(min(0.92 * cap / ((py + 2) * (pz + 2) * nu) - 2, 1.02 * tb / (py * pz * nu)))
    m = max(1, min(m, max_cells, nx))
    return -(-nx // -(-nx // m))


class MDSystem:
    """R independent periodic LJ systems, concatenated, resident on one GPU.

    Parameters mirror a workload description: per-replica atom counts and
    boxes, initial positions/velocities [N,3] (replicas concatenated), atom
    types, symmetric (eps, sigma) tables, masses per type, cutoff rc, skin,
    time step.  ``mode`` is "full" or "half" (Verlet list storage), ``prec``
    is "fp64" or "mixed" (FP32 pair polynomial, FP64 accumulation).
    """

    def __init__(self, natoms, box, pos, vel, types=None, eps=1.0, sig=1.0, mass=None,
                 rc=2.5, skin=0.3, dt=0.005, shift=1, mode="full", prec="fp64",
                 max_nbr=None, pos4=None, bonds=None, fene=(30.0, 1.5), angles=None,
                 angle_K=1.5, bonded_order="index", langevin=None,
                 tile_cells=None, tile_rows=(1, 1), fuse=True, sparse_tiles=None,
                 device="cuda"):
        self.lib = abi.load()
        self.dev = torch.device(device)
        natoms = np.asarray(natoms, dtype=np.int32).ravel()
        box = np.asarray(box, dtype=np.float64).reshape(-1, 3)
        self.R = int(natoms.shape[0])
        self.rc, self.skin, self.dt, self.shift = float(rc), float(skin), float(dt), int(shift)
        self.mode = {"full": abi.MD_FULL, "half": abi.MD_HALF, "tile": abi.MD_TILE_FULL}[mode]
        self.prec = abi.MD_FP64 if prec == "fp64" else abi.MD_FP32_MIXED
        eps = np.atleast_2d(np.asarray(eps, dtype=np.float64))
        sig = np.atleast_2d(np.asarray(sig, dtype=np.float64))
        self.ntypes = int(eps.shape[0])
        mass = np.ones(self.ntypes) if mass is None else np.asarray(mass, np.float64).ravel()

        # ---- host planning
        N, C, U = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check("md_plan_sizes", self.lib.md_plan_sizes(
            self.R, natoms.ctypes.data, box.ctypes.data, self.rc, self.skin,
            ctypes.byref(N), ctypes.byref(C), ctypes.byref(U)))
        self.N, self.C, self.n_units = N.value, C.value, U.value
        h_atom_off = np.zeros(self.R + 1, np.int32)
        h_cell_off = np.zeros(self.R + 1, np.int32)
        h_ncell = np.zeros(3 * self.R, np.int32)
        h_unit_rep = np.zeros(self.n_units, np.int32)
        h_unit_off = np.zeros(self.R + 1, np.int32)
        check("md_plan_fill", self.lib.md_plan_fill(
            self.R, natoms.ctypes.data, box.ctypes.data, self.rc, self.skin,
            h_atom_off.ctypes.data, h_cell_off.ctypes.data, h_ncell.ctypes.data,
            h_unit_rep.ctypes.data, h_unit_off.ctypes.data))
        self.h_atom_off, self.h_ncell, self.h_box = h_atom_off, h_ncell.reshape(-1, 3), box
        d = self.dev
        i32 = lambda a: torch.as_tensor(a, dtype=torch.int32).to(d)
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(d)
        self.atom_off, self.cell_off = i32(h_atom_off), i32(h_cell_off)
        self.ncell, self.box = i32(h_ncell), f64(box.ravel())
        self.unit_rep, self.unit_off = i32(h_unit_rep), i32(h_unit_off)
        self.batch = abi.MdBatch(self.R, self.N, self.C, self.n_units,
                                 self.atom_off.data_ptr(), self.cell_off.data_ptr(),
                                 self.ncell.data_ptr(), self.box.data_ptr(),
                                 self.unit_rep.data_ptr(), self.unit_off.data_ptr())

        # ---- atom state (SoA planes)
        pos = np.asarray(pos, np.float64).reshape(self.N, 3)
        vel = np.asarray(vel, np.float64).reshape(self.N, 3)
        types = np.zeros(self.N, np.int32) if types is None else np.asarray(types, np.int32)
        z64 = lambda: torch.zeros(self.N, dtype=torch.float64, device=d)
        # positions: one (x, y, z) buffer, or two that the fused force +
        # integrator call alternates between (it writes the next positions
        # into the other one); self._par names the current one
        self._pos = [tuple(f64(pos[:, k]) for k in range(3))]
        self._par = 0
        self.vx, self.vy, self.vz = (f64(vel[:, k]) for k in range(3))
        self.fx, self.fy, self.fz = z64(), z64(), z64()
        self.xb, self.yb, self.zb = self.x.clone(), self.y.clone(), self.z.clone()
        self.type = i32(types)
        self.id = torch.arange(self.N, dtype=torch.int32, device=d)
        self.img = torch.zeros(3 * self.N, dtype=torch.int32, device=d)
        self.where = torch.arange(self.N, dtype=torch.int32, device=d)
        # packed (x, y, z, 0) gather copy, maintained by the re-sort and the integrator
        if pos4 is None:
            # the packed copy feeds the global-list gathers, and tile staging
            # only when MD_TUNE_TILE_STAGE_PACKED is set
            pos4 = (mode != "tile" or
                    self.lib.md_tune_get(abi.MD_TUNE_TILE_STAGE_PACKED) == 1)
        self.pos4 = torch.zeros(4 * self.N, dtype=torch.float64, device=d) if pos4 else None
        self._atoms = [self._atoms_struct(xyz) for xyz in self._pos]
        # re-sort scratch planes
        self.s_x, self.s_y, self.s_z, self.s_vx, self.s_vy, self.s_vz = (z64() for _ in range(6))
        self.s_type = torch.zeros(self.N, dtype=torch.int32, device=d)
        self.s_id = torch.zeros(self.N, dtype=torch.int32, device=d)
        self.s_img = torch.zeros(3 * self.N, dtype=torch.int32, device=d)
        self.scratch = abi.MdAtoms(self.s_x.data_ptr(), self.s_y.data_ptr(), self.s_z.data_ptr(),
                                   self.s_vx.data_ptr(), self.s_vy.data_ptr(),
                                   self.s_vz.data_ptr(), None, None, None, None, None, None,
                                   self.s_type.data_ptr(), self.s_id.data_ptr(),
                                   self.s_img.data_ptr(), None, None)

        # ---- parameters, list, workspace, outputs
        self.eps_t, self.sig_t = f64(eps.ravel()), f64(sig.ravel())
        self.inv_mass = f64(1.0 / mass)
        self.lj = abi.MdLj(self.ntypes, self.shift, self.rc, self.eps_t.data_ptr(),
                           self.sig_t.data_ptr())
        self.cell_start = torch.zeros(self.C + 1, dtype=torch.int32, device=d)
        self.ld = (self.N + 63) // 64 * 64
        self.tile_need = torch.zeros(1, dtype=torch.int32, device=d)
        self.tile_cells, self.n_tiles = 0, 0
        self.h_tile_m, self.tile_m, self.tile_todo = None, None, None
        self.tile_py, self.tile_pz = (int(tile_rows[0]), int(tile_rows[1]))
        # occupied-tile list (one replica): on by default when most cells start
        # empty (a droplet or slab in vacuum), so empty tiles get no workgroup
        if sparse_tiles is None:
            sparse_tiles = (self.mode == abi.MD_TILE_FULL and self.R == 1 and
                            _empty_cell_fraction(pos, box[0], self.h_ncell[0]) > 0.5)
        self.sparse_tiles = bool(sparse_tiles) and self.mode == abi.MD_TILE_FULL
        if self.sparse_tiles and self.R != 1:
            raise ValueError("the occupied-tile list covers one replica")
        self.tile_active = None
        if self.mode == abi.MD_TILE_FULL:
            if tile_cells is None:
                # cells per tile from nu = mean atoms per occupied cell (so
                # vacuum does not dilute it), for each replica on its own: a
                # batch whose replicas have different cell sizes then gives
                # each the largest tiles it fits
                nu = _occupied_cell_density(pos, natoms, box, self.h_ncell)
                args = (self.lib.md_tile_capacity(), self.lib.md_tune_get(abi.MD_TUNE_TILE_THREADS),
                        self.tile_py, self.tile_pz, self.lib.md_tile_max_cells())
                per = np.array([_tile_cells_for(nu[r], int(self.h_ncell[r, 0]), *args)
                                for r in range(self.R)], dtype=np.int32)
                tile_cells = per if self.R > 1 and np.any(per != per[0]) else int(per[0])
            self._plan_tiles(tile_cells)
        if max_nbr is None:
            # ideal-gas estimate of neighbours within rc + skin, with margin
            rho = float(np.max(natoms / np.prod(box, axis=1)))
            full = 4.0 / 3.0 * math.pi * (self.rc + self.skin) ** 3 * rho
            max_nbr = int(1.35 * full * (0.5 if self.mode == abi.MD_HALF else 1.0)) + 16
        self._alloc_list(max_nbr)
        self.ws_bytes = int(self.lib.md_workspace_bytes(ctypes.byref(self.batch)))
        self.ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=d)
        self.gate = torch.ones(self.R, dtype=torch.int32, device=d)
        # the repeated fused NVE steps' gate: two words per replica, used
        # alternately with the two position buffers (md_lj_forces_vv's
        # gate_clear); _gate_cur is the gate the current step's re-sort and
        # list build read
        self.gates = torch.zeros(2, self.R, dtype=torch.int32, device=d)
        self._gate_cur = self.gate
        self.status = torch.zeros(1, dtype=torch.int32, device=d)
        self.need = torch.zeros(1, dtype=torch.int32, device=d)
        self.energy = torch.zeros(self.R, dtype=torch.float64, device=d)
        self.virial = torch.zeros(self.R, dtype=torch.float64, device=d)
        self.ke = torch.zeros(self.R, dtype=torch.float64, device=d)
        self._graph = None
        self._stepped = 0        # steps run since the status word was last read clean
        self.recoveries = []     # overflow recoveries of run()/run_checked(): sticky record

        # ---- optional FENE bonds (id pairs [Nb,2]) and Langevin thermostat
        self.bonds = None
        if bonds is not None and len(bonds):
            bonds = np.asarray(bonds, np.int64).reshape(-1, 2)
            if bonds.min() < 0 or bonds.max() >= self.N:
                raise ValueError("a bond names an atom outside the system")
            u_ = np.concatenate([bonds[:, 0], bonds[:, 1]])
            v_ = np.concatenate([bonds[:, 1], bonds[:, 0]])
            order = np.argsort(u_, kind="stable")
            u_, v_ = u_[order], v_[order]
            cnt = np.bincount(u_, minlength=self.N).astype(np.int32)
            if cnt.max() > abi.MD_MAX_BONDS:
                raise ValueError(f"an atom has more than {abi.MD_MAX_BONDS} bonds")
            start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
            part = np.full((abi.MD_MAX_BONDS, self.N), -1, np.int32)
            part[np.arange(len(u_)) - start[u_], u_] = v_
            mb = max(1, int(cnt.max()))
            self.bond_count = i32(cnt)
            self.bond_partner = i32(np.ascontiguousarray(part[:mb]))
            self.bonds = abi.MdBonds(mb, abi.MD_BY_ID, self.bond_count.data_ptr(),
                                     self.bond_partner.data_ptr())
            self.fene_K, self.fene_R0 = float(fene[0]), float(fene[1])
            self.energy_bond = torch.zeros(self.R, dtype=torch.float64, device=d)
            self.virial_bond = torch.zeros(self.R, dtype=torch.float64, device=d)
        # ---- optional cosine angle terms (id triples [Na,3], middle bead second),
        # each triple stored in the slot table of all three of its atoms
        self.angles = None
        if angles is not None and len(angles):
            tri = np.asarray(angles, np.int64).reshape(-1, 3)
            if tri.min() < 0 or tri.max() >= self.N:
                raise ValueError("an angle triple names an atom outside the system")
            if np.any((tri[:, 0] == tri[:, 1]) | (tri[:, 1] == tri[:, 2]) |
                      (tri[:, 0] == tri[:, 2])):
                raise ValueError("an angle triple names one atom twice")
            owner = tri.T.ravel()                          # role-major: a's, b's, c's
            which = np.tile(np.arange(tri.shape[0]), 3)
            order = np.lexsort((which, owner))             # by atom, then by triple
            owner, which = owner[order], which[order]
            cnt = np.bincount(owner, minlength=self.N).astype(np.int32)
            if cnt.max() > abi.MD_MAX_ANGLES:
                raise ValueError(f"an atom belongs to more than {abi.MD_MAX_ANGLES} triples")
            ma = max(1, int(cnt.max()))
            start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
            slot = np.arange(owner.shape[0]) - start[owner]
            table = np.full((ma, 3, self.N), -1, np.int32)
            for r in range(3):
                table[slot, r, owner] = tri[which, r]
            self.angle_count = i32(cnt)
            self.angle_tri = i32(np.ascontiguousarray(table.reshape(3 * ma, self.N)))
            self.angles = abi.MdAngles(ma, abi.MD_BY_ID, self.angle_count.data_ptr(),
                                       self.angle_tri.data_ptr())
            self.angle_K = float(angle_K)
            self.energy_angle = torch.zeros(self.R, dtype=torch.float64, device=d)
            self.virial_angle = torch.zeros(self.R, dtype=torch.float64, device=d)
        # ---- the bonded tables the kernels read: keyed by id as given, or
        # (default) re-keyed to the cell-sorted order after every re-sort
        if bonded_order not in ("index", "id"):
            raise ValueError("bonded_order is 'index' or 'id'")
        self.bonded_by_index = bonded_order == "index"
        self._bonds_k, self._angles_k = self.bonds, self.angles
        if self.bonded_by_index and self.bonds is not None:
            self.bond_count_ix = torch.zeros_like(self.bond_count)
            self.bond_partner_ix = torch.zeros_like(self.bond_partner)
            self._bonds_k = abi.MdBonds(self.bonds.max_bonds, abi.MD_BY_INDEX,
                                        self.bond_count_ix.data_ptr(),
                                        self.bond_partner_ix.data_ptr())
        if self.bonded_by_index and self.angles is not None:
            self.angle_count_ix = torch.zeros_like(self.angle_count)
            self.angle_tri_ix = torch.zeros_like(self.angle_tri)
            self._angles_k = abi.MdAngles(self.angles.max_angles, abi.MD_BY_INDEX,
                                          self.angle_count_ix.data_ptr(),
                                          self.angle_tri_ix.data_ptr())
        self.langevin_cfg = None
        if langevin is not None:
            gamma, temp, seed = langevin[:3]
            step0 = langevin[3] if len(langevin) > 3 else 0
            self.langevin_cfg = (float(gamma), float(temp), int(seed))
            self.mass_t = f64(mass)
            self.noise_step = torch.tensor([int(step0)], dtype=torch.int64, device=d)
        # pair forces on tile lists (typed for several types), with or without the
        # thermostat: the force call also advances the step
        # (md_lj_forces_vv); bonds or angles need the split calls
        self.fuse = bool(fuse) and self.mode == abi.MD_TILE_FULL and self.bonds is None \
            and self.angles is None and self.ntypes <= abi.MD_TILE_MAX_TYPES
        self.thermo = None
        if self.langevin_cfg is not None:
            gamma, temp, seed = self.langevin_cfg
            self.thermo = abi.MdThermostat(gamma, temp, seed, self.noise_step.data_ptr(),
                                           self.mass_t.data_ptr())
        # without the fused call, the thermostat force of a step is added by
        # the half kick that uses it (md_vv_step with the thermostat), not by
        # a separate md_langevin call; only the initial forces call it
        self.vv_thermo = self.thermo is not None and not self.fuse
        if self.fuse and self.pos4 is None:
            self._pos.append((z64(), z64(), z64()))
            self._atoms.append(self._atoms_struct(self._pos[1]))

    @property
    def x(self):
        return self._pos[self._par][0]

    @property
    def y(self):
        return self._pos[self._par][1]

    @property
    def z(self):
        return self._pos[self._par][2]

    @property
    def atoms(self):
        return self._atoms[self._par]

    def _atoms_struct(s, xyz):
        x, y, z = xyz
        return abi.MdAtoms(x.data_ptr(), y.data_ptr(), z.data_ptr(), s.vx.data_ptr(),
                           s.vy.data_ptr(), s.vz.data_ptr(), s.fx.data_ptr(), s.fy.data_ptr(),
                           s.fz.data_ptr(), s.xb.data_ptr(), s.yb.data_ptr(), s.zb.data_ptr(),
                           s.type.data_ptr(), s.id.data_ptr(), s.img.data_ptr(),
                           s.where.data_ptr(),
                           s.pos4.data_ptr() if s.pos4 is not None else None)

    def _plan_tiles(self, m):
        """Tiles of m cells along x: one int for every replica, or an array
        of one per replica (kept as ``h_tile_m``; ``tile_cells`` is then its
        largest value)."""
        ncell = np.ascontiguousarray(self.h_ncell.ravel(), dtype=np.int32)
        py, pz = self.tile_py, self.tile_pz
        if np.ndim(m) == 0:
            hm, mx = None, int(m)
        else:
            hm = np.ascontiguousarray(m, dtype=np.int32)
            mx = int(hm.max())
        hp = hm.ctypes.data if hm is not None else None
        n = self.lib.md_tile_plan(self.R, ncell.ctypes.data, mx, hp, py, pz, None, None)
        if n < 1:
            raise abi.MDError("md_tile_plan", n)
        rep = np.zeros(n, np.int32)
        off = np.zeros(self.R + 1, np.int32)
        check("md_tile_plan", min(0, self.lib.md_tile_plan(self.R, ncell.ctypes.data, mx, hp,
                                                           py, pz, rep.ctypes.data,
                                                           off.ctypes.data)))
        self.tile_cells, self.n_tiles = mx, n
        self.h_tile_m = hm
        self.tile_m = torch.as_tensor(hm).to(self.dev) if hm is not None else None
        # a batch's list build lists the tiles of the replicas it rebuilds here
        self.tile_todo = (torch.zeros(n + 1, dtype=torch.int32, device=self.dev)
                          if self.R > 1 else None)
        self.tile_rep = torch.as_tensor(rep).to(self.dev)
        self.tile_off = torch.as_tensor(off).to(self.dev)
        # per-tile staging records (capacity + 128 words each), written by the build
        self.tile_src_cap = self.lib.md_tile_capacity()
        self.tile_src = torch.zeros(n * (self.tile_src_cap + 128), dtype=torch.int32,
                                    device=self.dev)
        if self.sparse_tiles:
            # count, list, per-tile occupancy; written by the build
            self.tile_active = torch.zeros(2 * n + 1, dtype=torch.int32, device=self.dev)

    def _alloc_list(self, max_nbr):
        self.max_nbr = (int(max_nbr) + 15) // 16 * 16   # tile lists pad to 16 entries
        self.count = torch.zeros(self.N, dtype=torch.int32, device=self.dev)
        self.idx = torch.zeros(self.max_nbr * self.ld, dtype=torch.int32, device=self.dev)
        self._set_nlist()

    def _set_nlist(self):
        tiled = self.mode == abi.MD_TILE_FULL
        self.nlist = abi.MdNlist(
            self.mode, self.max_nbr, self.ld, self.tile_cells if tiled else 0,
            self.count.data_ptr(), self.idx.data_ptr(), self.n_tiles if tiled else 0,
            self.tile_py, self.tile_pz, self.ntypes if tiled and self.ntypes > 1 else 0,
            self.tile_rep.data_ptr() if tiled else None,
            self.tile_off.data_ptr() if tiled else None,
            self.tile_need.data_ptr(), self.cell_start.data_ptr() if tiled else None,
            self.tile_src_cap if tiled else 0, 0, self.tile_src.data_ptr() if tiled else None,
            self.tile_active.data_ptr() if tiled and self.tile_active is not None else None,
            self.tile_m.data_ptr() if tiled and self.tile_m is not None else None,
            self.tile_todo.data_ptr() if tiled and self.tile_todo is not None else None)

    @property
    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)

    # ------------------------------------------------------------ ABI calls
    def sort(self, gated=True):
        check("md_cell_sort", self.lib.md_cell_sort(
            ctypes.byref(self.batch), ctypes.byref(self.atoms), ctypes.byref(self.scratch),
            _ptr(self.cell_start), _ptr(self.ws), self.ws_bytes,
            _ptr(self._gate_cur) if gated else None, _ptr(self.status), self.stream))
        if self.bonded_by_index and (self.bonds is not None or self.angles is not None):
            check("md_bonded_reindex", self.lib.md_bonded_reindex(
                ctypes.byref(self.batch), ctypes.byref(self.atoms),
                ctypes.byref(self.bonds) if self.bonds is not None else None,
                _ptr(getattr(self, "bond_count_ix", None)),
                _ptr(getattr(self, "bond_partner_ix", None)),
                ctypes.byref(self.angles) if self.angles is not None else None,
                _ptr(getattr(self, "angle_count_ix", None)),
                _ptr(getattr(self, "angle_tri_ix", None)),
                _ptr(self._gate_cur) if gated else None, self.stream))

    def build(self, gated=True):
        check("md_verlet_build", self.lib.md_verlet_build(
            ctypes.byref(self.batch), ctypes.byref(self.atoms), _ptr(self.cell_start),
            self.rc, self.skin, ctypes.byref(self.nlist), _ptr(self.need),
            _ptr(self._gate_cur) if gated else None, _ptr(self.status), self.stream))

    def forces(self, accumulate=False, energies=True, atoms=None):
        e, w = (self.energy, self.virial) if energies else (None, None)
        check("md_lj_forces", self.lib.md_lj_forces(
            ctypes.byref(self.batch), ctypes.byref(atoms or self.atoms), ctypes.byref(self.nlist),
            ctypes.byref(self.lj), self.prec, int(accumulate), _ptr(e), _ptr(w),
            _ptr(self.ws), self.ws_bytes, _ptr(self.status), self.stream))

    def forces_vv(self, energies=True):
        """Forces at the current positions (plus the thermostat, if any), then
        velocity-Verlet phase 3, in one call (pair forces on tile lists).
        energies=False leaves energy, virial and ke as they were (the call
        then sums only the rebuild gate)."""
        two = len(self._pos) == 2
        nxt = self._pos[self._par ^ 1] if two else (None, None, None)
        e, w, k = (self.energy, self.virial, self.ke) if energies else (None, None, None)
        # repeated NVE steps with two position buffers: the gate words alternate
        # with the buffers, so the force kernel sets the gate itself
        alt = two and not energies and self.thermo is None
        g, gc = (self.gates[self._par], self.gates[self._par ^ 1]) if alt else (self.gate, None)
        self._gate_cur = g
        check("md_lj_forces_vv", self.lib.md_lj_forces_vv(
            ctypes.byref(self.batch), ctypes.byref(self.atoms), ctypes.byref(self.nlist),
            ctypes.byref(self.lj), self.prec, self.dt, _ptr(self.inv_mass), self.ntypes,
            self.skin, _ptr(g), _ptr(gc), _ptr(k), _ptr(e), _ptr(w),
            _ptr(nxt[0]), _ptr(nxt[1]), _ptr(nxt[2]),
            ctypes.byref(self.thermo) if self.thermo is not None else None,
            _ptr(self.ws), self.ws_bytes, _ptr(self.status), self.stream))
        if two:
            self._par ^= 1   # the next positions are now the current ones

    def vv(self, phase, energies=True):
        thermo = self.thermo if self.vv_thermo and phase >= 2 else None
        if phase != 2:
            self._gate_cur = self.gate
        check("md_vv_step", self.lib.md_vv_step(
            ctypes.byref(self.batch), ctypes.byref(self.atoms), int(phase), self.dt,
            _ptr(self.inv_mass), self.ntypes, self.skin, _ptr(self.gate),
            _ptr(self.ke if energies else None),
            ctypes.byref(thermo) if thermo is not None else None,
            _ptr(self.ws), self.ws_bytes, _ptr(self.status), self.stream))

    def vjp(self, gfx, gfy, gfz, gE, gx, geps=None, gsig=None):
        check("md_lj_forces_vjp", self.lib.md_lj_forces_vjp(
            ctypes.byref(self.batch), ctypes.byref(self.atoms), ctypes.byref(self.nlist),
            ctypes.byref(self.lj), self.prec, _ptr(gfx), _ptr(gfy), _ptr(gfz), _ptr(gE),
            _ptr(gx), _ptr(geps), _ptr(gsig), _ptr(self.ws), self.ws_bytes,
            _ptr(self.status), self.stream))

    def fene(self, energies=True, atoms=None):
        e, w = (self.energy_bond, self.virial_bond) if energies else (None, None)
        check("md_fene_forces", self.lib.md_fene_forces(
            ctypes.byref(self.batch), ctypes.byref(atoms or self.atoms), ctypes.byref(self._bonds_k),
            self.fene_K, self.fene_R0, _ptr(e), _ptr(w),
            _ptr(self.ws), self.ws_bytes, _ptr(self.status), self.stream))

    def bonded(self, energies=True, atoms=None):
        """FENE bonds and angle triples in one call (tables keyed by index)."""
        ebs = (self.energy_bond, self.virial_bond, self.energy_angle, self.virial_angle) \
            if energies else (None, None, None, None)
        check("md_bonded_forces", self.lib.md_bonded_forces(
            ctypes.byref(self.batch), ctypes.byref(atoms or self.atoms), ctypes.byref(self._bonds_k),
            self.fene_K, self.fene_R0, ctypes.byref(self._angles_k), self.angle_K,
            *(_ptr(q) for q in ebs), _ptr(self.ws), self.ws_bytes, _ptr(self.status),
            self.stream))

    def angle(self, energies=True, atoms=None):
        e, w = (self.energy_angle, self.virial_angle) if energies else (None, None)
        check("md_angle_forces", self.lib.md_angle_forces(
            ctypes.byref(self.batch), ctypes.byref(atoms or self.atoms), ctypes.byref(self._angles_k),
            self.angle_K, _ptr(e), _ptr(w),
            _ptr(self.ws), self.ws_bytes, _ptr(self.status), self.stream))

    def langevin(self):
        gamma, temp, seed = self.langevin_cfg
        check("md_langevin", self.lib.md_langevin(
            ctypes.byref(self.batch), ctypes.byref(self.atoms), _ptr(self.mass_t), self.ntypes,
            gamma, temp, self.dt, seed, _ptr(self.noise_step), _ptr(self.status),
            self.stream))

    def all_forces(self, initial=False, energies=True):
        """Pair forces, then (if configured) bond and angle forces and the
        thermostat (which the next half kick adds instead, except for the
        initial forces, when the split calls are used).  energies=False
        leaves the energy and virial outputs as they were."""
        self._conservative(energies)
        if self.langevin_cfg is not None and (initial or not self.vv_thermo):
            self.langevin()

    def _conservative(self, energies, atoms=None):
        # pair, bond and angle terms into the given atoms' force planes
        self.forces(energies=energies, atoms=atoms)
        if self.bonds is not None and self.angles is not None and self.bonded_by_index:
            self.bonded(energies=energies, atoms=atoms)
        else:
            if self.bonds is not None:
                self.fene(energies=energies, atoms=atoms)
            if self.angles is not None:
                self.angle(energies=energies, atoms=atoms)

    def energies_now(self):
        """Energy and virial outputs of the current positions, evaluated into
        the re-sort's scratch planes (free between steps), so that the forces,
        velocities and the thermostat's noise counter stay as they are."""
        a = self.atoms
        tmp = abi.MdAtoms(a.x, a.y, a.z, a.vx, a.vy, a.vz, self.s_vx.data_ptr(),
                          self.s_vy.data_ptr(), self.s_vz.data_ptr(), a.xb, a.yb, a.zb,
                          a.type, a.id, a.img, a.where, a.pos4)
        self._conservative(True, atoms=tmp)

    # ------------------------------------------------------------ the step
    def setup(self):
        """Initial re-sort, list build and forces (all replicas)."""
        self.sort(gated=False)
        self.build(gated=False)
        self.ensure_list()
        self.all_forces(initial=True)

    _OVERFLOW = abi.MD_F_NBR_OVERFLOW | abi.MD_F_TILE_OVERFLOW

    def _regrow(self, st):
        """Grow the list storage for the overflow flags in ``st``: smaller
        tiles for MD_F_TILE_OVERFLOW, a longer list for MD_F_NBR_OVERFLOW.
        Captured graphs hold the old pointers, so they are dropped."""
        if st & abi.MD_F_TILE_OVERFLOW:
            if self.tile_cells <= 1:
                raise RuntimeError("a single-cell tile exceeds the LDS staging capacity")
            if self.h_tile_m is not None:
                # only the replicas with a tile past the capacity get smaller
                # tiles: the build leaves every staged count in its record
                stride = self.tile_src_cap + 128
                tot = self.tile_src.view(self.n_tiles, stride)[:, self.tile_src_cap].cpu().numpy()
                bad = np.unique(self.tile_rep.cpu().numpy()[tot > self.tile_src_cap])
                m = self.h_tile_m.copy()
                if bad.size == 0 or np.all(m[bad] <= 1):
                    raise RuntimeError("a single-cell tile exceeds the LDS staging capacity")
                m[bad] = np.maximum(1, m[bad] - np.maximum(1, m[bad] // 4))
                self._plan_tiles(m)
            else:
                self._plan_tiles(max(1, self.tile_cells - max(1, self.tile_cells // 4)))
            self._set_nlist()
        if st & abi.MD_F_NBR_OVERFLOW:
            self._alloc_list(int(int(self.need.item()) * 1.2) + 8)
        self._graph = None
        self.status.zero_()
        self.need.zero_()
        self.tile_need.zero_()

    def ensure_list(self):
        """Synchronise and read the status word.

        Right after an ungated re-sort and list build (set-up, recovery) an
        overflow is repaired here: the list storage grows and the list is
        rebuilt until it fits.  After steps have run on a list, an overflow
        means some of those steps used a truncated list (forces, and in the
        fused call whole tiles, were skipped), so the trajectory is invalid:
        that raises ListOverflowError with the flag left set; run() with
        check_every > 0 recovers by itself instead.  Any other flag raises."""
        torch.cuda.synchronize(self.dev)
        st = int(self.status.item())
        if st & self._OVERFLOW and self._stepped:
            raise abi.ListOverflowError(
                f"the Verlet list overflowed during the last {self._stepped} steps "
                f"(status 0x{st:x}): their trajectory used a truncated list")
        while st & self._OVERFLOW:
            self._regrow(st)
            self.build(gated=False)
            torch.cuda.synchronize(self.dev)
            st = int(self.status.item())
        if st:
            raise RuntimeError(f"device status flags 0x{st:x}")
        self._stepped = 0
        return st

    # ------------------------------------------------- checkpoint / recovery
    _STATE = ("vx", "vy", "vz", "fx", "fy", "fz", "xb", "yb", "zb", "type", "id", "img",
              "where", "pos4", "noise_step", "energy", "virial", "ke")

    def checkpoint(self):
        """Device copy of the state a run evolves (positions, velocities,
        forces, build positions, atom order and images, the thermostat's
        noise counter); restore() brings it back."""
        torch.cuda.synchronize(self.dev)
        cp = {"par": self._par, "pos": tuple(t.clone() for t in self._pos[self._par])}
        for k in self._STATE:
            t = getattr(self, k, None)
            cp[k] = t.clone() if t is not None else None
        return cp

    def restore(self, cp):
        """Return to a checkpoint() and make the list valid for it: grow the
        list storage for the overflow flags that are set, clear the status,
        re-sort and rebuild (ungated, so the build positions are the current
        ones), and carry the checkpoint's forces over to the new atom order
        (the re-sort permutes every per-atom plane except the forces)."""
        torch.cuda.synchronize(self.dev)
        st = int(self.status.item())
        self._par = cp["par"]
        for dst, src in zip(self._pos[self._par], cp["pos"]):
            dst.copy_(src)
        for k in self._STATE:
            if cp[k] is not None:
                getattr(self, k).copy_(cp[k])
        # forces by atom id, on the host (a permutation, no arithmetic)
        ids = cp["id"].cpu().numpy()
        f_id = np.empty((self.N, 3))
        f_id[ids] = np.stack([cp["fx"].cpu().numpy(), cp["fy"].cpu().numpy(),
                              cp["fz"].cpu().numpy()], 1)
        if st & self._OVERFLOW:
            self._regrow(st)
        else:
            self.status.zero_()
        self.gates.zero_()
        self.sort(gated=False)
        self.build(gated=False)
        self._stepped = 0
        self.ensure_list()
        f_new = f_id[self.id.cpu().numpy()]
        for k, t in enumerate((self.fx, self.fy, self.fz)):
            t.copy_(torch.from_numpy(np.ascontiguousarray(f_new[:, k])))
        torch.cuda.synchronize(self.dev)
        return st

    @property
    def step_gate(self):
        """The rebuild gate ([R] device) that the latest step's re-sort and
        list build read."""
        return self._gate_cur

    def overflowed(self):
        """Synchronise; True if a list overflow flag is set (other flags raise)."""
        torch.cuda.synchronize(self.dev)
        st = int(self.status.item())
        if st & ~self._OVERFLOW:
            raise RuntimeError(f"device status flags 0x{st:x}")
        return bool(st & self._OVERFLOW)

    def step_body(self, first, energies=True):
        """One velocity-Verlet step except its final half kick."""
        self.vv(1 if first else 3, energies=energies)
        self.sort()
        self.build()
        self.all_forces(energies=energies)

    def fused_body(self):
        """The same work in the fused order: the forces of one step with its
        Integrate2 and the next step's Integrate1 (one call), then the gated
        re-sort and list build of the next step.  A run's energies are those
        its last step (the tail) computes, so the repeated steps sum only the
        rebuild gate."""
        self.forces_vv(energies=False)
        self.sort()
        self.build()

    def _body(self):
        # a run's energies are those its tail computes, so the repeated steps
        # sum only the rebuild gate
        self._stepped += 1
        if self.fuse:
            self.fused_body()
        else:
            self.step_body(first=False, energies=False)

    def _head(self):
        # first step up to its forces (fused: up to its list build)
        self._stepped += 1
        if self.fuse:
            self.vv(1)
            self.sort()
            self.build()
        else:
            self.step_body(first=True, energies=False)

    def _tail(self):
        # last step's forces (fused) or its energies (split: the forces are
        # those of the last step), and the final half kick
        if self.fuse:
            self.all_forces()
        else:
            self.energies_now()
        self.vv(2)

    def run(self, steps, check_every=50, max_recoveries=8):
        """`steps` full steps (Integrate2 of step s fused with Integrate1 of s+1).

        With check_every > 0 the status word is read every check_every steps.
        A list overflow seen there sends the run back to the state saved at
        the previous check (restore(): the list grows and is rebuilt), and
        the steps since are run again; each such recovery is recorded in
        self.recoveries (step, flags).  With check_every = 0 nothing is read
        and ensure_list() afterwards raises if the list overflowed."""
        if not check_every:
            self._head()
            for _ in range(1, steps):
                self._body()
            self._tail()
            return
        cp, at = self.checkpoint(), -1      # -1: before the first step's head
        self._head()
        done, tries = 0, 0
        while True:
            k = min(check_every, steps - 1 - done)
            for _ in range(k):
                self._body()
            done += k
            if self.overflowed():
                tries += 1
                if tries > max_recoveries:
                    raise abi.ListOverflowError("the Verlet list kept overflowing")
                flags = self.restore(cp)
                self.recoveries.append({"step": done, "flags": flags,
                                        "max_nbr": self.max_nbr,
                                        "tile_cells": self.tile_cells})
                if at < 0:
                    done = 0
                    self._head()
                else:
                    done = at
                continue
            if done >= steps - 1:
                break
            cp, at = self.checkpoint(), done
        self._tail()
        self._stepped = 0

    def capture(self, k):
        """Capture k repeated steps (Integrate2+Integrate1, gated re-sort and
        list build, forces) as one HIP graph; replays launch on the current
        stream.  With alternating position buffers a graph holds an even
        number of steps (k + 1 for odd k), so a replay ends on the buffer it
        started from."""
        kk = k + 1 if len(self._pos) == 2 and k % 2 else k
        par0 = self._par
        torch.cuda.synchronize(self.dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(kk):
                self._body()
        torch.cuda.synchronize(self.dev)
        assert self._par == par0
        self._graph = (k, g, kk, par0)
        return g

    def run_graphed(self, steps, k=50):
        """Same trajectory as run(steps) with the repeated steps replayed from a
        captured graph of k steps.  Status flags are not read here: call
        ensure_list() afterwards (it raises if the list overflowed), or use
        run_checked()."""
        if self._graph is None or self._graph[0] != k:
            self.capture(k)
        _, g, kk, par0 = self._graph
        self._head()
        rest = steps - 1
        if rest > 0 and self._par != par0:
            self._body()   # onto the buffer the graph starts from
            rest -= 1
        for _ in range(rest // kk):
            g.replay()
        for _ in range(rest % kk):
            self._body()
        self._tail()

    def run_checked(self, steps, k=50, max_recoveries=8):
        """run_graphed() from a checkpoint: if the list overflowed on the way,
        return to the checkpoint (the list grows) and run the steps again."""
        cp = self.checkpoint()
        for _ in range(max_recoveries + 1):
            self.run_graphed(steps, k=k)
            if not self.overflowed():
                self._stepped = 0
                return
            flags = self.restore(cp)
            self.recoveries.append({"step": None, "flags": flags, "max_nbr": self.max_nbr,
                                    "tile_cells": self.tile_cells})
        raise abi.ListOverflowError("the Verlet list kept overflowing")

    # ------------------------------------------------------------ readback
    def order(self):
        """Current slot of each original atom id."""
        return self.where.cpu().numpy()

    def positions(self):
        """Unwrapped positions [N,3] in original id order (x + img L)."""
        ids = self.id.cpu().numpy()
        L = np.repeat(self.h_box, np.diff(self.h_atom_off), axis=0)
        img = self.img.cpu().numpy().reshape(3, self.N).T
        p = np.stack([self.x.cpu().numpy(), self.y.cpu().numpy(), self.z.cpu().numpy()], 1)
        rep = np.repeat(np.arange(self.R), np.diff(self.h_atom_off))
        out = np.empty_like(p)
        out[ids] = p + img * self.h_box[rep]
        return out

    def _by_id(self, a, b, c):
        ids = self.id.cpu().numpy()
        out = np.empty((self.N, 3))
        out[ids] = np.stack([a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()], 1)
        return out

    def velocities(self):
        return self._by_id(self.vx, self.vy, self.vz)

    def forces_np(self):
        return self._by_id(self.fx, self.fy, self.fz)

    def tile_slot_table(self):
        """For MD_TILE_FULL lists: per tile, the global indices of its home
        atoms and of every staged slot, in the staged order documented in md.h."""
        cs = self.cell_start.cpu().numpy()
        rep = self.tile_rep.cpu().numpy()
        toff = self.tile_off.cpu().numpy()
        coff = np.concatenate([[0], np.cumsum(np.prod(self.h_ncell, axis=1))])
        py, pz = self.tile_py, self.tile_pz
        tables = []
        for t in range(self.n_tiles):
            r = rep[t]
            m = int(self.h_tile_m[r]) if self.h_tile_m is not None else self.tile_cells
            nx, ny, nz = self.h_ncell[r]
            tx, ty = -(-nx // m), -(-ny // py)
            local = t - toff[r]
            bx, rest = local % tx, local // tx
            by, bz = rest % ty, rest // ty
            a, b = bx * m, min(bx * m + m, nx) - 1
            y0, y1 = by * py, min(by * py + py, ny) - 1
            z0, z1 = bz * pz, min(bz * pz + pz, nz) - 1
            slots = []
            for zz in range(z0 - 1, z1 + 2):
                for yy in range(y0 - 1, y1 + 2):
                    rb = coff[r] + ((zz % nz) * ny + yy % ny) * nx
                    for xu in range(a - 1, b + 2):
                        c = rb + xu % nx
                        slots.extend(range(cs[c], cs[c + 1]))
            home = []
            for zz in range(z0, z1 + 1):
                for yy in range(y0, y1 + 1):
                    rb = coff[r] + (zz * ny + yy) * nx
                    home.extend(range(cs[rb + a], cs[rb + b + 1]))
            tables.append((np.array(home, dtype=np.int64), np.array(slots, dtype=np.int64)))
        return tables

    def tile_entries(self):
        """Tile-local list entries as [N, max_nbr] uint16 (entry k of atom i
        sits at (k // 8) * 8 ld + 8 i + k % 8 of the list)."""
        idx = self.idx.cpu().numpy().view(np.uint16)[:self.max_nbr * self.ld]
        idx = idx.reshape(self.max_nbr // 8, self.ld, 8)[:, :self.N, :]
        return np.ascontiguousarray(idx.transpose(1, 0, 2).reshape(self.N, self.max_nbr))

    def list_pairs(self):
        """Verlet list as (id_i, id_j) pairs [P,2] plus decoded image codes
        (image codes are not decoded for tile-local lists: None)."""
        if self.mode == abi.MD_TILE_FULL:
            cnt = self.count.cpu().numpy()
            ent = self.tile_entries()
            ids = self.id.cpu().numpy()
            out = []
            for home, slots in self.tile_slot_table():
                for i in home:
                    n = min(cnt[i], self.max_nbr)
                    js = slots[ent[i, :n].astype(np.int64) >> 3]
                    out.append(np.stack([np.full(n, ids[i]), ids[js]], 1))
            return np.concatenate(out), None
        cnt = self.count.cpu().numpy()
        n = np.minimum(cnt, self.max_nbr)
        idx = self.idx.cpu().numpy().view(np.uint32).reshape(self.max_nbr, self.ld)[:, :self.N]
        k = np.arange(self.max_nbr)[:, None]
        mask = k < n[None, :]
        ent = idx[mask.nonzero()]
        ii = np.nonzero(mask)[1]
        jj = (ent & abi.MD_IDX_MASK).astype(np.int64)
        ids = self.id.cpu().numpy()
        return np.stack([ids[ii], ids[jj]], 1), (ent >> abi.MD_IDX_BITS)
