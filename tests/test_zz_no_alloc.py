"""GPU test of md_lj_forces_noalloc, the workspace-free variant of
md_lj_forces whose scratch is a fixed array inside the library.

Two calls in a row on one GPU, the second on a smaller system, each compared
with md_lj_forces on the same inputs: the same kernels run in the same
order, so forces, energy and virial must agree bit for bit, and the FP64
results also meet the oracle bar of the parity tests (1e-10 absolute, energy
and virial 1e-12 relative).  The second call must not see the first call's
partial sums, which are still in the shared array.
"""
import ctypes

import numpy as np
import pytest

import md_inputs
import oracle

pytestmark = pytest.mark.gpu

RC = 2.5


def say(msg):
    print(msg, flush=True)


def _system(cfg, mode, prec):
    from paper_2109_10876_amd import MDSystem
    return MDSystem(cfg.natoms, cfg.box, cfg.pos, cfg.vel, cfg.types, cfg.eps, cfg.sig,
                    cfg.mass, rc=cfg.rc, skin=cfg.skin, dt=cfg.dt, shift=cfg.shift, mode=mode,
                    prec=prec)


def _noalloc(s):
    from paper_2109_10876_amd import _abi as abi
    P = ctypes.byref
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    return s.lib.md_lj_forces_noalloc(P(s.batch), P(s.atoms), P(s.nlist), P(s.lj), s.prec, 0,
                                      ptr(s.energy), ptr(s.virial), ptr(s.status), s.stream)


@pytest.mark.parametrize("mode,prec", [("full", "fp64"), ("tile", "fp64"), ("tile", "mixed")])
def test_noalloc_forces_equal_workspace_forces_on_two_calls(mode, prec):
    import torch
    from paper_2109_10876_amd import _abi as abi
    big = md_inputs.lj_fluid(10, temperature=0.72, seed=1, jitter_amp=0.1)    # 4000 atoms
    small = md_inputs.lj_fluid(7, temperature=0.72, seed=3, jitter_amp=0.1)   # 1372 atoms
    systems = []
    for cfg in (big, small):
        s = _system(cfg, mode, prec)
        s.setup()
        assert s.ensure_list() == 0
        systems.append((cfg, s))
    for k, (cfg, s) in enumerate(systems):
        say(f"case: noalloc {mode} {prec} call {k + 1} N={cfg.n}")
        s.forces()
        torch.cuda.synchronize()
        f_ws = s.forces_np().copy()
        e_ws, w_ws = float(s.energy[0]), float(s.virial[0])
        # poison the outputs so that a result not written by the call shows
        for t in (s.fx, s.fy, s.fz, s.energy, s.virial):
            t.fill_(float("nan"))
        rc = _noalloc(s)
        assert rc == abi.MD_OK, abi.strerror(rc)
        torch.cuda.synchronize()
        assert int(s.status[0]) == 0
        f_na = s.forces_np()
        assert np.array_equal(f_na, f_ws)
        assert float(s.energy[0]) == e_ws and float(s.virial[0]) == w_ws
        # no step has run: the oracle takes the input positions (id order)
        ref, e, w = oracle.lj_forces(cfg.pos, cfg.box[0], RC, shift=1)
        err = np.linalg.norm(f_na - ref) / np.linalg.norm(ref)
        say(f"  bitwise equal to md_lj_forces; e_F vs oracle {err:.3e}")
        if prec == "fp64":
            assert np.abs(f_na - ref).max() < 1e-10
            assert float(s.energy[0]) == pytest.approx(e, rel=1e-12)
            assert float(s.virial[0]) == pytest.approx(w, rel=1e-12)
        else:
            assert err < 1e-5
            assert float(s.energy[0]) == pytest.approx(e, rel=1e-6)
            assert float(s.virial[0]) == pytest.approx(w, rel=1e-6)
