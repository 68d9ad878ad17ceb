"""Differentiable LJ forces: torch.autograd.Function over md_lj_forces and its
hand-written adjoint md_lj_forces_vjp.

Forward returns the forces F [N,3] and per-replica energies E [R] of an
MDSystem for given positions and (eps, sigma) tables; backward returns
dL/dpositions and dL/d(eps, sigma) from dL/dF and dL/dE.  Pair terms are
recomputed in the backward kernel; nothing is stored by the forward.

Positions are in the system's current (cell-sorted) atom order and must lie
within half a skin of the positions the system's Verlet list was built from
(the list is not differentiated and not rebuilt here).  The (eps, sigma)
tables are symmetric [ntypes, ntypes]; their gradient follows the symmetric
convention: an off-diagonal parameter appears in two mirrored entries, each
receiving half of its derivative, so a symmetric perturbation of the table
changes the loss by exactly sum(grad * delta).
"""
from __future__ import annotations

import torch

from . import _abi as abi


def _set_state(system, pos, eps, sig):
    with torch.no_grad():
        system.x.copy_(pos[:, 0])
        system.y.copy_(pos[:, 1])
        system.z.copy_(pos[:, 2])
        if system.pos4 is not None:
            system.pos4.view(-1, 4)[:, :3].copy_(pos)
        system.eps_t.copy_(eps.reshape(-1))
        system.sig_t.copy_(sig.reshape(-1))


class LJForces(torch.autograd.Function):
    """(pos [N,3], eps [nt,nt], sig [nt,nt]) -> (F [N,3], E [R]) on a full list
    (global-index or tile-local)."""

    @staticmethod
    def forward(ctx, pos, eps, sig, system):
        if system.mode not in (abi.MD_FULL, abi.MD_TILE_FULL):
            raise ValueError("LJForces needs a full Verlet list (mode='full' or 'tile')")
        pos = pos.detach().to(torch.float64).contiguous()
        eps = eps.detach().to(torch.float64).contiguous()
        sig = sig.detach().to(torch.float64).contiguous()
        _set_state(system, pos, eps, sig)
        system.forces()
        F = torch.stack([system.fx, system.fy, system.fz], dim=1).clone()
        E = system.energy.clone()
        ctx.system = system
        ctx.save_for_backward(pos, eps, sig)
        return F, E

    @staticmethod
    def backward(ctx, gF, gE):
        system = ctx.system
        pos, eps, sig = ctx.saved_tensors
        _set_state(system, pos, eps, sig)
        N, nt = system.N, system.ntypes
        dev = system.dev
        if gF is None:
            gF = torch.zeros(N, 3, dtype=torch.float64, device=dev)
        gF = gF.to(torch.float64)
        gfx, gfy, gfz = (gF[:, k].contiguous() for k in range(3))
        gEt = gE.to(torch.float64).contiguous() if gE is not None else None
        gx = torch.empty(3 * N, dtype=torch.float64, device=dev)
        geps = torch.empty(nt * nt, dtype=torch.float64, device=dev)
        gsig = torch.empty(nt * nt, dtype=torch.float64, device=dev)
        system.vjp(gfx, gfy, gfz, gEt, gx, geps, gsig)
        gpos = gx.view(3, N).t().contiguous()
        # shared-parameter derivative -> symmetric per-entry split
        split = torch.full((nt, nt), 0.5, dtype=torch.float64, device=dev)
        split.fill_diagonal_(1.0)
        return gpos, geps.view(nt, nt) * split, gsig.view(nt, nt) * split, None


def lj_forces(system, pos, eps, sig):
    """Differentiable (F, E) of ``system`` at positions ``pos``."""
    return LJForces.apply(pos, eps, sig, system)


def force_matching_loss(system, pos, eps, sig, f_ref):
    """Mean squared force error sum |F(eps, sig) - F_ref|^2 / (3N), the loss of
    force-field fitting; differentiable in pos, eps and sig."""
    F, _ = lj_forces(system, pos, eps, sig)
    return ((F - f_ref) ** 2).sum() / F.numel()
