"""GPU: the autograd Function over md_lj_forces / md_lj_forces_vjp.

Checks the backward against central finite differences of the forward (both
on the GPU, FP64) and against the oracle's analytic gradient, and runs a few
steps of force matching (fitting eps/sigma to reference forces)."""
import numpy as np
import pytest

import md_inputs
import oracle

pytestmark = pytest.mark.gpu


def _system(cfg, prec="fp64", mode="full"):
    from paper_2109_10876_amd import MDSystem
    s = MDSystem(cfg.natoms, cfg.box, cfg.pos, cfg.vel, cfg.types, cfg.eps, cfg.sig, cfg.mass,
                 rc=cfg.rc, skin=cfg.skin, prec=prec, mode=mode)
    s.setup()
    s.ensure_list()
    return s


@pytest.fixture(scope="module")
def case():
    return md_inputs.replica_batch(nrep=2, nmin=1500, nmax=3000, seed=31)


@pytest.mark.parametrize("mode", ["full", "tile"])
def test_backward_matches_finite_differences(case, mode):
    import torch
    from paper_2109_10876_amd.autograd import lj_forces
    print(f"case: autograd fd {mode}", flush=True)
    s = _system(case, mode=mode)
    dev = s.dev
    pos0 = torch.stack([s.x, s.y, s.z], 1).clone()
    eps0 = torch.tensor(case.eps, device=dev)
    sig0 = torch.tensor(case.sig, device=dev)
    g = torch.Generator(device="cpu").manual_seed(0)
    G = torch.randn(s.N, 3, generator=g, dtype=torch.float64).to(dev)
    gE = torch.randn(s.R, generator=g, dtype=torch.float64).to(dev)

    def loss(p, e, sg):
        F, E = lj_forces(s, p, e, sg)
        return (F * G).sum() + (E * gE).sum()

    p = pos0.clone().requires_grad_(True)
    e = eps0.clone().requires_grad_(True)
    sg = sig0.clone().requires_grad_(True)
    loss(p, e, sg).backward()
    h = 1e-6
    v = torch.randn(s.N, 3, generator=g, dtype=torch.float64).to(dev) * 0.1
    with torch.no_grad():
        fd = (loss(pos0 + h * v, eps0, sig0) - loss(pos0 - h * v, eps0, sig0)) / (2 * h)
        assert float((p.grad * v).sum()) == pytest.approx(float(fd), rel=1e-6)
        sym = torch.tensor([[0.3, -0.7], [-0.7, 1.1]], dtype=torch.float64, device=dev)
        for grad, base, which in ((e.grad, eps0, "eps"), (sg.grad, sig0, "sig")):
            if which == "eps":
                lp, lm = loss(pos0, eps0 + h * sym, sig0), loss(pos0, eps0 - h * sym, sig0)
            else:
                lp, lm = loss(pos0, eps0, sig0 + h * sym), loss(pos0, eps0, sig0 - h * sym)
            fdp = (lp - lm) / (2 * h)
            assert float((grad * sym).sum()) == pytest.approx(float(fdp), rel=1e-6)


def test_backward_matches_oracle_gradient(case):
    import torch
    from paper_2109_10876_amd.autograd import lj_forces
    print("case: autograd vs oracle", flush=True)
    s = _system(case)
    dev = s.dev
    ids = s.id.cpu().numpy()
    pos_sorted = torch.stack([s.x, s.y, s.z], 1).clone().requires_grad_(True)
    eps = torch.tensor(case.eps, device=dev, requires_grad=True)
    sig = torch.tensor(case.sig, device=dev, requires_grad=True)
    rng = np.random.default_rng(3)
    G = rng.normal(size=(s.N, 3))            # by original id
    F, E = lj_forces(s, pos_sorted, eps, sig)
    (F * torch.tensor(G[ids], device=dev)).sum().backward()
    got = np.empty((s.N, 3))
    got[ids] = pos_sorted.grad.cpu().numpy()
    off = case.atom_off()
    geps = np.zeros((2, 2))
    for r in range(case.nrep):
        a, b = off[r], off[r + 1]
        gx, ge, _ = oracle.lj_vjp(case.pos[a:b], case.box[r], case.rc, G[a:b], 0.0, case.eps,
                                  case.sig, case.types[a:b], 1)
        assert np.linalg.norm(got[a:b] - gx) / np.linalg.norm(gx) < 1e-11
        geps += ge
    # symmetric split: mirrored entries each hold half of the shared derivative
    split = np.array([[1.0, 0.5], [0.5, 1.0]])
    np.testing.assert_allclose(eps.grad.cpu().numpy(), geps * split, rtol=1e-10)


def test_force_matching_reduces_the_loss(case):
    import torch
    from paper_2109_10876_amd.autograd import force_matching_loss, lj_forces
    print("case: force matching", flush=True)
    s = _system(case, prec="mixed")
    dev = s.dev
    pos = torch.stack([s.x, s.y, s.z], 1).clone()
    # reference forces at a second parameter set (target of the fit)
    eps_ref = torch.tensor([[1.05, 0.9], [0.9, 1.15]], dtype=torch.float64, device=dev)
    sig_ref = torch.tensor([[1.0, 1.05], [1.05, 0.95]], dtype=torch.float64, device=dev)
    with torch.no_grad():
        f_ref, _ = lj_forces(s, pos, eps_ref, sig_ref)
    eps = torch.tensor(case.eps, device=dev, requires_grad=True)
    sig = torch.tensor(case.sig, device=dev, requires_grad=True)
    opt = torch.optim.Adam([eps, sig], lr=5e-3)
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss = force_matching_loss(s, pos, eps, sig, f_ref)
        loss.backward()
        with torch.no_grad():   # keep the tables symmetric
            eps.grad.copy_(0.5 * (eps.grad + eps.grad.t()))
            sig.grad.copy_(0.5 * (sig.grad + sig.grad.t()))
        opt.step()
        losses.append(float(loss.detach()))
    assert losses[-1] < 0.5 * losses[0]
