"""GPU reverse mode against the oracle's adjoint and against finite differences.

Gradient of W = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV after N steps with
respect to the Psi_E coefficients.  FP64 GPU vs the FP64 oracle adjoint:
relative 1e-8; FP32 GPU vs the FP64 oracle adjoint: relative 1e-2 (FP32
rounding amplified through the run); FP32 GPU vs FP64 central differences
(h = 1e-6) at the 256x256, 8 ppc, 200-step size: relative 1e-2.
"""
import sys
import time

import numpy as np
import pytest

import pic_inputs as pi
from oracle import adjoint as OA
from oracle.ref import OracleSim

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(dims, n, order, ppc=2, gamma=4.0, seed=3, sigma=0.05, interp="galerkin", solver="yee", alpha=None):
    base = "beam2d_64_fp64" if dims == 2 else "beam3d_128x128x256"
    if alpha is None:
        alpha = 0.45 if dims == 2 else 0.4
    wl = pi.workload(base, n=n, ppc=ppc, order=order, correction=True, filter=pi.workloads.BINOMIAL4,
                     gamma=gamma, alpha=alpha, interp=interp, solver=solver)
    x, u = pi.load_beam(dims, n, ppc, gamma, sigma, seed)
    rng = np.random.default_rng(seed)
    shape = (3,) + ((n[1], 1, n[0]) if dims == 2 else (n[2], n[1], n[0]))
    E0 = rng.normal(size=shape) * 1e-3
    B0 = rng.normal(size=shape) * 1e-3
    return wl, x, u, E0, B0


def _gpu(wl, x, u, E0, B0, prec, nsteps, ckpt, psi=None):
    from paper_1401_0838_amd.sim import Simulation
    sim = Simulation(wl, (x, u), precision=prec, adjoint_steps=nsteps, adjoint_ckpt=ckpt,
                     psi=None if psi is None else [psi])
    for c in range(3):
        sim.set_field("E", c, E0[c])
        sim.set_field("B", c, B0[c])
    return sim


def _oracle(wl, x, u, E0, B0, nsteps):
    def mk():
        s = OracleSim(wl, x, u)
        s.E[:] = E0
        s.B[:] = B0
        return s
    return OA.loss_and_grad(mk, nsteps)


@pytest.mark.parametrize("dims,n,order,nsteps,ckpt", [(2, (32, 32), 1, 30, 10), (2, (24, 32), 3, 12, 5),
                                                      (3, (8, 8, 12), 1, 8, 4)])
def test_adjoint_fp64_matches_oracle(dims, n, order, nsteps, ckpt):
    wl, x, u, E0, B0 = _setup(dims, n, order)
    _say("adjoint fp64 %s order %d steps %d" % (n, order, nsteps))
    L_ref, g_ref, ref = _oracle(wl, x, u, E0, B0, nsteps)
    sim = _gpu(wl, x, u, E0, B0, "fp64", nsteps, ckpt)
    L = sim.adjoint_forward(nsteps)[0]
    g = sim.adjoint_backward()[0]
    _say("  L %.12e ref %.12e  g %s ref %s" % (L, L_ref, g, g_ref))
    assert abs(L - L_ref) < 1e-10 * L_ref
    assert np.max(np.abs(g - g_ref)) < 1e-8 * np.max(np.abs(g_ref))
    # the state is back at the end of the forward run
    assert np.linalg.norm(sim.fields("E") - ref.E) < 1e-10 * np.linalg.norm(ref.E)
    sim.close()


@pytest.mark.parametrize("dims,n,order,nsteps,ckpt,interp,solver,alpha", [
    (2, (32, 32), 1, 30, 10, "uniform", "yee", 0.45), (2, (24, 32), 3, 12, 5, "uniform", "yee", 0.45),
    (3, (8, 8, 12), 1, 8, 4, "uniform", "yee", None), (2, (32, 32), 1, 30, 10, "galerkin", "ck", 0.9),
    (2, (24, 32), 3, 12, 5, "uniform", "ck", 0.95)])
def test_adjoint_schemes_and_ck_fp64_match_oracle(dims, n, order, nsteps, ckpt, interp, solver, alpha):
    """The reverse sweep with the Uniform gather and with the Cole-Karkkainen
    solver (alpha up to 0.95), FP64, against the oracle's adjoint."""
    wl, x, u, E0, B0 = _setup(dims, n, order, interp=interp, solver=solver, alpha=alpha)
    _say("adjoint fp64 %s order %d steps %d %s %s alpha %s" % (n, order, nsteps, interp, solver, alpha))
    L_ref, g_ref, ref = _oracle(wl, x, u, E0, B0, nsteps)
    sim = _gpu(wl, x, u, E0, B0, "fp64", nsteps, ckpt)
    L = sim.adjoint_forward(nsteps)[0]
    g = sim.adjoint_backward()[0]
    _say("  L %.12e ref %.12e  g %s ref %s" % (L, L_ref, g, g_ref))
    assert abs(L - L_ref) < 1e-10 * L_ref
    assert np.max(np.abs(g - g_ref)) < 1e-8 * np.max(np.abs(g_ref))
    sim.close()
    # FP32 within the FP32 bar
    sim = _gpu(wl, x, u, E0, B0, "fp32", nsteps, ckpt)
    sim.adjoint_forward(nsteps)
    g32 = sim.adjoint_backward()[0]
    sim.close()
    assert np.max(np.abs(g32 - g_ref)) < 1e-2 * np.max(np.abs(g_ref))


def test_adjoint_fp32_close_to_oracle_and_autograd():
    import torch
    from paper_1401_0838_amd import autograd as AG
    wl, x, u, E0, B0 = _setup(2, (32, 32), 1)
    nsteps = 30
    L_ref, g_ref, _ = _oracle(wl, x, u, E0, B0, nsteps)
    sim = _gpu(wl, x, u, E0, B0, "fp32", nsteps, 10)
    L = sim.adjoint_forward(nsteps)[0]
    g = sim.adjoint_backward()[0]
    _say("fp32 L %.8e ref %.8e g %s ref %s" % (L, L_ref, g, g_ref))
    assert abs(L - L_ref) < 1e-4 * L_ref
    assert np.max(np.abs(g - g_ref)) < 1e-2 * np.max(np.abs(g_ref))
    a0 = sim.psi()[0]
    sim.close()

    # Psi_B stays at the library's own setup; Psi_E is the differentiated input
    from paper_1401_0838_amd import _lib as Lb
    _, _, b0 = Lb.pic_psi_coeffs(Lb.PIC_GALERKIN, wl["alpha"], 4)

    def make2(psi_e):
        return _gpu(wl, x, u, E0, B0, "fp32", nsteps, 10, psi=(psi_e[0], b0))
    p = torch.tensor(a0[None, :], dtype=torch.float64, requires_grad=True)
    W = AG.wperp(p, make2, nsteps)
    W.sum().backward()
    assert abs(float(W.detach()[0]) - L) <= 1e-6 * L
    assert np.allclose(p.grad.numpy()[0], g, rtol=1e-6, atol=0)


def test_adjoint_many_batched_instances_match_oracle():
    """24 instances of 256x256 reversed in one batched sweep (field tiles run in
    waves): every instance's gradient equals the oracle's."""
    from paper_1401_0838_amd.sim import Simulation
    wl, x, u, E0, B0 = _setup(2, (256, 256), 1, ppc=1)
    nsteps, ninst = 6, 24
    _say("adjoint 24 x 256x256 fp64, %d steps" % nsteps)
    L_ref, g_ref, _ = _oracle(wl, x, u, E0, B0, nsteps)
    sim = Simulation([wl] * ninst, [(x, u)] * ninst, precision="fp64", adjoint_steps=nsteps, adjoint_ckpt=3)
    for i in range(ninst):
        for c in range(3):
            sim.set_field("E", c, E0[c], i)
            sim.set_field("B", c, B0[c], i)
    L = sim.adjoint_forward(nsteps)
    g = sim.adjoint_backward()
    sim.close()
    worst = max(float(np.max(np.abs(gi - g_ref)) / np.max(np.abs(g_ref))) for gi in g)
    _say("  L0 %.12e ref %.12e worst gradient error %.3e" % (L[0], L_ref, worst))
    assert max(abs(Li - L_ref) for Li in L) < 1e-10 * L_ref
    assert worst < 1e-8


def test_adjoint_full_size_fd_and_cost_ratio():
    """256x256, 8 ppc, gamma 130, alpha 0.5, 200 steps with checkpoints every 20:
    FP32 adjoint gradient vs FP64 central differences (h = 1e-6) of the GPU forward,
    and the backward sweep (recompute + reverse) within 3x the plain forward run
    (timed after one warm-up pair that captures the segment graphs)."""
    wl = pi.workload("beam2d_256_adjoint")
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], 0)
    from paper_1401_0838_amd.sim import Simulation
    from paper_1401_0838_amd import _lib as Lb
    nsteps = wl["steps"]
    sim = Simulation(wl, (x, u), precision="fp32", adjoint_steps=nsteps, adjoint_ckpt=wl["checkpoint"])
    # forward-only timing of the same steps (graph replay) for the cost ratio
    fwd = Simulation(wl, (x, u), precision="fp32")
    fwd.step(5)
    fwd.synchronize()
    t0 = time.perf_counter()
    fwd.step(nsteps)
    fwd.synchronize()
    t_plain = time.perf_counter() - t0
    fwd.close()
    tsim = Simulation(wl, (x, u), precision="fp32", adjoint_steps=nsteps, adjoint_ckpt=wl["checkpoint"])
    tsim.adjoint_forward(wl["checkpoint"])
    tsim.adjoint_backward()
    tsim.synchronize()
    t0 = time.perf_counter()
    tsim.adjoint_forward(nsteps)
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    tsim.adjoint_backward()
    t_b = time.perf_counter() - t0
    tsim.close()
    L = sim.adjoint_forward(nsteps)[0]
    g = sim.adjoint_backward()[0]
    a0 = sim.psi()[0]
    sim.close()
    _, _, b0 = Lb.pic_psi_coeffs(Lb.PIC_GALERKIN, wl["alpha"], 4)
    _say("c4: W %.6e grad %s; forward %.3fs (plain %.3fs) backward %.3fs ratio %.2f"
         % (L, g, t_f, t_plain, t_b, t_b / t_plain))

    def W64(a):
        s = Simulation(wl, (x, u), precision="fp64", psi=[(a, b0)])
        s.step(nsteps)
        w = s.diag()["Wperp"]
        s.close()
        return w
    h = 1e-6
    fd = np.array([(W64(a0 + h * e) - W64(a0 - h * e)) / (2 * h) for e in np.eye(len(a0))])
    _say("c4 FD %s" % fd)
    assert np.max(np.abs(g - fd)) < 1e-2 * np.max(np.abs(fd))
    assert t_b / t_plain <= 3.0, (t_b, t_plain)
