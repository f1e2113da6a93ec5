"""Pins of the oracle's adjoint (reverse mode with exact transposes).  CPU only.

* the gradient of the late-time transverse field energy with respect to the
  Psi_E coefficients against float64 central finite differences;
* the Yee part as a linear map: <A d, l> = <d, A^T l> (dot-product test);
* the Boris reverse against finite differences of the Boris push.
"""
import ctypes as C

import numpy as np
import pytest

import pic_inputs as pi
from oracle import adjoint as A
from oracle import psi
from oracle.ref import OracleSim, _ptr

_P = C.POINTER(C.c_double)


def _maker(dims, n, order, seed=3, gamma=4.0, ppc=2, interp="galerkin", solver="yee", alpha=None):
    base = "beam2d_64_fp64" if dims == 2 else "beam3d_128x128x256"
    if alpha is None:
        alpha = 0.45 if dims == 2 else 0.4
    wl = pi.workload(base, n=n, ppc=ppc, order=order, correction=True, filter=pi.workloads.BINOMIAL4,
                     gamma=gamma, alpha=alpha, interp=interp, solver=solver)
    x, u = pi.load_beam(dims, n, ppc, gamma, 0.05, seed)
    a0, b0, _ = psi.psi_coeffs(interp, wl["alpha"])

    def mk(a=a0):
        s = OracleSim(wl, x, u, psi=(list(a), b0))
        rng = np.random.default_rng(seed)
        s.E[:] = rng.normal(size=s.E.shape) * 1e-3
        s.B[:] = rng.normal(size=s.B.shape) * 1e-3
        return s
    return mk, np.array(a0)


def _loss(mk, a, nsteps):
    s = mk(list(a))
    s.step(nsteps)
    return A.wperp(s)


@pytest.mark.parametrize("dims,n,order,nsteps,interp,solver,alpha", [
    (2, (16, 24), 1, 30, "galerkin", "yee", None), (2, (16, 16), 3, 12, "galerkin", "yee", None),
    (3, (8, 8, 10), 1, 6, "galerkin", "yee", None), (2, (16, 24), 1, 30, "uniform", "yee", 0.45),
    (3, (8, 8, 10), 3, 4, "uniform", "yee", None), (2, (16, 24), 1, 30, "galerkin", "ck", 0.9),
    (2, (16, 16), 3, 12, "uniform", "ck", 0.9)])
def test_adjoint_gradient_matches_finite_differences(dims, n, order, nsteps, interp, solver, alpha):
    """Also with the Uniform gather and the Cole-Karkkainen solver (alpha 0.9)."""
    mk, a0 = _maker(dims, n, order, interp=interp, solver=solver, alpha=alpha)
    L, g, _ = A.loss_and_grad(lambda: mk(), nsteps)
    assert abs(L - _loss(mk, a0, nsteps)) < 1e-14 * L
    # directional derivative along the gradient (well above the cancellation floor)
    dvec = g / np.linalg.norm(g)
    h = 1e-4
    fd = (_loss(mk, a0 + h * dvec, nsteps) - _loss(mk, a0 - h * dvec, nsteps)) / (2 * h)
    assert abs(fd - g @ dvec) < 1e-6 * abs(g @ dvec), (fd, g @ dvec)
    # each coefficient (h = 1e-3 keeps the float64 cancellation error small)
    for j in range(len(a0)):
        e = np.zeros_like(a0)
        e[j] = 1e-3
        fdj = (_loss(mk, a0 + e, nsteps) - _loss(mk, a0 - e, nsteps)) / 2e-3
        assert abs(fdj - g[j]) < 1e-5 * abs(g[j]) + 1e-9 * np.abs(g).max(), (j, fdj, g[j])


@pytest.mark.parametrize("solver", ["yee", "ck"])
def test_yee_reverse_is_exact_transpose(solver):
    """With no particles the step is linear in (E, B, J); its reverse must be its
    transpose (also with the Cole-Karkkainen curl, on square cells at alpha 0.9)."""
    if solver == "ck":
        wl = pi.workload("beam2d_64_fp64", n=(12, 10), correction=True, filter=pi.workloads.BINOMIAL4,
                         ion_mode=0, solver="ck", alpha=0.9)
    else:
        wl = pi.workload("beam2d_64_fp64", n=(12, 10), correction=True, filter=pi.workloads.BINOMIAL4,
                         ion_mode=0, d=(1.0, 0.8))
    sim = OracleSim(wl, np.zeros((0, 2)), np.zeros((0, 3)))
    rng = np.random.default_rng(1)
    dE, dB, dJ = (rng.normal(size=sim.E.shape) for _ in range(3))
    sim.E[:], sim.B[:], sim.J[:] = dE, dB, dJ
    sim.yee()
    E1, B1 = sim.E.copy(), sim.B.copy()
    lE0, lB0 = rng.normal(size=sim.E.shape), rng.normal(size=sim.B.shape)
    lE, lB = lE0.copy(), lB0.copy()
    lJ = np.zeros_like(lE)
    empty = np.zeros((3, 0))
    lx, lu = np.zeros((3, 0)), np.zeros((3, 0))
    A.reverse(sim, [(E1, B1, empty, empty)], lE, lB, lJ, lx, lu)
    lhs = np.sum(E1 * lE0) + np.sum(B1 * lB0)
    rhs = np.sum(dE * lE) + np.sum(dB * lB) + np.sum(dJ * lJ)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_boris_reverse_matches_finite_differences():
    lib = A._lib()
    rng = np.random.default_rng(7)
    q, m, dt = -1.0, 1.0, 0.45
    for _ in range(10):
        u = rng.normal(size=3) * 3
        E = rng.normal(size=3) * 0.3
        B = rng.normal(size=3) * 0.5
        lun = rng.normal(size=3)

        def push(uu, EE, BB):
            out = np.array(uu, dtype=np.float64)
            lib.o_boris(_ptr(out), _ptr(np.array(EE, float)), _ptr(np.array(BB, float)), q, m, dt)
            return out
        lu, lE, lB = np.zeros(3), np.zeros(3), np.zeros(3)
        lib.o_boris_adj(_ptr(u), _ptr(E), _ptr(B), q, m, dt, _ptr(lun), _ptr(lu), _ptr(lE), _ptr(lB))
        h = 1e-6
        for vec, lv, which in ((u, lu, 0), (E, lE, 1), (B, lB, 2)):
            for k in range(3):
                e = np.zeros(3)
                e[k] = h
                args_p = [u, E, B]
                args_m = [u, E, B]
                args_p[which] = vec + e
                args_m[which] = vec - e
                fd = (push(*args_p) - push(*args_m)) @ lun / (2 * h)
                assert abs(fd - lv[k]) < 1e-8 * (1 + abs(fd))
