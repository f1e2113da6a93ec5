"""Oracle adjoint: gradient of the late-time transverse field energy with respect
to the Psi_E coefficients (test infrastructure).

Loss: W = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV after N steps.  The forward
run stores every step's tape (fields after its Yee update, particles before
its push); the reverse sweep calls the C routine o_adj_step for each step in
reverse order (exact transposes, float64).  The gradient is the sum over
steps of <lambda_Et_c, F S_z^j E_c> over the two transverse E components,
which is where Psi_E's coefficient a_j enters (Sec. 2).
"""
import ctypes as C

import numpy as np

from . import ref as _ref

_P = C.POINTER(C.c_double)


def _lib():
    lib = _ref.lib()
    if not getattr(lib, "_adj_ready", False):
        ptr = C.POINTER(_ref._OSim)
        lib.o_adj_step.argtypes = [ptr, _P * 3, _P * 3, _P * 3, _P * 3, _P * 3, _P * 3, _P * 3, _P * 3,
                                   _P * 3, _P * 3, _P * 3, _P]
        lib.o_boris_adj.argtypes = [_P, _P, _P, C.c_double, C.c_double, C.c_double, _P, _P, _P, _P]
        lib.o_dspline.argtypes = [C.c_int, C.c_double]
        lib.o_dspline.restype = C.c_double
        lib._adj_ready = True
    return lib


def _arr3(planes):
    return (_P * 3)(*[_ref._ptr(p) for p in planes])


def wperp(sim):
    return 0.5 * sim.dV * float(np.sum(sim.E[0] ** 2) + np.sum(sim.E[1] ** 2)
                                + np.sum(sim.B[0] ** 2) + np.sum(sim.B[1] ** 2))


def forward_with_tape(sim, nsteps):
    tape = []
    for _ in range(nsteps):
        x0, u0 = sim.x.copy(), sim.u.copy()
        sim.yee()
        tape.append((sim.E.copy(), sim.B.copy(), x0, u0))
        sim.seen()
        sim.push_deposit()
    return tape


def reverse(sim, tape, lE, lB, lJ, lx, lu):
    """Run the reverse sweep over `tape`; the adjoint arrays are updated in place.
    Returns dL/da_j (length psi_deg + 1).  The transposed gather covers the
    Galerkin and Uniform schemes (samples at the Yee locations)."""
    if sim.s.interp == 2:
        raise NotImplementedError("reverse sweep of the momentum-conserving gather")
    if sim.s.correction == 2:
        raise NotImplementedError("reverse sweep of the exact Psi_E / Psi_B ratio")
    lib = _lib()
    grad = np.zeros(max(1, sim.s.psi_deg + 1))
    lEt = np.zeros_like(sim.E)
    lBt = np.zeros_like(sim.B)
    # o_adj_step overwrites sim.E / sim.B / sim.Et / sim.Bt as scratch; the
    # 2D y-component arrays of x, lx are unused but must exist
    for E1, B2, x0, u0 in reversed(tape):
        lib.o_adj_step(C.byref(sim.s), _arr3(E1), _arr3(B2), _arr3(x0), _arr3(u0),
                       _arr3(lE), _arr3(lB), _arr3(lJ), _arr3(lx), _arr3(lu), _arr3(lEt), _arr3(lBt),
                       grad.ctypes.data_as(_P))
    return grad


def loss_and_grad(make_sim, nsteps):
    """make_sim() -> fresh OracleSim.  Returns (W after nsteps, dW/dpsi_e, final sim)."""
    sim = make_sim()
    tape = forward_with_tape(sim, nsteps)
    L = wperp(sim)
    lE = np.zeros_like(sim.E)
    lB = np.zeros_like(sim.B)
    lE[0], lE[1] = sim.dV * sim.E[0], sim.dV * sim.E[1]
    lB[0], lB[1] = sim.dV * sim.B[0], sim.dV * sim.B[1]
    lJ = np.zeros_like(sim.J)
    lx = np.zeros_like(sim.x)
    lu = np.zeros_like(sim.u)
    work = make_sim()        # scratch instance for the reverse sweep
    grad = reverse(work, tape, lE, lB, lJ, lx, lu)
    return L, grad, sim
