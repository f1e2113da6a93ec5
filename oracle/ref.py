"""ctypes wrapper around the C oracle plus numpy diagnostics.

Test infrastructure only: used by tests, the smoke check and the CPU-baseline
timing.  Everything is float64.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build
from . import psi as _psi

_P = C.POINTER(C.c_double)


class _OSim(C.Structure):
    _fields_ = [("dims", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
                ("order", C.c_int), ("interp", C.c_int), ("solver", C.c_int),
                ("q", C.c_double), ("m", C.c_double), ("w", C.c_double),
                ("correction", C.c_int), ("psi_deg", C.c_int),
                ("psi_e", C.c_double * 9), ("psi_b", C.c_double * 9),
                ("nfilt", C.c_int), ("filt", C.c_double * 16), ("jbg", C.c_double * 3),
                ("E", _P * 3), ("B", _P * 3), ("J", _P * 3), ("Et", _P * 3), ("Bt", _P * 3),
                ("tmp", _P), ("tmp2", _P),
                ("np", C.c_long), ("x", _P * 3), ("u", _P * 3), ("status", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = C.CDLL(path)
        ptr = C.POINTER(_OSim)
        for name in ("o_yee", "o_seen", "o_push_deposit"):
            getattr(_lib, name).argtypes = [ptr]
        _lib.o_step.argtypes = [ptr, C.c_int]
        _lib.o_seen_plane.argtypes = [ptr, C.c_int, _P, _P]
        _lib.o_spline.argtypes = [C.c_int, C.c_double]
        _lib.o_spline.restype = C.c_double
        _lib.o_gather.argtypes = [ptr, _P, _P, _P]
        _lib.o_boris.argtypes = [_P, _P, _P, C.c_double, C.c_double, C.c_double]
        _lib.o_deposit.argtypes = [ptr, _P, _P, C.c_double]
        _lib.o_rho.argtypes = [ptr, _P]
        _lib.o_div.argtypes = [ptr, _P * 3, _P]
    return _lib


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def grid_shape(wl):
    """(nz, ny, nx) array shape of a workload's grid (ny = 1 in 2D)."""
    n = wl["n"]
    if wl["dims"] == 2:
        return (n[1], 1, n[0])
    return (n[2], n[1], n[0])


def cell_sizes(wl):
    d = wl.get("d", (1.0,) * wl["dims"])
    if wl["dims"] == 2:
        return (float(d[0]), 1.0, float(d[1]))
    return tuple(float(v) for v in d)


class OracleSim:
    """One simulation instance held in numpy arrays and stepped by the C code.

    wl   : workload dict (see pic_inputs.workloads)
    x, u : loader output, x (N, dims) absolute positions, u (N, 3)
    psi  : optional (a, b) coefficient lists; default computed by psi.py
    """

    def __init__(self, wl, x, u, psi=None, weight=None):
        self.wl = wl
        self.dims = wl["dims"]
        self.shape = grid_shape(wl)
        nz, ny, nx = self.shape
        dx, dy, dz = cell_sizes(wl)
        self.dV = dx * dz if self.dims == 2 else dx * dy * dz
        s = _OSim()
        s.dims, s.nx, s.ny, s.nz = self.dims, nx, ny, nz
        s.dx, s.dy, s.dz = dx, dy, dz
        s.dt = float(wl["alpha"]) * dz
        s.order = int(wl["order"])
        s.interp = {"galerkin": 0, "uniform": 1, "momentum": 2}[wl.get("interp", "galerkin")]
        s.solver = {"yee": 0, "ck": 1}[wl.get("solver", "yee")]
        if s.solver == 1 and (self.dims != 2 or dx != dz):
            raise ValueError("the Cole-Karkkainen solver is taken on square 2D cells only")
        s.q, s.m = float(wl["q"]), float(wl["m"])
        if weight is None:
            n0 = wl["omega_p"] ** 2 * wl["m"] / wl["q"] ** 2
            weight = n0 * self.dV / wl["ppc"]
        s.w = float(weight)
        corr = wl.get("correction")
        s.correction = 2 if corr == "ratio" else (1 if corr else 0)
        if psi is None and s.correction:
            a, b, _ = _psi.psi_coeffs(wl.get("interp", "galerkin"), wl["alpha"])
            psi = (a, b)
        if psi is not None:
            a, b = psi
            s.psi_deg = len(a) - 1
            for i, v in enumerate(a):
                s.psi_e[i] = v
            for i, v in enumerate(b):
                s.psi_b[i] = v
        self.psi = psi
        filt = list(wl.get("filter", []))
        s.nfilt = len(filt)
        for i, v in enumerate(filt):
            s.filt[i] = v
        ncell = nx * ny * nz
        self.E = np.zeros((3,) + self.shape)
        self.B = np.zeros((3,) + self.shape)
        self.J = np.zeros((3,) + self.shape)
        self.Et = np.zeros((3,) + self.shape)
        self.Bt = np.zeros((3,) + self.shape)
        self._tmp = np.zeros(ncell)
        self._tmp2 = np.zeros(ncell)
        for c in range(3):
            s.E[c], s.B[c], s.J[c] = _ptr(self.E[c]), _ptr(self.B[c]), _ptr(self.J[c])
            s.Et[c], s.Bt[c] = _ptr(self.Et[c]), _ptr(self.Bt[c])
        s.tmp, s.tmp2 = _ptr(self._tmp), _ptr(self._tmp2)
        npart = x.shape[0]
        self.x = np.zeros((3, npart))
        if self.dims == 2:
            self.x[0], self.x[2] = x[:, 0], x[:, 1]
        else:
            self.x[:] = x.T
        self.u = np.ascontiguousarray(u.T, dtype=np.float64).copy()
        s.np = npart
        for c in range(3):
            s.x[c], s.u[c] = _ptr(self.x[c]), _ptr(self.u[c])
        # uniform ion background current: minus the beam's initial mean current
        if wl.get("ion_mode", 1) == 1 and npart:
            g = np.sqrt(1.0 + np.sum(self.u ** 2, axis=0))
            vmean = np.sum(self.u / g, axis=1)
            V = ncell * self.dV
            for c in range(3):
                s.jbg[c] = -s.q * s.w * vmean[c] / V
        self.s = s
        self.step_count = 0
        self.rho0 = self.rho()

    # -- stepping -------------------------------------------------------
    def step(self, n=1):
        lib().o_step(C.byref(self.s), int(n))
        self.step_count += n

    def yee(self):
        lib().o_yee(C.byref(self.s))

    def seen(self):
        lib().o_seen(C.byref(self.s))

    def push_deposit(self):
        lib().o_push_deposit(C.byref(self.s))

    def seen_plane(self, which, plane):
        src = np.ascontiguousarray(plane, dtype=np.float64).reshape(self.shape).copy()
        out = np.zeros(self.shape)
        lib().o_seen_plane(C.byref(self.s), int(which), _ptr(src), _ptr(out))
        return out

    def gather_at(self, pos):
        p = np.ascontiguousarray(pos, dtype=np.float64)
        Eo, Bo = np.zeros(3), np.zeros(3)
        lib().o_gather(C.byref(self.s), _ptr(p), _ptr(Eo), _ptr(Bo))
        return Eo, Bo

    @property
    def status(self):
        return self.s.status

    # -- particles in loader layout ------------------------------------
    def positions(self):
        if self.dims == 2:
            return np.stack([self.x[0], self.x[2]], axis=1)
        return self.x.T.copy()

    def momenta(self):
        return self.u.T.copy()

    # -- diagnostics (all float64) --------------------------------------
    def rho(self):
        out = np.zeros(self.shape)
        lib().o_rho(C.byref(self.s), _ptr(out))
        return out

    def div(self, F):
        arr = (_P * 3)(*[_ptr(F[c]) for c in range(3)])
        out = np.zeros(self.shape)
        lib().o_div(C.byref(self.s), arr, _ptr(out))
        return out

    def gauss_residual(self):
        """div E^{n+1} - (rho^{n+1} - rho^0), with div E^{n+1} = div E^n - dt div J^{n+1/2}.

        After a step the grid holds E^n, J^{n+1/2} and particles at x^{n+1}; the
        curl of B has no divergence, so the next E's divergence needs only J.
        Zero (to rounding) when the deposit conserves charge exactly."""
        dE = self.div(self.E) - self.s.dt * self.div(self.J)
        return dE - (self.rho() - self.rho0)

    def energies(self):
        gam = np.sqrt(1.0 + np.sum(self.u ** 2, axis=0))
        WE = 0.5 * self.dV * np.sum(self.E.reshape(3, -1) ** 2, axis=1)
        WB = 0.5 * self.dV * np.sum(self.B.reshape(3, -1) ** 2, axis=1)
        Wkin = self.s.w * self.s.m * float(np.sum(gam - 1.0))
        return dict(WE=WE, WB=WB, Wkin=Wkin,
                    Wperp=float(WE[0] + WE[1] + WB[0] + WB[1]))

    def diag(self):
        d = self.energies()
        R = self.gauss_residual()
        d["gauss_l2"] = float(np.sqrt(np.sum(R ** 2)))
        d["gauss_linf"] = float(np.max(np.abs(R)))
        d["charge"] = float(np.sum(self.rho()) * self.dV)
        d["nonfinite"] = int(not (np.all(np.isfinite(self.E)) and np.all(np.isfinite(self.B))
                                  and np.all(np.isfinite(self.u))))
        return d
