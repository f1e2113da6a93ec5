"""Python front end of the GPU PIC step: device memory and streams from torch,
every step of the method in the HIP library (libpic.so).

A `Simulation` binds one or more instances (a batch) to one torch-allocated
device arena and one torch stream.  Workloads are the plain parameter dicts of
pic_inputs.workloads (dims, n, alpha, gamma, ppc, order, correction, filter,
precision, ...).
"""
import ctypes as C

import numpy as np

from . import _lib as L


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the PIC step runs on the GPU only; no GPU is visible")
    return torch


def make_config(wl, precision=None, tile=None, block=0, trace_capacity=0, psi=None, adjoint_steps=0,
                adjoint_ckpt=20):
    """pic_config for one workload dict.  The correction coefficients come from
    the library's own rational-interpolation setup unless `psi` is given."""
    c = L.pic_config()
    dims = int(wl["dims"])
    n = tuple(int(v) for v in wl["n"])
    d = tuple(float(v) for v in wl.get("d", (1.0,) * dims))
    c.dims = dims
    if dims == 2:
        c.nx, c.ny, c.nz = n[0], 1, n[1]
        c.dx, c.dy, c.dz = d[0], 1.0, d[1]
        dV = d[0] * d[1]
    else:
        c.nx, c.ny, c.nz = n
        c.dx, c.dy, c.dz = d
        dV = d[0] * d[1] * d[2]
    c.cdt = float(wl["alpha"]) * c.dz
    c.shape_order = int(wl["order"])
    c.interp = {"galerkin": L.PIC_GALERKIN, "uniform": L.PIC_UNIFORM,
                "momentum": L.PIC_MOMENTUM}[wl.get("interp", "galerkin")]
    c.solver = {"yee": L.PIC_YEE, "ck": L.PIC_CK}[wl.get("solver", "yee")]
    prec = precision or wl.get("precision", "fp32")
    c.precision = L.PIC_FP32 if prec == "fp32" else L.PIC_FP64
    corr = wl.get("correction")
    c.correction = L.PIC_CORR_RATIO if corr == "ratio" else (L.PIC_CORR_SPLIT if corr else L.PIC_CORR_NONE)
    if c.correction:
        if psi is None:
            rc, a, b = L.pic_psi_coeffs(c.interp, float(wl["alpha"]), 4)
            L.check(rc, "pic_psi_coeffs(alpha=%g)" % wl["alpha"])
        else:
            a, b = psi
        c.psi_deg = len(a) - 1
        for i, v in enumerate(a):
            c.psi_e[i] = float(v)
        for i, v in enumerate(b):
            c.psi_b[i] = float(v)
    filt = list(wl.get("filter", []))
    c.filter_npass = len(filt)
    for i, v in enumerate(filt):
        c.filter_w[i] = float(v)
    c.q, c.m = float(wl["q"]), float(wl["m"])
    n0 = wl["omega_p"] ** 2 * wl["m"] / wl["q"] ** 2
    c.weight = float(wl["weight"]) if "weight" in wl else n0 * dV / wl["ppc"]
    c.ion_mode = int(wl.get("ion_mode", 1))
    t = tile or wl.get("tile") or (0, 0, 0)
    for i in range(3):
        c.tile[i] = int(t[i])
    c.block = int(block)
    c.trace_capacity = int(trace_capacity)
    c.adjoint_steps = int(adjoint_steps)
    c.adjoint_ckpt = int(adjoint_ckpt) if adjoint_steps else 0
    return c


class Simulation:
    """Instances stepped together on one GPU.

    workloads : list of workload dicts
    particles : list of (x, u) loader arrays, x (N, dims) absolute positions, u (N, 3)
    static_arena : take the arena from the library's static device array
                   (pic_init_static, 64 MiB, one live state per device) instead
                   of allocating it
    tuned : take the tile, workgroup size, launch options and schedule from
            the autotuner's cache (tune.py; the tuner is not run here).  The
            entry, or None when the batch has none, is kept in self.tuning
    """

    def __init__(self, workloads, particles, precision=None, tile=None, block=0,
                 trace_capacity=0, psi=None, stream=None, adjoint_steps=0, adjoint_ckpt=20,
                 static_arena=False, tuned=False):
        torch = _require_gpu()
        L.load()
        if isinstance(workloads, dict):
            workloads, particles = [workloads], [particles]
        self.workloads = list(workloads)
        self.dims = int(self.workloads[0]["dims"])
        self.tuning = None
        pick = None
        if tuned:
            from . import tune
            prec = precision or self.workloads[0].get("precision", "fp32")
            pick = tune.lookup(self.workloads, prec)
            self.tuning = {"key": tune.key(self.workloads, prec), "pick": pick}
            if pick is not None and tile is None and not block:
                tile, block = tuple(pick["tile"]), int(pick["block"])
        self.cfgs = [make_config(wl, precision, tile, block, trace_capacity,
                                 None if psi is None else psi[i], adjoint_steps, adjoint_ckpt)
                     for i, wl in enumerate(self.workloads)]
        self.n_inst = len(self.cfgs)
        self.np = [int(p[0].shape[0]) for p in particles]
        nbytes = L.pic_plan(self.cfgs, self.np)
        if static_arena:
            # the library's static device array (pic_init_static): nothing allocated here
            self.arena = None
        else:
            self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            aligned = (self.arena.data_ptr() + 255) & ~255
        self.stream = stream or torch.cuda.Stream()
        keep = []
        parts = []
        for (x, u), cfg in zip(particles, self.cfgs):
            x = np.asarray(x, dtype=np.float64)
            u = np.asarray(u, dtype=np.float64)
            if self.dims == 2:
                cols = [np.ascontiguousarray(x[:, 0]), None, np.ascontiguousarray(x[:, 1])]
            else:
                cols = [np.ascontiguousarray(x[:, a]) for a in range(3)]
            mom = [np.ascontiguousarray(u[:, a]) for a in range(3)]
            keep.append((cols, mom))
            p = L.pic_particles()
            p.n = x.shape[0]
            for a in range(3):
                p.pos[a] = L.dptr(cols[a]) if cols[a] is not None else None
                p.mom[a] = L.dptr(mom[a])
            parts.append(p)
        torch.cuda.synchronize()
        if static_arena:
            self.st = L.pic_init_static(self.cfgs, parts, self.stream.cuda_stream)
        else:
            self.st = L.pic_init(self.cfgs, parts, aligned, nbytes, self.stream.cuda_stream)
        self.steps_taken = 0
        if pick is not None:
            for name, value in pick.get("options", {}).items():
                self.set_option(name, value)
            self.set_schedule(pick.get("schedule", "batched"), True)

    # ------------------------------------------------------------ stepping
    def step(self, n=1):
        L.pic_step(self.st, n)
        self.steps_taken += n

    def prepare(self, n):
        """Capture the graphs a following step(n) replays (no stepping)."""
        L.pic_prepare(self.st, n)

    def set_schedule(self, sched="batched", use_graph=True):
        L.pic_set_schedule(self.st, L.PIC_SCHED_BATCHED if sched == "batched" else L.PIC_SCHED_PLAIN,
                           1 if use_graph else 0)

    def set_option(self, name, value):
        L.pic_set_option(self.st, name, value)

    def get_option(self, name):
        return L.pic_get_option(self.st, name)

    def synchronize(self):
        self.stream.synchronize()

    # -------------------------------------------------------------- access
    def grid_shape(self, inst=0):
        c = self.cfgs[inst]
        return (c.nz, c.ny, c.nx)

    def field(self, which, comp, inst=0):
        which = {"E": L.PIC_FIELD_E, "B": L.PIC_FIELD_B, "J": L.PIC_FIELD_J, "Et": L.PIC_FIELD_SEEN_E,
                 "Bt": L.PIC_FIELD_SEEN_B, "rho": L.PIC_FIELD_RHO}[which]
        out = np.zeros(self.grid_shape(inst))
        L.pic_fields(self.st, inst, which, comp, out, L.PIC_GET)
        return out

    def fields(self, which, inst=0):
        return np.stack([self.field(which, c, inst) for c in range(3)])

    def set_field(self, which, comp, values, inst=0):
        which = {"E": L.PIC_FIELD_E, "B": L.PIC_FIELD_B}[which]
        arr = np.ascontiguousarray(np.broadcast_to(values, self.grid_shape(inst)), dtype=np.float64).copy()
        L.pic_fields(self.st, inst, which, comp, arr, L.PIC_SET)

    def particles(self, inst=0):
        n = self.np[inst]
        pos = [np.zeros(n), np.zeros(n) if self.dims == 3 else None, np.zeros(n)]
        mom = [np.zeros(n) for _ in range(3)]
        L.pic_get_particles(self.st, inst, pos, mom, n)
        if self.dims == 2:
            x = np.stack([pos[0], pos[2]], axis=1)
        else:
            x = np.stack(pos, axis=1)
        return x, np.stack(mom, axis=1)

    def diag(self, inst=0, check=False):
        rc, d = L.pic_diag(self.st, inst)
        if check:
            L.check(rc, "pic_diag")
        out = dict(WE=np.array(d.WE[:]), WB=np.array(d.WB[:]), Wkin=d.Wkin, gauss_l2=d.gauss_l2,
                   gauss_linf=d.gauss_linf, charge=d.charge, rho_max=d.rho_max,
                   n_particles=d.n_particles, step=d.step, nonfinite=d.nonfinite,
                   particle_error=d.particle_error, resorts=d.resorts, slow_tiles=d.slow_tiles,
                   current_range=d.current_range, rc=rc)
        out["Wperp"] = float(out["WE"][0] + out["WE"][1] + out["WB"][0] + out["WB"][1])
        return out

    def trace(self, inst=0, max_rows=1 << 20):
        buf = np.zeros((min(max_rows, max(1, self.cfgs[inst].trace_capacity)), 6))
        n = L.pic_read_trace(self.st, inst, buf)
        return buf[:n]

    def profile(self, nsteps):
        t = L.pic_profile(self.st, nsteps)
        self.steps_taken += nsteps
        return dict(yee_ms=t.yee_ms, seen_ms=t.seen_ms, particle_ms=t.particle_ms,
                    resort_ms=t.resort_ms, step_ms=t.step_ms, steps=t.steps)

    def adjoint_forward(self, nsteps):
        """Run nsteps with checkpoints; returns W per instance."""
        loss = L.pic_adjoint_forward(self.st, nsteps, self.n_inst)
        self.steps_taken += nsteps
        return loss

    def adjoint_backward(self):
        """dW/dpsi_e per instance, shape (n_inst, psi_deg + 1)."""
        g = L.pic_adjoint_backward(self.st, self.n_inst)
        return g[:, : self.cfgs[0].psi_deg + 1]

    def psi(self, inst=0):
        c = self.cfgs[inst]
        return (np.array(c.psi_e[: c.psi_deg + 1]), np.array(c.psi_b[: c.psi_deg + 1]))

    def info(self):
        return L.pic_info(self.st)

    def close(self):
        if getattr(self, "st", None):
            L.pic_destroy(self.st)
            self.st = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
