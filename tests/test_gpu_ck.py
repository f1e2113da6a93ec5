"""Cole-Karkkainen solver (2D, beta = 1/8) on the GPU against the FP64 oracle.

The paper's 2D runs use this solver so that c dt / dz can approach 1, beyond
the Yee limit 1/sqrt(2) on square cells.  Tolerances as for the Yee path:
FP64 relative L2 <= 1e-10 after 50 steps, FP32 <= 1e-4 after 10.  B starts
from seeded random values (E from zero, so Gauss's law holds) so that the
modified curl acts from the first step.
"""
import math
import sys

import numpy as np
import pytest

import pic_inputs as pi
from oracle.ref import OracleSim

pytestmark = pytest.mark.gpu


def _sim(*a, **k):
    from paper_1401_0838_amd.sim import Simulation
    return Simulation(*a, **k)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(wl, nsteps, precision, seed=0, amp=1e-3):
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], seed)
    _say("case ck n=%s alpha=%g order=%d interp=%s prec=%s steps=%d np=%d" % (
        wl["n"], wl["alpha"], wl["order"], wl["interp"], precision, nsteps, x.shape[0]))
    sim = _sim(wl, (x, u), precision=precision)
    ref = OracleSim(wl, x, u)
    if amp:
        B0 = np.random.default_rng(200 + seed).normal(size=ref.B.shape) * amp
        ref.B[:] = B0
        for c in range(3):
            sim.set_field("B", c, B0[c])
    sim.step(nsteps)
    ref.step(nsteps)
    return sim, ref


def _errors(sim, ref, wl):
    errs = {k: _rel(sim.fields(k), getattr(ref, k)) for k in ("E", "B", "J")}
    x, u = sim.particles()
    L = np.array(wl["n"], float)
    dx = np.abs(x - ref.positions())
    dx = np.minimum(dx, L - dx)
    errs["x"] = float(dx.max())
    errs["u"] = _rel(u, ref.momenta())
    return errs


def test_ck_vacuum_standing_mode_fp64():
    """A TM standing mode at alpha = 0.95 (above the Yee limit): the GPU matches
    the oracle and the scheme's closed-form frequency over 300 steps."""
    wl = pi.workload("beam2d_64_fp64", n=(48, 32), correction=False, filter=[], alpha=0.95, solver="ck")
    x, u = np.zeros((0, 2)), np.zeros((0, 3))
    sim = _sim(wl, (x, u), precision="fp64")
    ref = OracleSim(wl, x, u)
    nz, ny, nx = ref.shape
    kx, kz = 2 * math.pi * 3 / nx, 2 * math.pi * 5 / nz
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz)[:, None, None]
    mode = np.cos(kx * (i + 0.5)) * np.cos(kz * (k + 0.5)) * np.ones((1, 1, 1))
    sim.set_field("B", 1, mode)
    ref.B[1][:] = mode
    sim.step(300)
    for _ in range(300):
        ref.yee()
    assert _rel(sim.fields("E"), ref.E) < 1e-12
    assert _rel(sim.fields("B"), ref.B) < 1e-12
    dt = 0.95
    sx, sz = math.sin(kx / 2) ** 2, math.sin(kz / 2) ** 2
    w = 2 / dt * math.asin(dt * math.sqrt(sx * (1 - sz / 2) + sz * (1 - sx / 2)))
    assert np.max(np.abs(sim.field("B", 1) - math.cos(300 * w * dt) * mode)) < 1e-10


@pytest.mark.parametrize("alpha", [0.5, 0.9, 0.99])
@pytest.mark.parametrize("corr", [False, True])
def test_ck_beam_fp64_parity_50_steps(alpha, corr):
    wl = pi.workload("beam2d_64_fp64", alpha=alpha, solver="ck", correction=corr,
                     filter=pi.workloads.BINOMIAL4 if corr else [])
    sim, ref = _pair(wl, 50, "fp64")
    errs = _errors(sim, ref, wl)
    _say("  alpha %g corr %s %s" % (alpha, corr, errs))
    assert errs["E"] < 1e-10 and errs["B"] < 1e-10 and errs["J"] < 1e-10
    assert errs["x"] < 1e-9 and errs["u"] < 1e-10
    d = sim.diag()
    assert d["rc"] == 0 and d["nonfinite"] == 0 and d["particle_error"] == 0
    assert d["gauss_linf"] < 1e-11 * d["rho_max"]
    sim.close()


@pytest.mark.parametrize("interp", ["galerkin", "uniform", "momentum"])
def test_ck_fp32_parity_10_steps(interp):
    wl = pi.workload("beam2d_64_fp64", alpha=0.9, solver="ck", correction=True,
                     filter=pi.workloads.BINOMIAL4, interp=interp)
    sim, ref = _pair(wl, 10, "fp32")
    errs = _errors(sim, ref, wl)
    _say("  fp32 %s %s" % (interp, errs))
    assert errs["E"] < 1e-4 and errs["B"] < 1e-4 and errs["J"] < 1e-4
    assert errs["x"] < 1e-5 and errs["u"] < 1e-6
    sim.close()


def test_ck_paper_setting_cubic_eq6_fp64():
    """The Sec. 3 setting (cubic shapes, Eq. 6 filter, correction, alpha = 0.9)
    on a ragged 50 x 70 grid, 30 steps."""
    wl = pi.workload("beam2d_128_ck", n=(50, 70), ppc=4)
    sim, ref = _pair(wl, 30, "fp64")
    errs = _errors(sim, ref, wl)
    _say("  paper setting %s" % errs)
    assert max(errs["E"], errs["B"], errs["J"], errs["u"]) < 1e-10
    sim.close()


@pytest.mark.parametrize("prec,steps,tol", [("fp64", 50, 1e-10), ("fp32", 10, 1e-4)])
def test_ck_sqrt_eq6_filter_one_pass_each(prec, steps, tol):
    """Sec. 4's filter with one bilinear and one compensation pass per axis (the
    square root of Eq. 6) in the Sec. 3 setting (cubic, CK, correction,
    alpha = 0.9) on a ragged 50 x 70 grid: fields, current and particles follow
    the oracle (FP64 within 1e-10 after 50 steps, FP32 within 1e-4 after 10)."""
    wl = pi.workload("beam2d_128_ck", n=(50, 70), ppc=4, filter=pi.workloads.PAPER_EQ6_SQRT)
    sim, ref = _pair(wl, steps, prec)
    errs = _errors(sim, ref, wl)
    _say("  sqrt eq6 %s %s" % (prec, errs))
    assert max(errs["E"], errs["B"], errs["J"]) < tol
    sim.close()


def test_ck_batched_matches_oracle_plain_and_tile_heights():
    """Two CK instances in one batch match their oracles; FP32 results are
    bitwise the same batched or plain and for every Yee tile height."""
    wls = [pi.workload("beam2d_512", n=(64, 32), alpha=0.8, ppc=4, solver="ck", tag="a"),
           pi.workload("beam2d_512", n=(32, 96), alpha=0.95, ppc=4, gamma=10.0, solver="ck", tag="b")]
    parts = [pi.load_beam(2, w["n"], w["ppc"], w["gamma"], 1e-3, 40 + i) for i, w in enumerate(wls)]
    sim = _sim(wls, parts, precision="fp64")
    sim.step(20)
    for i, (w, (x, u)) in enumerate(zip(wls, parts)):
        ref = OracleSim(w, x, u)
        ref.step(20)
        e = max(_rel(sim.fields(k, i), getattr(ref, k)) for k in ("E", "B", "J"))
        _say("  ck batched inst %d err %.3e" % (i, e))
        assert e < 1e-10
    sim.close()
    res = []
    for sched, tz in (("batched", 8), ("plain", 8), ("batched", 4), ("batched", 16)):
        sim = _sim(wls, parts, precision="fp32")
        sim.set_schedule(sched, True)
        sim.set_option("yee_tile_z", tz)
        sim.step(12)
        res.append([sim.fields(k, i) for i in range(2) for k in ("E", "B")])
        sim.close()
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert np.array_equal(a, b)


def test_ck_full_size_512_fp32_parity_10_steps():
    """512 x 512, 16 particles per cell, alpha = 0.9 with the CK solver, FP32,
    batched with graphs (the configuration the benchmark times for CK)."""
    wl = pi.workload("beam2d_512", alpha=0.9, solver="ck")
    sim, ref = _pair(wl, 10, "fp32", amp=0.0)
    errs = _errors(sim, ref, wl)
    _say("  512 ck fp32 %s" % errs)
    assert errs["E"] < 1e-4 and errs["B"] < 1e-4 and errs["J"] < 1e-4
    d = sim.diag()
    assert d["gauss_linf"] < 1e-5 * d["rho_max"]
    sim.close()
