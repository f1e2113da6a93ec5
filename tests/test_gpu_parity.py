"""GPU path (libpic.so through the C ABI) against the FP64 oracle.

Tolerances: FP64 fields relative L2 <= 1e-10 after 50 steps; FP32 <= 1e-4
after 10 steps (relative L2 over each field vector).  Inputs are seeded
synthetic beams from pic_inputs, identical on both sides.
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


def _pair(wl, nsteps, precision, seed=0, sigma=None, x=None, u=None):
    if x is None:
        x, u = pi.load_beam(wl["dims"], wl["n"], wl["ppc"], wl["gamma"],
                            wl["sigma"] if sigma is None else sigma, seed)
    _say("case %s n=%s prec=%s steps=%d np=%d" % (wl.get("name"), wl["n"], precision, nsteps, x.shape[0]))
    sim = _sim(wl, (x, u), precision=precision)
    ref = OracleSim(wl, x, u)
    sim.step(nsteps)
    ref.step(nsteps)
    return sim, ref


def _field_errors(sim, ref):
    return {k: _rel(sim.fields(k), getattr(ref, k)) for k in ("E", "B", "J")}


def _particle_errors(sim, ref, wl):
    x, u = sim.particles()
    rx = ref.positions()
    L = np.array(wl["n"], float) * np.array(wl.get("d", (1.0,) * wl["dims"]))
    dx = np.abs(x - rx)
    dx = np.minimum(dx, L - dx)
    return float(dx.max()), _rel(u, ref.momenta())


# ------------------------------------------------------------------ Yee

def test_yee_standing_mode_fp64():
    wl = pi.workload("beam2d_64_fp64", n=(48, 32), correction=False, filter=[], alpha=0.45)
    x = np.zeros((0, 2))
    u = np.zeros((0, 3))
    sim = _sim(wl, (x, u), precision="fp64")
    ref = OracleSim(wl, x, u)
    nz, ny, nx = ref.shape
    kx, kz = 2 * math.pi * 3 / nx, 2 * math.pi * 2 / nz
    mode = np.sin(kx * np.arange(nx))[None, None, :] * np.sin(kz * np.arange(nz))[:, None, None]
    sim.set_field("E", 1, mode)
    ref.E[1][:] = mode
    sim.step(300)
    for _ in range(300):
        ref.yee()
    assert _rel(sim.fields("E"), ref.E) < 1e-12
    assert _rel(sim.fields("B"), ref.B) < 1e-12
    dt = 0.45
    w = 2 / dt * math.asin(dt * math.sqrt(math.sin(kx / 2) ** 2 + math.sin(kz / 2) ** 2))
    assert np.max(np.abs(sim.field("E", 1) - math.cos(300 * w * dt) * mode)) < 1e-11


# ------------------------------------------------------------ beam parity

@pytest.mark.parametrize("corr", [False, True])
def test_beam_fp64_parity_50_steps(corr):
    wl = pi.workload("beam2d_64_fp64", correction=corr,
                     filter=pi.workloads.BINOMIAL4 if corr else [])
    sim, ref = _pair(wl, 50, "fp64")
    errs = _field_errors(sim, ref)
    _say("fp64 corr=%s %s" % (corr, errs))
    assert errs["E"] < 1e-10 and errs["B"] < 1e-10 and errs["J"] < 1e-10
    dxm, du = _particle_errors(sim, ref, wl)
    assert dxm < 1e-9 and du < 1e-10
    assert _rel(sim.fields("Et"), ref.Et) < 1e-10
    d = sim.diag()
    assert d["rc"] == 0 and d["nonfinite"] == 0 and d["particle_error"] == 0
    assert d["gauss_linf"] < 1e-11 * d["rho_max"]
    od = ref.diag()
    assert abs(d["Wkin"] - od["Wkin"]) < 1e-10 * od["Wkin"]
    assert abs(d["Wperp"] - od["Wperp"]) <= 1e-9 * od["Wperp"] + 1e-300
    assert abs(d["charge"] - od["charge"]) < 1e-10 * abs(od["charge"])
    sim.close()


def test_beam_fp32_parity_10_steps():
    wl = pi.workload("beam2d_64_fp64", correction=True, filter=pi.workloads.BINOMIAL4)
    sim, ref = _pair(wl, 10, "fp32")
    errs = _field_errors(sim, ref)
    _say("fp32 %s" % errs)
    assert errs["E"] < 1e-4 and errs["B"] < 1e-4 and errs["J"] < 1e-4
    dxm, du = _particle_errors(sim, ref, wl)
    assert dxm < 1e-5 and du < 1e-6
    d = sim.diag()
    assert d["gauss_linf"] < 1e-5 * d["rho_max"]
    sim.close()


@pytest.mark.parametrize("alpha", [0.3, 0.7])
def test_beam_fp64_parity_alpha_scan(alpha):
    wl = pi.workload("beam2d_512", n=(64, 96), alpha=alpha, ppc=4, precision="fp64")
    sim, ref = _pair(wl, 50, "fp64")
    errs = _field_errors(sim, ref)
    _say("alpha %g %s" % (alpha, errs))
    assert max(errs.values()) < 1e-10
    sim.close()


def test_cubic_2d_fp64_parity():
    wl = pi.workload("beam2d_64_fp64", n=(48, 64), order=3, correction=True, filter=pi.workloads.BINOMIAL4)
    sim, ref = _pair(wl, 30, "fp64")
    errs = _field_errors(sim, ref)
    _say("cubic2d %s" % errs)
    assert max(errs.values()) < 1e-10
    sim.close()


@pytest.mark.parametrize("order,prec,tol", [(1, "fp64", 1e-10), (3, "fp64", 1e-10), (1, "fp32", 1e-4),
                                            (3, "fp32", 1e-4)])
def test_3d_parity(order, prec, tol):
    wl = pi.workload("beam3d_128x128x256", n=(16, 12, 24), ppc=2, order=order)
    sim, ref = _pair(wl, 10, prec)
    errs = _field_errors(sim, ref)
    _say("3d order %d %s %s" % (order, prec, errs))
    assert max(errs.values()) < tol
    d = sim.diag()
    assert d["gauss_linf"] < (1e-11 if prec == "fp64" else 1e-5) * d["rho_max"]
    sim.close()


@pytest.mark.parametrize("order,interp", [(1, "galerkin"), (3, "galerkin"), (1, "momentum")])
def test_3d_rows_of_64_parity(order, interp):
    """Grids whose rows are a multiple of 64 cells take the x-direction seen pass
    that stages each wave's row segment (with its wrapped ends) in LDS; the
    other 3D tests (rows of 16 and 32) take the per-tap form.  64 x 8 x 16 and
    128 x 8 x 8 against the oracle after 10 steps: FP64 within 1e-10, FP32
    within 1e-4, with the wider stencil of the momentum-conserving gather too."""
    for n in ((64, 8, 16), (128, 8, 8)):
        wl = pi.workload("beam3d_128x128x256", n=n, ppc=2, order=order, interp=interp)
        x, u = pi.load_beam(3, wl["n"], wl["ppc"], wl["gamma"], 1e-3, 4)
        _say("case 3d rows of 64 n=%s order %d %s" % (n, order, interp))
        ref = OracleSim(wl, x, u)
        ref.step(10)
        for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
            sim = _sim(wl, (x, u), precision=prec)
            sim.step(10)
            errs = _field_errors(sim, ref)
            _say("  %s %s" % (prec, errs))
            assert max(errs.values()) < tol
            sim.close()


def test_3d_batched_rows_of_64_and_ragged_rows():
    """Two 3D instances in one batched launch, one with 64-cell rows (staged x
    pass; 3840 cells, so its second workgroup holds only part of its 2048) and
    one with 40-cell rows (per-tap x pass) and more cells, so the x pass's grid
    is sized by the larger: each against its own oracle (FP64 within 1e-10),
    and the plain schedule equal to the batched one bitwise in FP32."""
    wls = [pi.workload("beam3d_128x128x256", n=(64, 6, 10), ppc=2, order=1, tag="a"),
           pi.workload("beam3d_128x128x256", n=(40, 8, 12), ppc=2, order=1, tag="b")]
    parts = [pi.load_beam(3, w["n"], w["ppc"], w["gamma"], 1e-3, 30 + i) for i, w in enumerate(wls)]
    _say("case 3d batched rows %s" % [w["n"] for w in wls])
    sim = _sim(wls, parts, precision="fp64")
    sim.step(8)
    for i, (w, (x, u)) in enumerate(zip(wls, parts)):
        ref = OracleSim(w, x, u)
        ref.step(8)
        errs = {k: _rel(sim.fields(k, i), getattr(ref, k)) for k in ("E", "B", "J")}
        _say("  instance %d %s" % (i, errs))
        assert max(errs.values()) < 1e-10
    sim.close()
    res = []
    for sched in ("batched", "plain"):
        sim = _sim(wls, parts, precision="fp32")
        sim.set_schedule(sched, True)
        sim.step(6)
        res.append([sim.fields("E", i) for i in range(2)] + [sim.fields("Et", i) for i in range(2)])
        sim.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n,order", [((16, 12, 24), 1), ((16, 12, 24), 3), ((64, 8, 8), 3)])
def test_3d_fp64_parity_50_steps(n, order):
    """The FP64 bar over 50 steps in 3D (relative L2 of E, B, J at most 1e-10),
    linear and cubic shapes, with rows of 16 cells (per-tap x pass) and of 64
    (staged x pass); the Gauss residual stays at rounding level."""
    wl = pi.workload("beam3d_128x128x256", n=n, ppc=2, order=order)
    sim, ref = _pair(wl, 50, "fp64")
    errs = _field_errors(sim, ref)
    d = sim.diag()
    _say("3d fp64 50 steps n=%s order %d %s gauss %.3e" % (n, order, errs, d["gauss_linf"] / d["rho_max"]))
    assert max(errs.values()) < 1e-10
    assert d["gauss_linf"] < 1e-11 * d["rho_max"]
    sim.close()


def test_3d_cubic_multipass_tiles_parity():
    """The 3D cubic workload's particle density (8 ppc) on a 32x32x64 grid: a
    cubic tile is 8x2x4 = 64 cells, so every tile holds about 512 particles and
    its loop runs two passes of 256 threads.  FP64 within 1e-10 and FP32 within
    1e-4 of the oracle after 10 steps, one oracle run for both."""
    wl = pi.workload("beam3d_128x128x256", n=(32, 32, 64), ppc=8, order=3)
    x, u = pi.load_beam(3, wl["n"], wl["ppc"], wl["gamma"], 1e-3, 0)
    _say("case 3d cubic multipass n=%s np=%d" % (wl["n"], x.shape[0]))
    ref = OracleSim(wl, x, u)
    ref.step(10)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        sim = _sim(wl, (x, u), precision=prec)
        sim.step(10)
        errs = _field_errors(sim, ref)
        d = sim.diag()
        _say("3d cubic multipass %s %s slow=%d" % (prec, errs, d["slow_tiles"]))
        assert max(errs.values()) < tol
        assert d["gauss_linf"] < (1e-11 if prec == "fp64" else 1e-5) * d["rho_max"]
        sim.close()


@pytest.mark.parametrize("order", [1, 3])
def test_3d_dense_tiles_keep_32bit_lds_sums_in_range(order):
    """3D float sums a tile's current in 32-bit words whose quantum grows with the
    tile's particle count (kq, from a bound on one particle's contribution), so
    that all of a tile's particles adding to one cell stay below 2^30.  A dense
    clump — 96 particles in each of the 64 cells of one tile, 6144 in the tile,
    kq = 9 (cubic) and 11 (linear) — must still match the oracle to the FP32
    bound, with the Gauss residual at rounding level and no range flag."""
    from paper_1401_0838_amd import _lib as L
    n = (16, 8, 16)
    wl = pi.workload("beam3d_128x128x256", n=n, ppc=96, order=order)
    tile = [i + n[0] * (j + n[1] * k) for i in range(8, 16) for j in range(2, 4) for k in range(4, 8)]
    x, u = pi.load_beam(3, n, 96, wl["gamma"], 1e-3, 9, cells=np.array(tile))
    _say("case 3d dense tile order %d np=%d" % (order, x.shape[0]))
    ref = OracleSim(wl, x, u)
    ref.step(6)
    sim = _sim(wl, (x, u), precision="fp32")
    sim.step(6)
    errs = _field_errors(sim, ref)
    d = sim.diag()
    _say("  %s gauss %.3e rho_max %.3e slow=%d" % (errs, d["gauss_linf"], d["rho_max"], d["slow_tiles"]))
    assert d["rc"] == L.PIC_OK and d["current_range"] == 0
    assert max(errs.values()) < 1e-4
    assert d["gauss_linf"] < 1e-5 * d["rho_max"]
    sim.close()


@pytest.mark.parametrize("dims,order,sigma", [(2, 1, 0.05), (2, 3, 0.05), (3, 1, 0.05), (3, 3, 0.05),
                                               (2, 1, 3.0)])
def test_charge_density_and_diagnostics_match_oracle(dims, order, sigma):
    """rho on the nodes (tiled LDS deposit), kinetic energy, charge and the Gauss
    residual after a few steps; sigma 3 makes a hot beam whose tiles outgrow their
    windows (global fallback path)."""
    base = "beam2d_64_fp64" if dims == 2 else "beam3d_128x128x256"
    n = (48, 40) if dims == 2 else (12, 10, 16)
    wl = pi.workload(base, n=n, order=order, ppc=3, gamma=3.0)
    sim, ref = _pair(wl, 6, "fp64", sigma=sigma)
    r = sim.field("rho", 0)
    rr = ref.rho()
    _say("rho dims %d order %d sigma %g: rel %.3e" % (dims, order, sigma, _rel(r, rr)))
    assert _rel(r, rr) < 1e-12
    d, od = sim.diag(), ref.diag()
    assert abs(d["Wkin"] - od["Wkin"]) < 1e-11 * od["Wkin"]
    assert abs(d["charge"] - od["charge"]) < 1e-11 * abs(od["charge"])
    assert abs(d["gauss_linf"] - od["gauss_linf"]) < 1e-9 * d["rho_max"]
    sim.close()


# ----------------------------------------------------------- edge cases

def test_ragged_grid_and_tiny_grid():
    # (100, 70) and (130, 21): several 64-column field tiles with a ragged last one
    for n in [(50, 37), (8, 8), (5, 70), (100, 70), (130, 21)]:
        wl = pi.workload("beam2d_64_fp64", n=n, correction=True, filter=pi.workloads.BINOMIAL4)
        sim, ref = _pair(wl, 25, "fp64", sigma=1e-2)
        errs = _field_errors(sim, ref)
        _say("grid %s %s" % (n, errs))
        assert max(errs.values()) < 1e-10
        sim.close()


def test_nonfinite_field_is_reported():
    """A NaN written into one E value is reported by pic_diag as PIC_ENONFINITE with
    the non-finite flag set (fields are checked without stepping, so the NaN never
    reaches a particle); once the value is finite again the diagnostics are clean."""
    from paper_1401_0838_amd import _lib as L
    wl = pi.workload("beam2d_64_fp64", n=(24, 20), correction=True, filter=pi.workloads.BINOMIAL4)
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], 1e-3, 2)
    for prec in ("fp64", "fp32"):
        _say("case nonfinite %s" % prec)
        sim = _sim(wl, (x, u), precision=prec)
        sim.step(3)
        d = sim.diag()
        assert d["rc"] == L.PIC_OK and d["nonfinite"] == 0
        ex = sim.field("E", 0)
        bad = ex.copy()
        bad[7, 0, 5] = np.nan
        sim.set_field("E", 0, bad)
        d = sim.diag()
        assert d["rc"] == L.PIC_ENONFINITE and d["nonfinite"] == 1
        with pytest.raises(L.PicError) as e:
            sim.diag(check=True)
        assert e.value.code == L.PIC_ENONFINITE
        sim.set_field("E", 0, ex)
        d = sim.diag()
        assert d["rc"] == L.PIC_OK and d["nonfinite"] == 0
        sim.close()


def test_current_range_is_flagged():
    """Float mode keeps the current in HBM as 32-bit fixed point with a quantum
    2^shift times the LDS one, chosen at init from the densest cell (a word holds
    about 2^10 times the current a beam at c carries through it).  A cold
    gamma = 130 clump of 2000 macro-particles in one cell stays in range with the
    chosen quantum; forcing the finest quantum (shift 0) from the host makes the
    same sums leave the 32-bit range, and pic_diag must return PIC_ERANGE with
    current_range set.  FP64 (double current) never flags."""
    from paper_1401_0838_amd import _lib as L
    wl = pi.workload("beam2d_64_fp64", n=(16, 16), correction=True, filter=pi.workloads.BINOMIAL4)
    x, u = pi.load_beam(2, (16, 16), 2000, 130.0, 1e-6, 3, cells=np.array([5 + 16 * 7]))
    for shift, prec, expect in ((None, "fp32", L.PIC_OK), (0, "fp32", L.PIC_ERANGE), (None, "fp64", L.PIC_OK)):
        _say("case current range shift=%s %s" % (shift, prec))
        sim = _sim(dict(wl, ppc=2000), (x, u), precision=prec)
        if shift is not None:
            sim.set_option("current_quantum_shift", shift)
        elif prec == "fp32":
            _say("  chosen shift %d" % sim.get_option("current_quantum_shift"))
        sim.step(2)
        d = sim.diag()
        _say("  rc %d current_range %d" % (d["rc"], d["current_range"]))
        assert d["rc"] == expect
        assert d["current_range"] == (1 if expect == L.PIC_ERANGE else 0)
        sim.close()


def test_empty_and_clumped_beams():
    wl = pi.workload("beam2d_64_fp64", n=(32, 32), correction=True, filter=pi.workloads.BINOMIAL4)
    # empty: fields stay zero
    sim = _sim(wl, (np.zeros((0, 2)), np.zeros((0, 3))), precision="fp64")
    sim.step(5)
    assert np.all(sim.fields("E") == 0)
    sim.close()
    # clumped: all particles in a 3x3 block of cells, hot enough to spread across tiles
    cells = np.array([i + 32 * k for i in range(10, 13) for k in range(10, 13)])
    x, u = pi.load_beam(2, (32, 32), 64, 1.5, 0.8, 4, cells=cells)
    sim, ref = _pair(wl, 40, "fp64", x=x, u=u)
    errs = _field_errors(sim, ref)
    d = sim.diag()
    _say("clumped %s resorts=%d slow=%d" % (errs, d["resorts"], d["slow_tiles"]))
    assert max(errs.values()) < 1e-10
    assert d["resorts"] >= 1           # the clump outgrew its tiles' windows and was re-sorted
    sim.close()


_DEFER_BASE = [(2, 1, "fp64", "galerkin"), (2, 1, "fp32", "galerkin"), (2, 3, "fp64", "galerkin"),
               (2, 1, "fp64", "uniform"), (2, 1, "fp64", "momentum"), (3, 1, "fp64", "galerkin"),
               (3, 3, "fp32", "galerkin")]


# 3D has only the deferring form, so it is listed with defer = 1 alone
@pytest.mark.parametrize("dims,order,prec,interp,defer",
                         [b + (d,) for b in _DEFER_BASE for d in ((0, 1) if b[0] == 2 else (1,))])
def test_deferred_tiles_match_oracle(dims, order, prec, interp, defer):
    """A hot beam with re-sorting held off: tile boxes outgrow their LDS windows
    and are stepped in global memory, inside the particle kernel (defer 0) or by
    the second launch (defer 1; 3D always), and the step still matches the
    oracle."""
    if dims == 2:
        wl = pi.workload("beam2d_64_fp64", n=(40, 48), ppc=4, order=order, correction=True,
                         filter=pi.workloads.BINOMIAL4, interp=interp)
    else:
        wl = pi.workload("beam3d_128x128x256", n=(16, 12, 24), ppc=2, order=order)
    nsteps = 24
    x, u = pi.load_beam(dims, wl["n"], wl["ppc"], 1.5, 0.8, 5)
    _say("deferred case dims=%d order=%d %s %s defer=%d steps=%d" % (dims, order, prec, interp, defer, nsteps))
    sim = _sim(wl, (x, u), precision=prec)
    sim.set_option("resort_every", 1024)
    sim.set_option("particle_defer", defer)
    ref = OracleSim(wl, x, u)
    sim.step(nsteps)
    ref.step(nsteps)
    errs = _field_errors(sim, ref)
    d = sim.diag()
    _say("deferred %s slow=%d resorts=%d" % (errs, d["slow_tiles"], d["resorts"]))
    assert d["slow_tiles"] >= 1        # the deferred pass did run
    assert max(errs.values()) < (1e-10 if prec == "fp64" else 1e-4)
    sim.close()


def test_resort_in_a_batch_keeps_parity():
    """Two instances, one hot (re-sorted every 4 steps) and one cold, stepped as a
    batch in FP32 and FP64: each matches its own oracle and only the hot one is
    re-sorted."""
    wl_hot = pi.workload("beam2d_64_fp64", n=(48, 32), correction=True, filter=pi.workloads.BINOMIAL4, tag="hot")
    wl_cold = pi.workload("beam2d_64_fp64", n=(32, 48), correction=True, filter=pi.workloads.BINOMIAL4,
                          alpha=0.4, tag="cold")
    hot = pi.load_beam(2, wl_hot["n"], 4, 1.5, 0.9, 21)
    cold = pi.load_beam(2, wl_cold["n"], 4, 130.0, 1e-6, 22)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        sim = _sim([wl_hot, wl_cold], [hot, cold], precision=prec)
        sim.set_option("resort_every", 4)
        sim.step(30)
        for i, (w, (x, u)) in enumerate(((wl_hot, hot), (wl_cold, cold))):
            ref = OracleSim(w, x, u)
            ref.step(30)
            e = max(_rel(sim.fields(k, i), getattr(ref, k)) for k in ("E", "B", "J"))
            d = sim.diag(i)
            _say("batch resort %s inst %d: err %.3e resorts %d slow %d" % (prec, i, e, d["resorts"], d["slow_tiles"]))
            assert e < tol
            if i == 0:
                assert d["resorts"] >= 1
            else:
                assert d["resorts"] == 0
        sim.close()


def test_strong_instability_growth_fp64():
    """No correction, no filter, 200 steps (the plain 64x64 case): fields grow by many
    orders of magnitude and GPU and oracle still agree."""
    wl = pi.workload("beam2d_64_fp64")
    sim, ref = _pair(wl, 200, "fp64")
    errs = _field_errors(sim, ref)
    _say("plain 200 steps %s Wperp=%g" % (errs, ref.energies()["Wperp"]))
    assert errs["E"] < 1e-8 and errs["B"] < 1e-8
    sim.close()


# ------------------------------------------------------ determinism / modes

def test_fp32_bitwise_deterministic_and_graph_equals_eager():
    """Graph replay (pieces: 5 steps, then 18 from step 5 = head of 11 with the
    re-sort check at step 16 and a tail of 7, prepared ahead or captured on use)
    and eager stepping give bitwise the same FP32 fields."""
    wl = pi.workload("beam2d_64_fp64", n=(64, 64), correction=True, filter=pi.workloads.BINOMIAL4)
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], 1e-3, 9)
    out = []
    for graph, prep in ((True, False), (True, True), (False, False)):
        sim = _sim(wl, (x, u), precision="fp32")
        sim.set_schedule("batched", graph)
        sim.step(5)
        if prep:
            sim.prepare(18)
        sim.step(18)
        out.append((sim.fields("E"), sim.fields("B"), sim.fields("J")))
        sim.close()
    for k in range(3):
        assert np.array_equal(out[0][k], out[1][k])
        assert np.array_equal(out[0][k], out[2][k])


def test_batched_instances_match_own_oracle_and_plain():
    wls = [pi.workload("beam2d_512", n=(64, 32), alpha=0.35, ppc=4, precision="fp64", tag="a"),
           pi.workload("beam2d_512", n=(32, 96), alpha=0.55, ppc=4, gamma=10.0, precision="fp64", tag="b"),
           pi.workload("beam2d_512", n=(48, 48), alpha=0.45, ppc=2, gamma=50.0, precision="fp64", tag="c")]
    parts = [pi.load_beam(2, w["n"], w["ppc"], w["gamma"], 1e-4, 20 + i) for i, w in enumerate(wls)]
    sim = _sim(wls, parts, precision="fp64")
    sim.step(20)
    for i, (w, (x, u)) in enumerate(zip(wls, parts)):
        ref = OracleSim(w, x, u)
        ref.step(20)
        assert _rel(sim.fields("E", i), ref.E) < 1e-10
        assert _rel(sim.fields("B", i), ref.B) < 1e-10
    sim.close()
    # plain (one launch per instance) equals batched bitwise in fp32
    res = []
    for sched in ("batched", "plain"):
        sim = _sim(wls, parts, precision="fp32")
        sim.set_schedule(sched, True)
        sim.step(12)
        res.append([sim.fields("E", i) for i in range(3)])
        sim.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_many_batched_instances_fp64_match_oracle():
    """32 instances of 512x512 in one batched launch: far more field tiles than
    the chip holds at once, so tiles run in waves.  Every instance must still
    equal the oracle (a field kernel that read a neighbour's already-updated
    halo would make the instances differ)."""
    wl = pi.workload("beam2d_512", ppc=1, precision="fp64")
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], 1e-3, 5)
    rng = np.random.default_rng(5)
    E0 = rng.normal(size=(3, 512, 1, 512)) * 1e-3
    B0 = rng.normal(size=(3, 512, 1, 512)) * 1e-3
    ninst = 32
    _say("case 32 x 512x512 fp64 batched, 3 steps")
    sim = _sim([wl] * ninst, [(x, u)] * ninst, precision="fp64")
    for i in range(ninst):
        for c in range(3):
            sim.set_field("E", c, E0[c], i)
            sim.set_field("B", c, B0[c], i)
    ref = OracleSim(wl, x, u)
    ref.E[:] = E0
    ref.B[:] = B0
    sim.step(3)
    ref.step(3)
    worst = 0.0
    for i in range(ninst):
        for k in ("E", "B", "J"):
            worst = max(worst, _rel(sim.fields(k, i), getattr(ref, k)))
    _say("  worst relative error over instances %.3e" % worst)
    sim.close()
    assert worst < 1e-10


# ------------------------------------------------------ full-size sample

def test_full_size_512_fp32_parity_10_steps():
    """The 512x512, 16 ppc workload in the launch configuration the benchmark
    times (FP32, batched, graph), against the oracle after 10 steps."""
    wl = pi.workload("beam2d_512")
    sim, ref = _pair(wl, 10, "fp32")
    errs = _field_errors(sim, ref)
    _say("512 fp32 %s" % errs)
    assert errs["E"] < 1e-4 and errs["B"] < 1e-4 and errs["J"] < 1e-4
    d = sim.diag()
    assert d["gauss_linf"] < 1e-5 * d["rho_max"]
    sim.close()


@pytest.mark.parametrize("n,interp", [((96, 80), "galerkin"), ((64, 160), "momentum"), ((200, 264), "galerkin"),
                                      ((128, 96), "galerkin"), ((64, 48), "momentum")])
def test_streamed_seen_fields_equal_the_tiled_ones(n, interp):
    """The streamed seen-field pass (128-column strips, 128-row segments, 32-row
    chunks, a ring of x-filtered rows) computes the same sums in the same order
    as the tiled pass: bitwise equal seen fields, also on segments of one to
    four chunks (nz = 264, 48, 80, 128 rows), with a ragged last chunk (nz = 80,
    264), a ragged strip (nx = 96, 200), the wider stencil of the
    momentum-conserving gather, and widths that are a multiple of 64 (nx = 64,
    128), where the strips start past the 64-cell boundary and the last one
    wraps (for nx = 64 half of that strip repeats columns stored elsewhere and
    is not stored)."""
    wl = pi.workload("beam2d_512", n=n, ppc=2, interp=interp)
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], 1e-3, 5)
    out = []
    for tz in (None, 128):
        sim = _sim(wl, (x, u), precision="fp32")
        if tz:
            sim.set_option("seen_tile_z", tz)
            assert sim.get_option("seen_tile_z") == tz
        sim.step(3)
        out.append((sim.fields("Et"), sim.fields("Bt"), sim.fields("E")))
        sim.close()
    _say("streamed seen %s %s: max |diff| %g" % (n, interp, max(float(np.max(np.abs(a - b)))
                                                                  for a, b in zip(*out))))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_tuning_knobs_leave_fp32_results_bitwise_unchanged():
    """Workgroup size, field tile heights, the particle-kernel variants and the
    inline or deferred form change only the schedule: every FP32 result is
    bitwise the same (integer current sums).  The particle tile shape and the
    re-sort period change which particles share a tile, and each tile's current
    sum is rounded once to the HBM quantum (about 2^-21 of the densest cell's beam
    current), so those agree to that rounding: relative L2 below 1e-5 after 21
    steps.  Also runs the autotuner on a short candidate list."""
    from paper_1401_0838_amd import tune
    wl = pi.workload("beam2d_512", n=(128, 96), ppc=4)
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], 1e-3, 11)
    runs = [(dict(), True), (dict(block=512), True),
            (dict(opts={"yee_tile_z": 4, "seen_tile_z": 32}), True), (dict(opts={"seen_tile_z": 128}), True),
            (dict(opts={"particle_waves4": 1}), True), (dict(opts={"particle_prefetch": 1}), True),
            (dict(opts={"particle_waves4": 1, "particle_prefetch": 1}), True),
            (dict(opts={"particle_defer": 1}), True), (dict(opts={"particle_defer": 0}), True),
            (dict(tile=(8, 1, 8)), False), (dict(tile=(32, 1, 16), block=512), False),
            (dict(opts={"resort_every": 5}), False)]
    ref = None
    for r, bitwise in runs:
        sim = _sim(wl, (x, u), precision="fp32", tile=r.get("tile"), block=r.get("block", 0))
        for k, v in r.get("opts", {}).items():
            sim.set_option(k, v)
        sim.step(21)
        got = (sim.fields("E"), sim.fields("B"), sim.fields("J"))
        sim.close()
        if ref is None:
            ref = got
        elif bitwise:
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), r
        else:
            for a, b in zip(ref, got):
                assert _rel(b, a) < 1e-5, (r, _rel(b, a))
    best = tune.tune(wl, (x, u), precision="fp32", steps=3, warmup=1, cache=None,
                     candidates=[((16, 1, 16), 256), ((8, 1, 8), 256)],
                     options=[{}, {"seen_tile_z": 32}, {"particle_defer": 1}])
    _say("tuner picked %s" % best)
    assert best["tile"] in ([16, 1, 16], [8, 1, 8]) and best["step_ms"] > 0
    assert best["options"] in ({}, {"seen_tile_z": 32}, {"particle_defer": 1})
