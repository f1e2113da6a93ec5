"""pic_init_static (arena in the library's static device array) against pic_init
(arena allocated by the caller): the same instances stepped the same way give
the same fields, currents, particles and diagnostics.  FP32 steps are bitwise
reproducible for a given tiling (integer current sums), so E, B, J and the
particles must match exactly; the float64 diagnostics reductions use atomics and
are compared to 1e-12.  Two calls in a row, the second with a smaller input."""
import sys

import numpy as np
import pytest

import pic_inputs as pi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(wl, seed, nsteps):
    from paper_1401_0838_amd.sim import Simulation
    x, u = pi.load_beam(2, wl["n"], wl["ppc"], wl["gamma"], wl["sigma"], seed)
    ref = Simulation(wl, (x, u), precision="fp32", trace_capacity=nsteps)
    sta = Simulation(wl, (x, u), precision="fp32", trace_capacity=nsteps, static_arena=True)
    assert sta.arena is None
    for sim in (ref, sta):
        sim.step(nsteps)
    try:
        for which in ("E", "B", "J", "Et", "Bt"):
            a, b = ref.fields(which), sta.fields(which)
            assert np.array_equal(a, b), which
        xa, ua = ref.particles()
        xb, ub = sta.particles()
        assert np.array_equal(xa, xb) and np.array_equal(ua, ub)
        da, db = ref.diag(check=True), sta.diag(check=True)
        for k in ("WE", "WB"):
            assert np.allclose(da[k], db[k], rtol=1e-12, atol=0), k
        for k in ("Wkin", "charge"):
            assert abs(da[k] - db[k]) <= 1e-12 * abs(da[k]), k
        assert da["step"] == db["step"] == nsteps
        ta, tb = ref.trace(), sta.trace()
        assert ta.shape == tb.shape and np.allclose(ta, tb, rtol=1e-12, atol=0)
    finally:
        ref.close()
        sta.close()


def test_static_arena_matches_allocated_arena_twice():
    # 128 x 128, 8 ppc (10 MiB of arena), then 64 x 64, 4 ppc: the second call
    # reuses the array the first one left behind
    cases = [(pi.workload("beam2d_512", n=(128, 128), ppc=8, alpha=0.5), 3, 40),
             (pi.workload("beam2d_512", n=(64, 64), ppc=4, alpha=0.7), 4, 24)]
    for wl, seed, n in cases:
        _say("case static arena %s ppc %d alpha %.1f seed %d steps %d" % (wl["n"], wl["ppc"], wl["alpha"], seed, n))
        _pair(wl, seed, n)


def test_static_arena_limits():
    from paper_1401_0838_amd import _lib as L
    from paper_1401_0838_amd.sim import Simulation
    small = pi.workload("beam2d_512", n=(64, 64), ppc=4, alpha=0.5)
    x, u = pi.load_beam(2, small["n"], small["ppc"], small["gamma"], small["sigma"], 0)
    _say("case static arena one live state per device")
    a = Simulation(small, (x, u), precision="fp32", static_arena=True)
    try:
        with pytest.raises(L.PicError) as e:
            Simulation(small, (x, u), precision="fp32", static_arena=True)
        assert e.value.code == L.PIC_ESTATE
    finally:
        a.close()
    b = Simulation(small, (x, u), precision="fp32", static_arena=True)   # released by close
    b.step(2)
    b.close()
    _say("case static arena oversize")
    big = pi.workload("beam2d_512", n=(512, 512), ppc=16, alpha=0.5)
    xb, ub = pi.load_beam(2, big["n"], big["ppc"], big["gamma"], big["sigma"], 0)
    with pytest.raises(L.PicError) as e:
        Simulation(big, (xb, ub), precision="fp32", static_arena=True)
    assert e.value.code == L.PIC_ENOMEM and "static arena" in str(e.value)
