"""C-ABI library: loads, exports every declared entry point, and its host-only
logic (coefficient setup, configuration checks) behaves.  CPU only."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

import pic_inputs as pi
from paper_1401_0838_amd import _lib as L
from paper_1401_0838_amd.sim import make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic_api.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(L.LIB_PATH)
    names = _declared()
    assert "pic_step" in names and "pic_init" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTED) == names


def test_strerror_codes():
    for code in range(0, -11, -1):
        assert L.strerror(code) and L.strerror(code) != "unknown error"


@pytest.mark.parametrize("case", json.load(open(os.path.join(ROOT, "tests", "golden", "psi_coeffs.json")))["cases"])
def test_psi_setup_matches_oracle_golden(case):
    """The library's 113-bit setup reproduces the oracle's 50-digit coefficients
    (stored by tests/golden/make_psi_golden.py) to float64 rounding."""
    interp = {"galerkin": L.PIC_GALERKIN, "uniform": L.PIC_UNIFORM, "momentum": L.PIC_MOMENTUM}[case["interp"]]
    rc, a, b = L.pic_psi_coeffs(interp, case["alpha"], 4)
    ea = np.array([float(v) for v in case["psi_e"]])
    eb = np.array([float(v) for v in case["psi_b"]])
    if case["positive"]:
        assert rc == L.PIC_OK
    else:
        assert rc == L.PIC_EPSI
    assert np.max(np.abs(a - ea) / np.maximum(np.abs(ea), 1e-300)) <= 4e-16
    assert np.max(np.abs(b - eb) / np.maximum(np.abs(eb), 1e-300)) <= 4e-16


def test_psi_setup_rejects_breakdown():
    """Sec. 3 notes a narrow alpha window where the determination breaks down; for the
    Galerkin multiplier Psi_B turns negative near alpha = 0.69 (reading used here)."""
    rc, a, b = L.pic_psi_coeffs(L.PIC_GALERKIN, 0.69, 4)
    assert rc == L.PIC_EPSI
    rc, _, _ = L.pic_psi_coeffs(L.PIC_GALERKIN, 1.2, 4)
    assert rc == L.PIC_EINVAL


def _cfg(**kw):
    wl = pi.workload("beam2d_64_fp64", n=(16, 16))
    wl.update(kw)
    return make_config(wl)


def test_plan_validates_configs():
    assert L.pic_plan([_cfg()], [1024]) > 0
    with pytest.raises(L.PicError) as e:
        L.pic_plan([_cfg(alpha=0.71)], [1024])      # 2D Yee limit 1/sqrt(2)
    assert e.value.code == L.PIC_ECOURANT
    c = _cfg(correction=True)
    c.psi_b[4] = -5.0
    with pytest.raises(L.PicError) as e:
        L.pic_plan([c], [16])
    assert e.value.code == L.PIC_EPSI
    c = _cfg()
    c.shape_order = 2
    with pytest.raises(L.PicError) as e:
        L.pic_plan([c], [16])
    assert e.value.code == L.PIC_EINVAL
    assert L.pic_plan([_cfg(interp="uniform")], [16]) > 0
    assert L.pic_plan([_cfg(interp="momentum", correction=True)], [16]) > 0
    c = _cfg(interp="uniform")
    c.interp = 7
    with pytest.raises(L.PicError) as e:
        L.pic_plan([c], [16])
    assert e.value.code == L.PIC_EINVAL
    with pytest.raises(L.PicError) as e:     # schemes are shared by a batch
        L.pic_plan([_cfg(), _cfg(interp="uniform")], [16, 16])
    assert e.value.code == L.PIC_EINVAL
    c = _cfg(interp="momentum")
    c.filter_npass = 8                        # node average needs one more x cell
    with pytest.raises(L.PicError) as e:
        L.pic_plan([c], [16])
    assert e.value.code == L.PIC_EINVAL
    c = _cfg(interp="momentum")
    c.adjoint_steps, c.adjoint_ckpt = 4, 2
    with pytest.raises(L.PicError) as e:
        L.pic_plan([c], [16])
    assert e.value.code == L.PIC_EUNSUPPORTED
    c = _cfg(interp="uniform")
    c.adjoint_steps, c.adjoint_ckpt = 4, 2
    assert L.pic_plan([c], [16]) > 0
    # exact ratio: nz <= 1024, shared by a batch, forward only
    assert L.pic_plan([_cfg(correction="ratio")], [16]) > 0
    with pytest.raises(L.PicError) as e:
        L.pic_plan([_cfg(correction="ratio", n=(16, 2048))], [16])
    assert e.value.code == L.PIC_EUNSUPPORTED
    with pytest.raises(L.PicError) as e:
        L.pic_plan([_cfg(correction=True), _cfg(correction="ratio")], [16, 16])
    assert e.value.code == L.PIC_EINVAL
    c = _cfg(correction="ratio")
    c.adjoint_steps, c.adjoint_ckpt = 4, 2
    with pytest.raises(L.PicError) as e:
        L.pic_plan([c], [16])
    assert e.value.code == L.PIC_EUNSUPPORTED
    # Cole-Karkkainen: 2D square cells, c dt < dx, shared by a batch, forward only
    assert L.pic_plan([_cfg(solver="ck", alpha=0.95)], [16]) > 0
    with pytest.raises(L.PicError) as e:
        L.pic_plan([_cfg(solver="ck", alpha=1.0)], [16])
    assert e.value.code == L.PIC_ECOURANT
    with pytest.raises(L.PicError) as e:
        L.pic_plan([_cfg(solver="ck", d=(1.0, 0.8))], [16])
    assert e.value.code == L.PIC_EUNSUPPORTED
    with pytest.raises(L.PicError) as e:
        L.pic_plan([_cfg(solver="ck", dims=3, n=(8, 8, 8))], [16])
    assert e.value.code == L.PIC_EUNSUPPORTED
    with pytest.raises(L.PicError) as e:
        L.pic_plan([_cfg(), _cfg(solver="ck")], [16, 16])
    assert e.value.code == L.PIC_EINVAL
    c = _cfg(solver="ck")
    c.adjoint_steps, c.adjoint_ckpt = 4, 2
    assert L.pic_plan([c], [16]) > 0
    with pytest.raises(L.PicError):
        L.pic_plan([_cfg(), _cfg(dims=3, n=(8, 8, 8))], [16, 16])


def test_plan_rejects_particle_counts_beyond_32bit_offsets():
    """Particle arrays are addressed with 32-bit byte offsets: at most 2^30 - 1
    particles per instance in FP32 (4-byte elements) and 2^29 - 1 in FP64."""
    c32 = _cfg(precision="fp32")
    assert L.pic_plan([c32], [(1 << 30) - 1]) > 0
    with pytest.raises(L.PicError):
        L.pic_plan([c32], [1 << 30])
    c64 = _cfg(precision="fp64")
    with pytest.raises(L.PicError):
        L.pic_plan([c64], [1 << 29])
    with pytest.raises(L.PicError):
        L.pic_plan([c32], [-1])


def test_plan_grows_with_batch():
    one = L.pic_plan([_cfg()], [1024])
    two = L.pic_plan([_cfg(), _cfg(n=(32, 16))], [1024, 2048])
    assert two > one


def test_default_tiles_shrink_only_for_small_batches():
    """2D tiles default to 16 x 16 cells, or 8 x 8 when the whole batch has fewer
    than 1024 of the 16 x 16 tiles; the arena that pic_plan sizes shows which."""
    def plan(n, tile=None, count=1):
        wl = pi.workload("beam2d_64_fp64", n=n)
        cfgs = [make_config(wl, tile=tile) for _ in range(count)]
        return L.pic_plan(cfgs, [n[0] * n[1] * 4] * count)
    assert plan((256, 256)) == plan((256, 256), tile=(8, 1, 8))
    assert plan((256, 256)) != plan((256, 256), tile=(16, 1, 16))
    assert plan((512, 512)) == plan((512, 512), tile=(16, 1, 16))
    assert plan((256, 256), count=4) == plan((256, 256), tile=(16, 1, 16), count=4)
    assert plan((256, 256), count=3) == plan((256, 256), tile=(8, 1, 8), count=3)


def test_scan_growth_table_on_synthetic_traces():
    """Peak over alpha per gamma and the fitted power of gamma, on traces that
    grow as exp(2 Gamma t) with Gamma = 0.01 gamma^-0.5 at the best alpha."""
    from paper_1401_0838_amd import scan
    pts, traces, wkin = [], [], []
    for g in (3.0, 10.0, 30.0, 130.0):
        for a, f in ((0.5, 0.6), (0.7, 1.0), (0.9, 0.8)):
            gam = 0.01 * g ** -0.5 * f
            t = np.arange(3000) * a
            pts.append((g, a))
            traces.append(1e-6 * np.exp(2 * gam * t))
            wkin.append(1e30)
    rates, peaks, power = scan.growth_table(pts, traces, wkin)
    for (g, a), r in zip(pts, rates):
        f = {0.5: 0.6, 0.7: 1.0, 0.9: 0.8}[a]
        assert abs(r - 0.01 * g ** -0.5 * f) < 1e-9
    assert all(peaks[g][1] == 0.7 for g in peaks)
    assert abs(power + 0.5) < 1e-9


def test_variant_configs_plan():
    """Every Sec. 3 variant of the CK cubic Eq. 6 setting is a valid plan, and a
    batch mixing the split variants is accepted (the exact ratio goes alone)."""
    from paper_1401_0838_amd import scan
    base = pi.workload("beam2d_128_ck", n=(32, 32))
    cfgs = {k: make_config(dict(base, **v)) for k, v in scan.VARIANTS.items()}
    for k, c in cfgs.items():
        assert L.pic_plan([c], [64]) > 0, k
    split = [c for k, c in cfgs.items() if k != "ratio_on_transverse_E"]
    assert L.pic_plan(split, [64] * len(split)) > 0
