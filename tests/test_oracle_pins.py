"""Pins of the FP64 oracle against what the paper and the mathematics fix.

CPU only.  Each test names the passage or the closed form it relies on.
"""
import json
import math
import os

import numpy as np
import pytest

import pic_inputs as pi
from oracle import fit as ofit
from oracle import psi
from oracle.brute import BruteSim
from oracle.ref import OracleSim

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FACTS = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))

CASES = [("galerkin", 0.3), ("galerkin", 0.5), ("galerkin", 0.7),
         ("uniform", 0.3), ("uniform", 0.7), ("uniform", 0.9),
         ("momentum", 0.3), ("momentum", 0.5), ("momentum", 0.7)]


def _wl(**kw):
    wl = pi.workload("beam2d_64_fp64")
    wl.update(kw)
    return wl


def _empty_sim(wl):
    dims = wl["dims"]
    return OracleSim(wl, np.zeros((0, dims)), np.zeros((0, 3)))


# ------------------------------------------------------ Psi (Sec. 2, Eqs. 3-5)

@pytest.mark.parametrize("interp,alpha", CASES)
def test_psi_interpolates_at_nine_uniform_nodes(interp, alpha):
    """Sec. 2: nine nodes uniform in s on [0, 1]; the ratio equals M there."""
    a, b, ident = psi.psi_coeffs(interp, alpha)
    assert not ident
    assert len(a) == FACTS["psi_degree"]["value"] + 1
    nn = FACTS["psi_nodes"]["value"]
    for j in range(nn):
        s = j / (nn - 1)
        M = float(psi.multiplier(interp, alpha, s))
        pe, pb = psi.poly(a, s), psi.poly(b, s)
        assert abs(pe - M * pb) <= 1e-13 * max(1.0, abs(pb)), (j, pe, M * pb)


@pytest.mark.parametrize("interp,alpha", CASES)
def test_psi_ratio_accuracy_bound(interp, alpha):
    """Sec. 2 (Fig. 1 text): ratio within 1e-6 of M at small k, 1e-5 at the largest k shown.
    Checked for k dz <= pi/2 (1e-6) and k dz <= 2 (1e-5)."""
    a, b, _ = psi.psi_coeffs(interp, alpha)
    tol_small = FACTS["rational_accuracy"]["small_k"]
    tol_large = FACTS["rational_accuracy"]["largest_k"]
    for i in range(1, 201):
        k = 2.0 * i / 200
        s = math.sin(k / 2) ** 2
        err = abs(psi.poly(a, s) / psi.poly(b, s) - float(psi.multiplier(interp, alpha, s)))
        assert err <= (tol_small if k <= math.pi / 2 else tol_large), (k, err)


@pytest.mark.parametrize("interp,alpha", CASES)
def test_psi_small_k_slope_matches_taylor(interp, alpha):
    """Psi_E(0) = Psi_B(0) = 1, so d(Psi_E/Psi_B)/ds at 0 is a1 - b1; it must match the
    Taylor slope of Eqs. 3-5 (independent closed form)."""
    a, b, _ = psi.psi_coeffs(interp, alpha)
    assert a[0] == 1.0 and b[0] == 1.0
    assert abs((a[1] - b[1]) - psi.multiplier_slope0(interp, alpha)) < 2e-6


def test_psi_uniform_magic_step_is_identity():
    """Sec. 1, Sec. 4: the Uniform scheme at alpha = 0.5 is the magic step; Eq. 4 is
    identically 1 there, so the correction reduces to the identity."""
    alpha = FACTS["magic_step_uniform"]["value"]
    for s in np.linspace(0, 1, 17):
        assert abs(float(psi.multiplier("uniform", alpha, s)) - 1.0) < 1e-40
    a, b, ident = psi.psi_coeffs("uniform", alpha)
    assert ident and a == [1.0, 0, 0, 0, 0] and b == [1.0, 0, 0, 0, 0]


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
def test_psi_momentum_vanishes_at_nyquist(alpha):
    """Eq. 5 carries cot(k_z dz / 2), which is exactly zero at k_z dz = pi (s = 1):
    the interpolant, which passes through the node s = 1, has Psi_E(1) = 0 up to
    rounding and Psi_B(1) > 0, and that is not a breakdown of the determination."""
    assert float(psi.multiplier("momentum", alpha, 1)) == pytest.approx(0.0, abs=1e-40)
    a, b, ident = psi.psi_coeffs("momentum", alpha)
    assert not ident
    assert abs(psi.poly(a, 1.0)) < 1e-13 * sum(abs(v) for v in a)
    assert psi.poly(b, 1.0) > 1e-4
    assert psi.psi_positive(a, b)
    bad = list(a)
    bad[0] -= 1e-9      # Psi_E(1) clearly below zero: rejected
    assert not psi.psi_positive(bad, b)


def test_multipliers_in_k_form():
    """Eqs. 3-5 written in k_z (numpy, float64) agree with the s-form used by the solver,
    and Eq. 3 / Eq. 4 = theta / sin(theta) (the Galerkin ratio of spline orders)."""
    alpha, dz = 0.55, 1.0
    dt = alpha * dz
    for k in np.linspace(0.05, math.pi - 0.05, 23):
        th = k * dz / 2
        common = math.sin(k * dt / 2) * math.cos(k * dt / 2) * dz / dt
        mg = common * th / math.sin(th) ** 2
        mu = common / math.sin(th)
        mm = common * math.cos(th) / math.sin(th)
        s = math.sin(th) ** 2
        assert abs(float(psi.multiplier("galerkin", alpha, s)) - mg) < 1e-13
        assert abs(float(psi.multiplier("uniform", alpha, s)) - mu) < 1e-13
        assert abs(float(psi.multiplier("momentum", alpha, s)) - mm) < 1e-13
        assert abs(mg / mu - th / math.sin(th)) < 1e-13


def test_psi_golden_file_matches_solver():
    """tests/golden/psi_coeffs.json was written by make_psi_golden.py from oracle/psi.py."""
    doc = json.load(open(os.path.join(GOLDEN, "psi_coeffs.json")))
    for case in doc["cases"][:4]:
        a, b, ident = psi.psi_coeffs(case["interp"], case["alpha"])
        assert [float(v) for v in case["psi_e"]] == a
        assert [float(v) for v in case["psi_b"]] == b


# ------------------------------------------ seen-field stencils (Sec. 2, 3)

def _impulse_response(which, filt, nz=64, nx=32):
    wl = _wl(n=(nx, nz), correction=True, filter=filt, alpha=0.5)
    sim = _empty_sim(wl)
    delta = np.zeros(sim.shape)
    delta[nz // 2, 0, nx // 2] = 1.0
    return sim, sim.seen_plane(which, delta)[:, 0, :], (nz // 2, nx // 2)


def _dtft(h, centre, kz, kx):
    nz, nx = h.shape
    z = np.arange(nz)[:, None] - centre[0]
    x = np.arange(nx)[None, :] - centre[1]
    return np.sum(h * np.exp(-1j * (kz * z + kx * x)))


@pytest.mark.parametrize("which", [0, 1])
def test_psi_stencil_fourier_response(which):
    """Sec. 2: applying Psi(s) through powers of the (1,-2,1) stencil gives, at any k_z,
    the response Psi(sin^2(k_z dz / 2)) -- evaluated at non-grid wavenumbers."""
    sim, h, c = _impulse_response(which, [])
    coef = sim.psi[which]
    rng = np.random.default_rng(0)
    for kz in rng.uniform(-math.pi, math.pi, 25):
        H = _dtft(h, c, kz, 0.3)
        # no x dependence: the response is independent of kx
        assert abs(H - psi.poly(coef, math.sin(kz / 2) ** 2)) < 1e-14
    assert abs(h.sum() - 1.0) < 1e-14        # Psi(0) = 1
    assert np.count_nonzero(np.abs(h) > 0) == 9  # quartic -> 9 taps in z


@pytest.mark.parametrize("interp,alpha", [("galerkin", 0.5), ("galerkin", 0.7), ("uniform", 0.9),
                                          ("momentum", 0.5)])
def test_psi_ratio_applied_exactly_is_the_multiplier(interp, alpha):
    """Sec. 2: Psi_E applied through the stencil and Psi_B inverted along z give,
    at every wavenumber of the periodic grid, exactly Psi_E(s)/Psi_B(s) (an
    inverse is a circulant, diagonal in the DFT), and that ratio is the
    scheme's multiplier (Eqs. 3-5) to the paper's stated accuracy, taken as in
    the coefficient pin: 1e-6 for k_z dz <= pi/2, 1e-5 up to k_z dz = 2."""
    nz, nx = 64, 8
    wl = _wl(n=(nx, nz), correction="ratio", filter=[], alpha=alpha, interp=interp)
    sim = _empty_sim(wl)
    a, b = sim.psi
    delta = np.zeros(sim.shape)
    delta[0, 0, 3] = 1.0
    h = sim.seen_plane(3, delta)[:, 0, 3]
    assert np.max(np.abs(sim.seen_plane(3, delta)[:, 0, np.arange(nx) != 3])) == 0.0
    H = np.fft.fft(h)
    for m in range(nz):
        kz = 2 * math.pi * m / nz
        s2 = math.sin(kz / 2) ** 2
        ratio = psi.poly(a, s2) / psi.poly(b, s2)
        # rounding: about eps sum|coef| in each applied polynomial, amplified by 1/Psi_B(s)
        tol = 1e-14 * (sum(abs(v) for v in a) + sum(abs(v) for v in b) * abs(ratio)) / psi.poly(b, s2)
        assert abs(H[m] - ratio) < tol, (m, H[m], ratio, tol)
        kk = min(kz, 2 * math.pi - kz)
        if kk <= 2.0:
            M = float(psi.multiplier(interp, alpha, math.sin(kk / 2) ** 2))
            tol_m = FACTS["rational_accuracy"]["small_k" if kk <= math.pi / 2 else "largest_k"]
            assert abs(H[m] - M) < tol_m, (m, H[m], M)


@pytest.mark.parametrize("preset", ["binomial4", "paper-eq6", "paper-eq6-sqrt"])
def test_filter_fourier_response(preset):
    """Sec. 3, Eq. 6: two bilinear plus two compensation passes per axis respond as
    cos^4(5 - 4cos^2)^2 per axis; the 4-pass binomial as cos^8; one pass each as the
    square root of Eq. 6."""
    filt = {"binomial4": pi.workloads.BINOMIAL4, "paper-eq6": pi.workloads.PAPER_EQ6,
            "paper-eq6-sqrt": pi.workloads.PAPER_EQ6_SQRT}[preset]
    sim, h, c = _impulse_response(2, filt)
    rng = np.random.default_rng(1)
    for kz, kx in rng.uniform(-math.pi, math.pi, (20, 2)):
        cz, cx = math.cos(kz / 2) ** 2, math.cos(kx / 2) ** 2
        if preset == "binomial4":
            expect = cz ** 4 * cx ** 4
        elif preset == "paper-eq6":
            expect = cz ** 2 * (5 - 4 * cz) ** 2 * cx ** 2 * (5 - 4 * cx) ** 2
        else:
            expect = cz * (5 - 4 * cz) * cx * (5 - 4 * cx)
        assert abs(_dtft(h, c, kz, kx) - expect) < 1e-13


# ------------------------------------------------------------- Yee (textbook)

@pytest.mark.parametrize("dims,comp", [(2, "Ey"), (2, "By"), (3, "Ey"), (3, "Bz")])
def test_yee_standing_mode_dispersion(dims, comp):
    """Textbook Yee: a single standing mode oscillates as cos(n w dt) with
    sin^2(w dt/2)/dt^2 = sum_d sin^2(k_d d_d/2)/d_d^2 (exact for the split-B leapfrog)."""
    if dims == 2:
        n, d = (24, 32), (1.0, 0.7)
    else:
        n, d = (12, 8, 16), (1.0, 0.9, 0.8)
    wl = _wl(dims=dims, n=n, d=d, alpha=0.45, correction=False, filter=[])
    sim = _empty_sim(wl)
    nz, ny, nx = sim.shape
    dx, dy, dz = (d[0], 1.0, d[1]) if dims == 2 else d
    mx, mz = 2, 3
    kx, kz = 2 * math.pi * mx / (nx * dx), 2 * math.pi * mz / (nz * dz)
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz)[:, None, None]
    if comp == "Ey":       # E_y on integer x, z nodes; y-invariant TE mode
        mode = np.sin(kx * i * dx) * np.sin(kz * k * dz) * np.ones((1, ny, 1))
        sim.E[1][:] = mode
    elif comp == "By":     # B_y at (i+1/2, k+1/2)
        mode = np.cos(kx * (i + 0.5) * dx) * np.cos(kz * (k + 0.5) * dz) * np.ones((1, ny, 1))
        sim.B[1][:] = mode
    else:                  # B_z at (i+1/2, j+1/2, k), varying in x and y: divergence-free
        ky = 2 * math.pi * 1 / (ny * dy)
        j = np.arange(ny)[None, :, None]
        mode = np.cos(kx * (i + 0.5) * dx) * np.cos(ky * (j + 0.5) * dy) * np.ones((nz, 1, 1))
        sim.B[2][:] = mode
        kz, dz = ky, dy    # the second wave-vector component is along y here
    dt = sim.s.dt
    kap2 = (math.sin(kx * dx / 2) / dx) ** 2 + (math.sin(kz * dz / 2) / dz) ** 2
    w = 2.0 / dt * math.asin(dt * math.sqrt(kap2))
    nsteps = 1000
    for _ in range(nsteps):
        sim.yee()
    got = {"Ey": sim.E[1], "By": sim.B[1], "Bz": sim.B[2]}[comp]
    err = np.max(np.abs(got - math.cos(nsteps * w * dt) * mode))
    assert err < 1e-11, err


@pytest.mark.parametrize("comp", ["Ey", "By"])
@pytest.mark.parametrize("alpha", [0.5, 0.9, 0.99])
def test_ck_standing_mode_dispersion(comp, alpha):
    """Cole-Karkkainen (beta = 1/8, square cells): Faraday's differences are
    averaged across lines with (1/8, 3/4, 1/8), whose symbol is 1 - sin^2(k/2)/2,
    so a standing mode oscillates as cos(n w dt) with
    sin^2(w dt/2)/dt^2 = sx (1 - sz/2) + sz (1 - sx/2), sx = sin^2(kx/2), sz = sin^2(kz/2),
    also above the 2D Yee limit alpha < 1/sqrt(2) (Secs. 2-3 run it up to alpha near 1)."""
    n = (24, 32)
    wl = _wl(dims=2, n=n, alpha=alpha, correction=False, filter=[], solver="ck")
    sim = _empty_sim(wl)
    nz, ny, nx = sim.shape
    kx, kz = 2 * math.pi * 5 / nx, 2 * math.pi * 7 / nz
    i = np.arange(nx)[None, None, :]
    k = np.arange(nz)[:, None, None]
    if comp == "Ey":
        mode = np.sin(kx * i) * np.sin(kz * k) * np.ones((1, ny, 1))
        sim.E[1][:] = mode
    else:
        mode = np.cos(kx * (i + 0.5)) * np.cos(kz * (k + 0.5)) * np.ones((1, ny, 1))
        sim.B[1][:] = mode
    dt = sim.s.dt
    sx, sz = math.sin(kx / 2) ** 2, math.sin(kz / 2) ** 2
    w = 2.0 / dt * math.asin(dt * math.sqrt(sx * (1 - sz / 2) + sz * (1 - sx / 2)))
    nsteps = 1000
    for _ in range(nsteps):
        sim.yee()
    got = sim.E[1] if comp == "Ey" else sim.B[1]
    err = np.max(np.abs(got - math.cos(nsteps * w * dt) * mode))
    assert err < 1e-10, err


def test_ck_stable_where_yee_is_not():
    """At alpha = 0.95 on square 2D cells the Yee update amplifies the grid's
    highest mode (Courant limit 1/sqrt(2)); the Cole-Karkkainen update keeps
    random vacuum fields bounded over 2000 steps (its limit is alpha = 1)."""
    rng = np.random.default_rng(9)
    E0 = rng.normal(size=(3, 16, 1, 16))
    B0 = rng.normal(size=(3, 16, 1, 16))
    peak = {}
    for solver in ("yee", "ck"):
        wl = _wl(dims=2, n=(16, 16), alpha=0.95, correction=False, filter=[], solver=solver)
        sim = _empty_sim(wl)
        sim.E[:] = E0
        sim.B[:] = B0
        e0 = float(np.sum(sim.E ** 2) + np.sum(sim.B ** 2))
        worst = 1.0
        for _ in range(2000):
            sim.yee()
            worst = max(worst, float(np.sum(sim.E ** 2) + np.sum(sim.B ** 2)) / e0)
            if worst > 1e6:
                break
        peak[solver] = worst
    assert peak["yee"] > 1e6
    assert peak["ck"] < 20.0, peak


# ---------------------------------------------------------- Boris (textbook)

def _single_particle_sim(dims, B=None, E=None, gamma=3.0, order=1, corr=True):
    n = (16, 16) if dims == 2 else (8, 8, 8)
    wl = _wl(dims=dims, n=n, order=order, correction=corr, filter=pi.workloads.BINOMIAL4,
             alpha=0.4, ion_mode=0)
    x = np.full((1, dims), 4.3)
    u = np.array([[0.0, 0.0, math.sqrt(gamma ** 2 - 1)]])
    sim = OracleSim(wl, x, u, weight=0.0)   # zero weight: no self-field
    for c in range(3):
        if B is not None:
            sim.B[c][:] = B[c]
        if E is not None:
            sim.E[c][:] = E[c]
    return sim


@pytest.mark.parametrize("dims", [2, 3])
def test_boris_gyration_in_uniform_B(dims):
    """Textbook Boris (1970): in uniform B the push is an exact rotation by
    phi = 2 atan(|q| B dt / (2 m gamma)) per step and |u| is conserved."""
    B0 = 0.3
    sim = _single_particle_sim(dims, B=(0.0, B0, 0.0))
    u0 = sim.u[:, 0].copy()
    g = math.sqrt(1 + u0 @ u0)
    phi = 2 * math.atan(abs(sim.s.q) * B0 * sim.s.dt / (2 * sim.s.m * g))
    nsteps = 200
    sim.step(nsteps)
    th = nsteps * phi
    # q < 0 and B along +y: rotation about +y by +phi each step
    ux = u0[0] * math.cos(th) + u0[2] * math.sin(th)
    uz = -u0[0] * math.sin(th) + u0[2] * math.cos(th)
    assert abs(np.linalg.norm(sim.u[:, 0]) - np.linalg.norm(u0)) < 1e-13
    assert abs(sim.u[0, 0] - ux) < 1e-12 and abs(sim.u[2, 0] - uz) < 1e-12
    assert abs(sim.u[1, 0]) < 1e-15


def test_boris_uniform_E_acceleration():
    """With E only, each step adds q E dt / m to u exactly."""
    E0 = 0.02
    sim = _single_particle_sim(2, E=(0.0, 0.0, E0))
    uz0 = sim.u[2, 0]
    sim.step(50)
    assert abs(sim.u[2, 0] - (uz0 + 50 * sim.s.q * E0 * sim.s.dt / sim.s.m)) < 1e-12


# --------------------------------------------------------------- gather

@pytest.mark.parametrize("interp", ["galerkin", "uniform", "momentum"])
@pytest.mark.parametrize("dims,order", [(2, 1), (2, 3), (3, 1), (3, 3)])
def test_gather_partition_of_unity(dims, order, interp):
    """Every spline set sums to one (and a node average of a constant is that
    constant), so uniform seen fields are reproduced exactly."""
    n = (16, 16) if dims == 2 else (8, 8, 8)
    wl = _wl(dims=dims, n=n, order=order, correction=True, filter=pi.workloads.BINOMIAL4,
             interp=interp)
    sim = _empty_sim(wl)
    vals = [0.3, -1.1, 2.5, 0.7, -0.2, 1.9]
    for c in range(3):
        sim.E[c][:] = vals[c]
        sim.B[c][:] = vals[3 + c]
    sim.seen()
    rng = np.random.default_rng(2)
    L = np.array([n[0], 1.0, n[-1]]) if dims == 2 else np.array(n, float)
    for _ in range(50):
        p = rng.random(3) * L
        Eo, Bo = sim.gather_at(p)
        assert np.max(np.abs(np.concatenate([Eo, Bo]) - vals)) < 1e-14


STAG = {"Ex": (1, 0, 0), "Ey": (0, 1, 0), "Ez": (0, 0, 1),
        "Bx": (0, 1, 1), "By": (1, 0, 1), "Bz": (1, 1, 0)}


def _gather_response(sim, axis, kk, npt=12):
    """Cell average of g(x_a) exp(-i k x_a) for every gathered component, where
    g is the gather of the plane wave exp(i k x_a) sampled at each component's
    own Yee location.  By Poisson summation this average is the Fourier
    transform of the component's interpolation function along the axis (the
    shape factor S of the Eq. 1 ratio)."""
    names = ["Ex", "Ey", "Ez", "Bx", "By", "Bz"]
    nz, ny, nx = sim.shape
    coord = {0: np.arange(nx)[None, None, :], 1: np.arange(ny)[None, :, None],
             2: np.arange(nz)[:, None, None]}[axis]
    gl, gw = np.polynomial.legendre.leggauss(npt)
    # the interpolation functions are polynomial on each half cell
    pts = np.concatenate([0.25 + 0.25 * gl, 0.75 + 0.25 * gl])
    wts = np.concatenate([0.25 * gw, 0.25 * gw])
    acc = np.zeros(6, complex)
    for part, fn in ((1.0, np.cos), (1j, np.sin)):
        for c, nm in enumerate(names):
            plane = fn(kk * (coord + 0.5 * STAG[nm][axis])) * np.ones(sim.shape)
            (sim.Et if c < 3 else sim.Bt)[c % 3][:] = plane
        for t, wgt in zip(pts, wts):
            p = np.array([2.3, 1.7, 3.1])   # off-node in every other axis
            p[axis] = 3.0 + t
            Eo, Bo = sim.gather_at(p)
            g = np.concatenate([Eo, Bo])
            acc += part * wgt * g * np.exp(-1j * kk * p[axis])
    return dict(zip(names, acc))


@pytest.mark.parametrize("interp", ["galerkin", "uniform", "momentum"])
@pytest.mark.parametrize("dims,order", [(2, 1), (2, 3), (3, 1), (3, 3)])
def test_gather_shape_factors_match_eqs_3_to_5(dims, order, interp):
    """Fourier transform of each component's gather along each axis against its
    closed form: a centred order-o B-spline has transform sinc(k/2)^(o+1);
    Galerkin lowers o by one along half-staggered axes, Uniform keeps o = l,
    and the node average of the momentum-conserving scheme multiplies by
    cos(k/2) along half-staggered axes.  The z ratio S^By / S^Ex then equals the
    ratio of the scheme's multiplier to the Uniform one, since the Eq. 1
    multiplier differs between schemes only through S^By / S^Ex, which is 1 for
    Uniform (Eqs. 3-5: theta / sin(theta), 1 and cos(theta), theta = k_z dz / 2).
    A wrong order, a wrong stagger offset (a phase) or a node average taken
    from the wrong neighbours fails here."""
    n = (16, 16) if dims == 2 else (8, 8, 8)
    wl = _wl(dims=dims, n=n, order=order, correction=False, filter=[], interp=interp)
    sim = _empty_sim(wl)
    axes = (0, 2) if dims == 2 else (0, 1, 2)
    for axis in axes:
        na = n[axis] if dims == 3 else n[0 if axis == 0 else 1]
        for m in range(1, na // 2 + 1):
            kk = 2.0 * math.pi * m / na
            th = 0.5 * kk
            R = _gather_response(sim, axis, kk)
            for nm, st in STAG.items():
                o = order - st[axis] if interp == "galerkin" else order
                want = (math.sin(th) / th) ** (o + 1)
                if interp == "momentum" and st[axis]:
                    want *= math.cos(th)
                assert abs(R[nm] - want) < 1e-13, (axis, m, nm, R[nm], want)
            if axis == 2:
                s = math.sin(th) ** 2
                ratio = float(psi.multiplier(interp, 0.5, s) / psi.multiplier("uniform", 0.5, s))
                assert abs(R["By"] - ratio * R["Ex"]) < 1e-13, (m, R["By"], R["Ex"], ratio)


# ------------------------------------------------------------ Esirkepov

def _noisy_beam_sim(dims, order, n, ppc=2, seed=5, steps_fields=True):
    wl = _wl(dims=dims, n=n, order=order, ppc=ppc, gamma=4.0, correction=True,
             filter=pi.workloads.BINOMIAL4, alpha=0.4 if dims == 2 else 0.35)
    x, u = pi.load_beam(dims, n, ppc, 4.0, 0.3, seed)
    sim = OracleSim(wl, x, u)
    rng = np.random.default_rng(seed)
    sim.E[:] = rng.normal(size=sim.E.shape) * 0.05
    sim.B[:] = rng.normal(size=sim.B.shape) * 0.05
    return sim


@pytest.mark.parametrize("dims,order", [(2, 1), (2, 3), (3, 1), (3, 3)])
def test_esirkepov_discrete_continuity(dims, order):
    """Esirkepov (2001): rho^{n+1} - rho^n + dt div J = 0 on the grid, per step."""
    n = (12, 16) if dims == 2 else (8, 8, 10)
    sim = _noisy_beam_sim(dims, order, n)
    rho0 = sim.rho()
    sim.yee()
    sim.seen()
    sim.push_deposit()
    resid = sim.rho() - rho0 + sim.s.dt * sim.div(sim.J)
    assert np.max(np.abs(resid)) < 1e-13 * np.max(np.abs(rho0))
    assert sim.status == 0


def test_gauss_invariant_over_long_run():
    """div E - rho stays at its initial value to rounding over every step of a run
    with the instability growing (beam, no correction, no filter)."""
    wl = _wl(n=(16, 16), ppc=4, correction=False, filter=[])
    x, u = pi.load_beam(2, (16, 16), 4, 130.0, 1e-3, 7)
    sim = OracleSim(wl, x, u)
    rmax = np.max(np.abs(sim.rho0))
    worst = 0.0
    for _ in range(400):
        sim.step(1)
        worst = max(worst, float(np.max(np.abs(sim.gauss_residual()))))
    assert worst < 1e-12 * rmax, worst


# ---------------------------------------------------- brute force (8x8 etc.)

def _brute_pair(dims, n, order, filt, corr=True, npart=10, seed=3, steps=20, interp="galerkin",
                solver="yee", alpha=None):
    """corr: False, True (Psi_E / Psi_B split over the components) or "ratio"."""
    if alpha is None:
        alpha = 0.45 if dims == 2 else 0.4
    wl = _wl(dims=dims, n=n, order=order, correction=corr, filter=list(filt),
             alpha=alpha, gamma=3.0, interp=interp, solver=solver)
    rng = np.random.default_rng(seed)
    x = rng.random((npart, dims)) * np.array(n, float)
    u = rng.normal(size=(npart, 3)) * 0.8 + np.array([0.0, 0.0, 1.5])
    o = OracleSim(wl, x, u)
    o.E[:] = rng.normal(size=o.E.shape) * 0.05
    o.B[:] = rng.normal(size=o.B.shape) * 0.05
    s = o.s
    b = BruteSim(dims, o.shape, (s.dx, s.dy, s.dz), s.dt, order, s.q, s.m, s.w,
                 psi_e=o.psi[0] if o.psi else None, psi_b=o.psi[1] if o.psi else None,
                 filt=filt, jbg=tuple(_loader_background_current(wl, u, s.w, o.dV * float(np.prod(o.shape)))),
                 interp=interp, solver=solver, ratio=(corr == "ratio"))
    b.E[:] = o.E
    b.B[:] = o.B
    bx, bu = o.x.copy(), o.u.copy()
    for _ in range(steps):
        o.step(1)
        b.step(bx, bu)
    return o, b, bx, bu


@pytest.mark.parametrize("interp", ["galerkin", "uniform", "momentum"])
@pytest.mark.parametrize("dims,n,order,steps", [
    (2, (8, 8), 1, 20), (2, (8, 10), 3, 20), (3, (8, 8, 8), 1, 4), (3, (8, 8, 9), 3, 2)])
def test_oracle_matches_brute_force(dims, n, order, steps, interp):
    """Full step (Yee, Psi, filter, gather of each scheme, Boris, move, Esirkepov)
    against the dense/DFT brute force on tiny grids."""
    o, b, bx, bu = _brute_pair(dims, n, order, (0.25, 0.25, -1.0), steps=steps,
                               npart=10 if dims == 2 else 4, interp=interp)

    def rel(a, r):
        return np.linalg.norm(a - r) / np.linalg.norm(r)
    assert rel(o.E, b.E) < 1e-13 and rel(o.B, b.B) < 1e-13 and rel(o.J, b.J) < 1e-13
    assert rel(o.u, bu) < 1e-13
    dx = np.abs(o.x - bx)
    L = [n[0], 1, n[1]] if dims == 2 else list(n)
    for a in range(3):
        dx[a] = np.minimum(dx[a], L[a] - dx[a])
    assert dx.max() < 1e-12


@pytest.mark.parametrize("order,interp", [(1, "galerkin"), (3, "galerkin"), (1, "uniform")])
def test_oracle_ck_matches_brute_force(order, interp):
    """Full 2D steps with the Cole-Karkkainen solver at alpha = 0.9 against the
    brute force, whose modified curl is a product of dense matrices."""
    n = (8, 10)
    o, b, bx, bu = _brute_pair(2, n, order, (0.25, 0.25, -1.0), steps=15, interp=interp,
                               solver="ck", alpha=0.9)

    def rel(a, r):
        return np.linalg.norm(a - r) / np.linalg.norm(r)
    assert rel(o.E, b.E) < 1e-13 and rel(o.B, b.B) < 1e-13 and rel(o.J, b.J) < 1e-13
    assert rel(o.u, bu) < 1e-13


@pytest.mark.parametrize("dims,n,steps", [(2, (8, 10), 15), (3, (8, 8, 8), 3)])
def test_oracle_exact_ratio_matches_brute_force(dims, n, steps):
    """The exact-ratio variant (Psi_E / Psi_B on the transverse E only, by dense
    LU solves along z) against the brute force, which multiplies by the ratio in
    Fourier space."""
    o, b, bx, bu = _brute_pair(dims, n, 1, (0.25, 0.25, -1.0), corr="ratio", steps=steps,
                               npart=10 if dims == 2 else 4)

    def rel(a, r):
        return np.linalg.norm(a - r) / np.linalg.norm(r)
    assert rel(o.E, b.E) < 1e-13 and rel(o.B, b.B) < 1e-13 and rel(o.J, b.J) < 1e-13
    assert rel(o.u, bu) < 1e-13


# --------------------------------------------------------- growth fit

def test_growth_fit_recovers_rate():
    dt, gam = 0.5, 0.013
    t = np.arange(2000) * dt
    W = 1e-12 * np.exp(2 * gam * t) + 1e-12
    G, (lo, hi) = ofit.growth_rate(list(W), dt, wkin0=1e4)
    assert lo > 0 and abs(G - gam) < 0.02 * gam


def _ramp_then_growth(dt, gam, n_ramp, n, w_sat):
    """A run's shape: W climbs from ~0 along a straight ramp (the start-up rise to
    the noise level), then grows as exp(2 gam t) until it saturates at w_sat."""
    t = np.arange(n) * dt
    W = 1e-3 * (np.arange(n) + 1e-12)
    W[n_ramp:] = W[n_ramp - 1] * np.exp(2 * gam * (t[n_ramp:] - t[n_ramp - 1]))
    return np.minimum(W, w_sat)


@pytest.mark.parametrize("dt,gam,n_ramp", [(0.5, 0.01, 300), (0.3, 0.006, 500), (0.7, 0.02, 150)])
def test_growth_fit_leaves_out_the_startup_ramp(dt, gam, n_ramp):
    """The start-up rise has a steep log-slope (1/t) early on; the window must sit
    in the exponential phase and recover its rate within 1 %, on both fits, and
    stop before the saturation cap."""
    from paper_1401_0838_amd import fit as gfit
    wkin0 = 1e4
    W = _ramp_then_growth(dt, gam, n_ramp, 2000, 0.5 * wkin0)
    for G, (lo, hi) in (ofit.growth_rate(list(W), dt, wkin0), gfit.growth_rate(W, dt, wkin0)):
        assert lo >= n_ramp - 1, (lo, hi)
        assert W[hi - 1] <= 1e-2 * wkin0 * math.exp(2 * gam * dt) + 1e-12
        assert abs(G - gam) < 0.01 * gam, (G, gam)
    # a planted mistake: starting the search at step 1 fits the ramp's 1/t slope
    G_bad = ofit.growth_rate(list(W), dt, wkin0, omega_p=1e6)[0]
    assert abs(G_bad - gam) > 0.1 * gam


def test_growth_fits_agree_on_a_noisy_trace():
    """The oracle's plain-loop fit and the library's running-sum fit give the same
    rate and window on an irregular trace."""
    from paper_1401_0838_amd import fit as gfit
    rng = np.random.default_rng(4)
    n, dt = 1200, 0.45
    W = _ramp_then_growth(dt, 0.008, 250, n, 1e9) * np.exp(0.2 * rng.standard_normal(n))
    a = ofit.growth_rate(list(W), dt, 1e4)
    b = gfit.growth_rate(W, dt, 1e4)
    assert a[1] == b[1] and abs(a[0] - b[0]) < 1e-9 * abs(a[0])


# --------------------------------------------------------------- loader

def test_loader_is_stratified_and_seeded():
    x, u = pi.load_beam(2, (8, 6), 4, 130.0, 1e-4, 11)
    cells = np.floor(x[:, 0]).astype(int) + 8 * np.floor(x[:, 1]).astype(int)
    assert np.all(np.bincount(cells, minlength=48) == 4)
    assert np.all(cells == np.repeat(np.arange(48), 4))
    x2, u2 = pi.load_beam(2, (8, 6), 4, 130.0, 1e-4, 11)
    assert np.array_equal(x, x2) and np.array_equal(u, u2)
    assert abs(np.mean(u[:, 2]) / math.sqrt(130.0 ** 2 - 1) - 1) < 1e-4


# ------------------------------------------------- ion background current

def _loader_background_current(wl, u, weight, V):
    """Closed form of the immobile ions' uniform current, computed here from the
    loader's momenta and not read from the oracle: minus the beam's initial mean
    current q w sum_p v_p / V, with v = u / sqrt(1 + u^2)."""
    if wl.get("ion_mode", 1) != 1:
        return np.zeros(3)
    v = u / np.sqrt(1.0 + np.sum(u * u, axis=1))[:, None]
    return -wl["q"] * weight * v.sum(axis=0) / V


@pytest.mark.parametrize("ion_mode,sigma", [(0, 1e-3), (1, 1e-3), (1, 0.0)])
def test_uniform_mode_of_E_follows_ampere_with_ion_current(ion_mode, sigma):
    """The k = 0 mode of E obeys dE/dt = -(mean J + J_ion) exactly on a periodic
    grid (the curl of B has zero mean), and the Esirkepov current's mean is the
    beam's charge times its displacement per step.  A step's Yee update uses the
    current deposited by the step before, so after N steps
        mean E_a = -(q w / V) sum_p (displacement of p along a in steps 1..N-1)
                   - N dt J_ion,a
    (2D y: the displacement is dt sum_n v_y^{n+1/2}).  J_ion is the closed form
    above; with ions carrying charge only it is zero and E_z ramps."""
    wl = _wl(n=(16, 12), ppc=4, correction=False, filter=[], ion_mode=ion_mode)
    x, u = pi.load_beam(2, (16, 12), 4, 130.0, sigma, 5)
    sim = OracleSim(wl, x, u)
    q, w, dt = wl["q"], sim.s.w, sim.s.dt
    V = 16 * 12 * sim.dV
    jion = _loader_background_current(wl, u, w, V)
    L = np.array([16.0, 12.0])
    disp = np.zeros(3)
    prev = sim.positions()
    N = 200
    for n in range(N):
        if n == N - 1:
            held = disp.copy()          # the last deposit is not in E yet
        sim.step(1)
        cur = sim.positions()
        d = cur - prev
        d -= L * np.round(d / L)            # minimum image: |step| < one cell
        disp[0] += d[:, 0].sum()
        disp[2] += d[:, 1].sum()
        gam = np.sqrt(1.0 + np.sum(sim.u ** 2, axis=0))
        disp[1] += dt * np.sum(sim.u[1] / gam)
        prev = cur
    assert sim.status == 0
    scale = N * dt * abs(q) * w * x.shape[0] / V      # |ramp| if every particle moved at c
    for a in range(3):
        pred = -(q * w / V) * held[a] - N * dt * jion[a]
        got = float(np.mean(sim.E[a]))
        assert abs(got - pred) < 1e-12 * scale, (a, got, pred)
    Ez = float(np.mean(sim.E[2]))
    if ion_mode == 0:
        # the beam's own current ramps E_z at about -N dt q n0 v
        assert Ez > 0.9 * scale
    elif sigma == 0.0:
        # cold beam with the ion current: no ramp.  The uniform E_z holds the one
        # step of ion current the first update applied before any deposit
        # (J^{-1/2} = 0), -dt J_ion,z, up to the small changes of the particles'
        # velocities in the noise fields (the exact balance is asserted above)
        assert abs(Ez + dt * jion[2]) < 1e-5 * scale, (Ez, -dt * jion[2])


def test_oracle_background_current_matches_closed_form():
    """The value the oracle uses equals the closed form from the loader's momenta
    (sign and scale), for a drifting beam with transverse spread."""
    wl = _wl(n=(8, 6), ppc=3)
    x, u = pi.load_beam(2, (8, 6), 3, 50.0, 0.3, 9)
    sim = OracleSim(wl, x, u)
    V = 8 * 6 * sim.dV
    ref = _loader_background_current(wl, u, sim.s.w, V)
    assert np.allclose(np.array(sim.s.jbg[:]), ref, rtol=1e-14, atol=0.0)
    assert ref[2] > 0      # electrons (q < 0) drifting along +z: the ions' current is +z
