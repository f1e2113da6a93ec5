"""Workload parameter tables for the synthetic beams (shapes of Sec. 3).

Units: c = 1, eps0 = mu0 = 1, cell size 1 on every axis, electron charge
q = -1 and mass m = 1, so alpha = c*dt/dz is dt itself.  The plasma
frequency is held at omega_p = 0.1 (omega_p*dt = 0.05 at alpha = 0.5), which
fixes the beam density n0 = omega_p^2 * m / q^2.  The beam moves along +z.

Each workload is a plain dict of parameters; filter passes are listed
explicitly as the weight w of a 3-point (w, 1-2w, w) pass applied along every
axis (0.25 = bilinear, -1 = compensation).
"""
import numpy as np

_COMMON = dict(q=-1.0, m=1.0, omega_p=0.1, interp="galerkin", solver="yee", ion_mode=1)

BINOMIAL4 = [0.25, 0.25, 0.25, 0.25]
PAPER_EQ6 = [0.25, 0.25, -1.0, -1.0]      # two bilinear + two compensation passes
PAPER_EQ6_SQRT = [0.25, -1.0]             # one pass of each

WORKLOADS = {
    # 64x64, plain method (no correction, no filter), FP64, 200 steps
    "beam2d_64_fp64": dict(_COMMON, dims=2, n=(64, 64), alpha=0.5, gamma=130.0, ppc=4,
                           order=1, correction=False, filter=[], precision="fp64",
                           steps=200, seeds=(0, 1, 2), sigma=1e-6),
    # 512x512, correction + 4-pass binomial, FP64 and FP32, 2000 steps
    "beam2d_512": dict(_COMMON, dims=2, n=(512, 512), alpha=0.5, alphas=(0.3, 0.5, 0.7),
                       gamma=130.0, ppc=16, order=1, correction=True, filter=BINOMIAL4,
                       precision="fp32", steps=2000, seeds=(0,), sigma=1e-4),
    # 3D 128x128x256, cubic, correction + filter, FP32, 500 steps
    "beam3d_128x128x256": dict(_COMMON, dims=3, n=(128, 128, 256), alpha=0.5, gamma=130.0,
                               ppc=8, order=3, correction=True, filter=BINOMIAL4,
                               precision="fp32", steps=500, seeds=(0,), sigma=1e-6),
    # Sec. 3 setting: 128x128, cubic shapes, Cole-Karkkainen solver (beta = 1/8),
    # correction + the Eq. 6 filter, gamma 130, c dt / dz up to ~1
    "beam2d_128_ck": dict(_COMMON, dims=2, n=(128, 128), alpha=0.9, alphas=(0.5, 0.7, 0.9, 0.99),
                          gamma=130.0, ppc=16, order=3, correction=True, filter=PAPER_EQ6,
                          solver="ck", precision="fp32", steps=2000, seeds=(0,), sigma=1e-6),
    # 256x256 differentiation case, FP32 forward, 200 steps, checkpoints every 20
    "beam2d_256_adjoint": dict(_COMMON, dims=2, n=(256, 256), alpha=0.5, gamma=130.0, ppc=8,
                               order=1, correction=True, filter=BINOMIAL4, precision="fp32",
                               steps=200, checkpoint=20, seeds=(0,), sigma=1e-6),
}


def workload(name, **overrides):
    """Return a copy of a named workload with optional parameter overrides."""
    w = dict(WORKLOADS[name])
    w.update(overrides)
    w["name"] = name
    return w


def batched_candidates(seed=0, count=256):
    """Candidate instances for the batched scan (64 are used).

    nx, nz are drawn iid from {64, 128, 256, 512}, alpha uniform in [0.3, 0.7]
    (rounded to 1e-4 so that acceptance tests are reproducible), gamma from
    {10, 50, 130}.  A consumer walks the list in order and keeps the first 64
    whose correction coefficients it accepts; the particle seed of a candidate
    is its position in this list.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.array([64, 128, 256, 512])
    gammas = np.array([10.0, 50.0, 130.0])
    out = []
    for i in range(count):
        nx = int(rng.choice(sizes))
        nz = int(rng.choice(sizes))
        alpha = float(np.round(rng.uniform(0.3, 0.7), 4))
        gamma = float(rng.choice(gammas))
        out.append(dict(_COMMON, dims=2, n=(nx, nz), alpha=alpha, gamma=gamma, ppc=8,
                        order=1, correction=True, filter=BINOMIAL4, precision="fp32",
                        steps=1000, seeds=(1000 * seed + i,), sigma=1e-6,
                        name="batched_%d" % i))
    return out


# Sec. 3 variants of its CK / Eq. 6 setting, as workload overrides: no digital
# filtering apart from Psi_B; Psi_E / Psi_B on the transverse E only (Psi_B
# inverted); no compensation passes; the Sec. 4 filter with one pass of each
# kind (the square root of Eq. 6)
VARIANTS = {
    "baseline": dict(correction=True),
    "no_filter": dict(correction=True, filter=[]),
    "ratio_on_transverse_E": dict(correction="ratio"),
    "no_compensation": dict(correction=True, filter=[0.25, 0.25]),
    "sqrt_eq6": dict(correction=True, filter=PAPER_EQ6_SQRT),
}


def growth_cases():
    """Instances whose FP64 growth traces are stored as goldens, as
    (key, workload, particle seed, steps).  The 64-instance batch is not listed
    here: it is the first 64 accepted entries of batched_candidates(0).

    c1   : the 512x512 workload at its three alphas, 2000 steps
    scan : the Sec. 3 setting on a 64x64 grid with 8 ppc (gamma 3 and 130, alpha
           0.5 and 0.9, with and without the correction), 1000 steps; the seed of
           point (gamma index gi, alpha index ai) is 1000 gi + ai
    var  : the variants above in that setting at gamma 130, alpha 0.7 and 0.95,
           1000 steps; seed = alpha index
    """
    out = []
    base512 = workload("beam2d_512")
    for a in base512["alphas"]:
        out.append(("c1_a%g" % a, dict(base512, alpha=a, name="c1_a%g" % a), 0, 2000))
    for corr in (True, False):
        base = workload("beam2d_128_ck", n=(64, 64), ppc=8, correction=corr)
        for gi, g in enumerate((3.0, 130.0)):
            for ai, a in enumerate((0.5, 0.9)):
                k = "scan_%s_g%g_a%g" % ("corr" if corr else "plain", g, a)
                out.append((k, dict(base, alpha=a, gamma=g, name=k), 1000 * gi + ai, 1000))
    for name, over in VARIANTS.items():
        base = workload("beam2d_128_ck", n=(64, 64), ppc=8, gamma=130.0)
        base.update(over)
        for ai, a in enumerate((0.7, 0.95)):
            k = "var_%s_a%g" % (name, a)
            out.append((k, dict(base, alpha=a, name=k), ai, 1000))
    return out
