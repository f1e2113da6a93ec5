"""Correction-stencil coefficients Psi_E / Psi_B (oracle side, 50 digits).

Test infrastructure only.

Sec. 2 gives, for the multiplier that cancels the m_z = 0 mismatch term C2 at
omega = k_z, closed forms for three interpolation schemes: Eq. 3 (Galerkin),
Eq. 4 (Uniform) and Eq. 5 (momentum-conserving).  With theta = k_z dz / 2,
s = sin^2(theta) and alpha = c dt / dz they read
    M_G(s) = sin(2 alpha theta) theta / (2 alpha sin^2 theta)
    M_U(s) = sin(2 alpha theta) / (2 alpha sin theta)
    M_M(s) = sin(2 alpha theta) cos theta / (2 alpha sin theta)
each tending to 1 as s -> 0.

Sec. 2 then approximates M by a ratio of quartics in s, Psi_E(s) / Psi_B(s),
obtained by rational interpolation through nine points spaced uniformly in
s on [0, 1].  Reading taken here: nodes s_j = j / 8 with both ends included,
normalisation b_0 = 1 (so both polynomials equal 1 at s = 0), solved in
50-digit arithmetic and rounded to float64.  When M is identically 1 (the
Uniform scheme at the alpha = 1/2 "magic" step of Sec. 4) the system is
singular; the reading is Psi_E = Psi_B = 1.
"""
import mpmath as mp

DPS = 50


def multiplier(interp, alpha, s):
    """M(s) of Eq. 3 ('galerkin'), Eq. 4 ('uniform') or Eq. 5 ('momentum')."""
    with mp.workdps(DPS):
        s = mp.mpf(s)
        alpha = mp.mpf(alpha)
        if s == 0:
            return mp.mpf(1)
        th = mp.asin(mp.sqrt(s))
        num = mp.sin(2 * alpha * th)
        if interp == "galerkin":
            return num * th / (2 * alpha * mp.sin(th) ** 2)
        if interp == "uniform":
            return num / (2 * alpha * mp.sin(th))
        if interp == "momentum":
            return num * mp.cos(th) / (2 * alpha * mp.sin(th))
        raise ValueError(interp)


def multiplier_slope0(interp, alpha):
    """dM/ds at s = 0 from the Taylor expansion of Eqs. 3-5 in theta.

    With sin(2 a th) = 2 a th (1 - (2 a th)^2 / 6 + ...), sin^2 th = th^2 (1 - th^2/3 + ...),
    s = th^2 + O(th^4):  M_G = 1 + (1 - 2 a^2)/3 s,  M_U = 1 + (1 - 4 a^2)/6 s,
    M_M = M_U (1 - s/2) = 1 + ((1 - 4 a^2)/6 - 1/2) s.
    """
    a2 = alpha * alpha
    if interp == "galerkin":
        return (1.0 - 2.0 * a2) / 3.0
    if interp == "uniform":
        return (1.0 - 4.0 * a2) / 6.0
    if interp == "momentum":
        return (1.0 - 4.0 * a2) / 6.0 - 0.5
    raise ValueError(interp)


def psi_coeffs(interp, alpha, deg=4):
    """Return (a, b, identity): power-series coefficients of Psi_E and Psi_B in s.

    Solves sum_i a_i s_j^i - M(s_j) sum_{i>=1} b_i s_j^i = M(s_j) at the
    2*deg + 1 nodes s_j = j / (2*deg), with b_0 = 1.
    """
    nn = 2 * deg + 1
    with mp.workdps(DPS):
        nodes = [mp.mpf(j) / (nn - 1) for j in range(nn)]
        Ms = [multiplier(interp, alpha, sj) for sj in nodes]
        if max(abs(Mj - 1) for Mj in Ms) < mp.mpf(10) ** (-DPS // 2):
            return [1.0] + [0.0] * deg, [1.0] + [0.0] * deg, True
        A = mp.matrix(nn, nn)
        rhs = mp.matrix(nn, 1)
        for r, (sj, Mj) in enumerate(zip(nodes, Ms)):
            for i in range(deg + 1):
                A[r, i] = sj ** i
            for i in range(1, deg + 1):
                A[r, deg + i] = -Mj * sj ** i
            rhs[r] = Mj
        sol = mp.lu_solve(A, rhs)
        a = [float(sol[i]) for i in range(deg + 1)]
        b = [1.0] + [float(sol[deg + i]) for i in range(1, deg + 1)]
        return a, b, False


def poly(c, s):
    """Evaluate sum_i c_i s^i (float or mpf)."""
    acc = 0
    for ci in reversed(c):
        acc = acc * s + ci
    return acc


def psi_positive(a, b, npts=4096):
    """True when the determination has not broken down (Sec. 3): Psi_B > 0 on a
    uniform grid of [0, 1] and Psi_E > 0 on [0, 1).  At s = 1 (k_z dz = pi)
    the momentum-conserving multiplier of Eq. 5 is exactly zero (the cotangent
    vanishes), so the interpolant's Psi_E(1) is zero up to rounding there;
    Psi_E(1) only has to be >= -1e-12 sum |a_i|."""
    tol = 1e-12 * sum(abs(v) for v in a)
    for i in range(npts + 1):
        s = i / npts
        pe, pb = poly(a, s), poly(b, s)
        if pb <= 0.0:
            return False
        if pe <= 0.0 and not (i == npts and pe >= -tol):
            return False
    return True
