// Host setup of the correction-stencil coefficients (Sec. 2, Eqs. 3-5).
//
// The multiplier M(s) that zeroes the m_z = 0 mismatch term at omega = k_z is
// approximated by Psi_E(s) / Psi_B(s), two polynomials of degree deg in
// s = sin^2(k_z dz / 2), by rational interpolation at 2*deg+1 nodes spaced
// uniformly on [0, 1] with Psi_B(0) = 1.  The linear system is badly
// conditioned (around 1e8 for quartics), so it is assembled and solved in
// 113-bit binary floating point (libquadmath) and only the result is rounded
// to double.  Built with g++ (quadmath is a GCC runtime library).
#include <quadmath.h>

#include <cmath>
#include <complex>

#include "pic_api.h"

namespace {

typedef __float128 quad;

quad multiplier(int interp, quad alpha, quad s)
{
    if (s == 0) return 1;
    quad th = asinq(sqrtq(s));       // theta = k_z dz / 2
    quad sn = sinq(th);
    quad num = sinq(2 * alpha * th); // 2 sin(k dt/2) cos(k dt/2)
    switch (interp) {
    case PIC_GALERKIN: return num * th / (2 * alpha * sn * sn);         // Eq. 3
    case PIC_UNIFORM:  return num / (2 * alpha * sn);                   // Eq. 4
    default:           return num * cosq(th) / (2 * alpha * sn);        // Eq. 5
    }
}

}  // namespace

// Real roots of sum_j coef[j] s^j (degree deg, trailing zero coefficients
// dropped): Weierstrass (Durand-Kerner) iteration in long double, each root
// then polished by Newton steps on the real axis.  Returns the number of
// roots written to roots[] and the leading coefficient in *lead, or -1 if a
// root is not real (|Im r| > 1e-9 (1 + |r|)).
int psi_real_roots(const double *coef, int deg, double *roots, double *lead)
{
    typedef std::complex<long double> cl;
    while (deg > 0 && coef[deg] == 0.0) deg--;
    *lead = coef[deg];
    if (deg == 0) return 0;
    auto p = [&](cl z) {
        cl acc = 0;
        for (int i = deg; i >= 0; i--) acc = acc * z + (long double)coef[i];
        return acc;
    };
    cl z[8];
    const cl seed(0.4L, 0.9L);
    z[0] = 1;
    for (int k = 1; k < deg; k++) z[k] = z[k - 1] * seed;
    for (int k = 0; k < deg; k++) z[k] *= seed;
    for (int it = 0; it < 2000; it++) {
        long double moved = 0;
        for (int k = 0; k < deg; k++) {
            cl den = (long double)coef[deg];
            for (int j = 0; j < deg; j++)
                if (j != k) den *= z[k] - z[j];
            const cl step = p(z[k]) / den;
            z[k] -= step;
            moved = std::max(moved, std::abs(step) / (1.0L + std::abs(z[k])));
        }
        if (moved < 1e-18L) break;
    }
    for (int k = 0; k < deg; k++) {
        if (std::fabs(z[k].imag()) > 1e-9L * (1.0L + std::abs(z[k]))) return -1;
        long double r = z[k].real();
        for (int it = 0; it < 8; it++) {
            long double f = 0, df = 0;
            for (int i = deg; i >= 0; i--) { df = df * r + f; f = f * r + (long double)coef[i]; }
            if (df == 0) break;
            r -= f / df;
        }
        roots[k] = (double)r;
    }
    return deg;
}

// Breakdown test (Sec. 3): Psi_B > 0 on [0, 1] and Psi_E > 0 on [0, 1), on a
// 4097-point grid.  The Eq. 5 multiplier is exactly zero at s = 1 (its
// cotangent vanishes at k_z dz = pi), so there Psi_E only has to be zero up
// to rounding: Psi_E(1) >= -1e-12 sum |psi_e[i]|.
bool psi_positive(const double *psi_e, const double *psi_b, int deg)
{
    double tol = 0.0;
    for (int i = 0; i <= deg; i++) tol += std::fabs(psi_e[i]);
    tol *= 1e-12;
    for (int k = 0; k <= 4096; k++) {
        double s = k / 4096.0, pe = 0, pb = 0;
        for (int i = deg; i >= 0; i--) { pe = pe * s + psi_e[i]; pb = pb * s + psi_b[i]; }
        if (!(pb > 0.0)) return false;
        if (!(pe > 0.0) && !(k == 4096 && pe >= -tol)) return false;
    }
    return true;
}

extern "C" int pic_psi_coeffs(int interp, double alpha_d, int deg, double *psi_e, double *psi_b)
{
    if (!psi_e || !psi_b || deg < 1 || deg > 8 || !(alpha_d > 0.0) || alpha_d >= 1.0 ||
        interp < PIC_GALERKIN || interp > PIC_MOMENTUM)
        return PIC_EINVAL;
    const int nn = 2 * deg + 1;
    const quad alpha = alpha_d;
    quad M[17];
    quad dev = 0;
    for (int j = 0; j < nn; j++) {
        M[j] = multiplier(interp, alpha, (quad)j / (nn - 1));
        quad d = fabsq(M[j] - 1);
        if (d > dev) dev = d;
    }
    for (int i = 0; i <= deg; i++) psi_e[i] = psi_b[i] = (i == 0) ? 1.0 : 0.0;
    if (dev < (quad)1e-28) return PIC_OK;   // multiplier identically 1: identity

    // unknowns a_0..a_deg, b_1..b_deg;  sum a_i s^i - M sum_{i>=1} b_i s^i = M
    quad A[17][18];
    for (int r = 0; r < nn; r++) {
        quad s = (quad)r / (nn - 1), p = 1;
        for (int i = 0; i <= deg; i++) {
            A[r][i] = p;
            if (i >= 1) A[r][deg + i] = -M[r] * p;
            p *= s;
        }
        A[r][nn] = M[r];
    }
    quad scale = 0;
    for (int r = 0; r < nn; r++)
        for (int c = 0; c < nn; c++) scale = fmaxq(scale, fabsq(A[r][c]));
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < nn; c++) {
        int piv = c;
        for (int r = c + 1; r < nn; r++)
            if (fabsq(A[r][c]) > fabsq(A[piv][c])) piv = r;
        if (fabsq(A[piv][c]) < scale * (quad)1e-30) return PIC_EPSI;
        if (piv != c)
            for (int k = 0; k <= nn; k++) { quad t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
        for (int r = c + 1; r < nn; r++) {
            quad f = A[r][c] / A[c][c];
            for (int k = c; k <= nn; k++) A[r][k] -= f * A[c][k];
        }
    }
    quad x[17];
    for (int r = nn - 1; r >= 0; r--) {
        quad acc = A[r][nn];
        for (int k = r + 1; k < nn; k++) acc -= A[r][k] * x[k];
        x[r] = acc / A[r][r];
    }
    for (int i = 0; i <= deg; i++) psi_e[i] = (double)x[i];
    for (int i = 1; i <= deg; i++) psi_b[i] = (double)x[deg + i];
    return psi_positive(psi_e, psi_b, deg) ? PIC_OK : PIC_EPSI;
}
