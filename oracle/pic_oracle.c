/*
 * FP64 CPU oracle for one FDTD-Esirkepov PIC timestep with the small-k_z
 * correction stencils of Godfrey & Vay (arXiv:1401.0838).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  It shares no code with the GPU library and is
 * never part of the product path.  Build: gcc -O2 -ffp-contract=off -shared.
 *
 * Conventions (c = eps0 = mu0 = 1).  Fields live on the Yee staggered mesh
 * (Sec. 2 names "the usual Yee staggered mesh"); the staggering of each
 * component, as offsets of half a cell along (x, y, z), is
 *     Ex (1,0,0)  Ey (0,1,0)  Ez (0,0,1)  Bx (0,1,1)  By (1,0,1)  Bz (1,1,0)
 * and J shares E's staggering.  A half-integer location i+1/2 is stored at
 * array index i.  Arrays are [nz][ny][nx], x fastest, periodic on every axis.
 * 2D runs use ny == 1 with y-invariance (2D3V: y is not tracked for particles).
 * Particles carry absolute positions and u = gamma*v per unit mass.
 *
 * One step (the order used throughout this project):
 *   1. Yee: B -= dt/2 curl E;  E += dt (curl B - J - Jbg);  B -= dt/2 curl E
 *      (with the Cole-Karkkainen solver named in Secs. 2-4, the curl of E in the
 *      two B half steps is its modified one; see yee_b_half)
 *   2. fields as seen by the particles: Psi series along z (Sec. 2), then the
 *      3-point digital filter passes along z, then x, then y (Sec. 3, Eq. 6)
 *   3. J = 0; per particle, in order: gather (Galerkin, Uniform or
 *      momentum-conserving: the schemes of Eqs. 3, 4 and 5), Boris push, move,
 *      Esirkepov deposit
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int dims;                 /* 2 or 3 */
    int nx, ny, nz;           /* ny == 1 when dims == 2 */
    double dx, dy, dz, dt;
    int order;                /* charge shape order l (1 or 3) */
    int interp;               /* 0 Galerkin, 1 Uniform, 2 momentum-conserving */
    int solver;               /* 0 Yee, 1 Cole-Karkkainen (2D, square cells) */
    double q, m, w;           /* charge, mass, macro-particle weight */
    int correction;           /* 0 none; 1 Psi_E on transverse E, Psi_B on the rest;
                                 2 the ratio Psi_E / Psi_B on transverse E only */
    int psi_deg;              /* polynomial degree of Psi (<= 8) */
    double psi_e[9], psi_b[9];/* power-series coefficients in s = sin^2(kz dz/2) */
    int nfilt;                /* number of 3-point passes per axis (<= 16) */
    double filt[16];          /* pass weights w of (w, 1-2w, w) */
    double jbg[3];            /* uniform background current (ion current) */
    double *E[3], *B[3], *J[3];
    double *Et[3], *Bt[3];    /* fields as seen by the particles */
    double *tmp, *tmp2;       /* scratch planes, ncell each */
    long np;
    double *x[3];             /* absolute positions (x[1] unused in 2D) */
    double *u[3];
    int status;               /* 1 if some particle moved a full cell or more */
} OSim;

static const int STAG_E[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
static const int STAG_B[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

static long ncell(const OSim *s) { return (long)s->nx * s->ny * s->nz; }

static long wrap(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

static long at(const OSim *s, long i, long j, long k)
{
    return (wrap(k, s->nz) * s->ny + wrap(j, s->ny)) * s->nx + wrap(i, s->nx);
}

/* ---------------------------------------------------------------- Yee ---- */

/* forward differences of plane F at (i, j, k) along x and along z */
static double fdx(const OSim *s, const double *F, long i, long j, long k)
{
    return (F[at(s, i + 1, j, k)] - F[at(s, i, j, k)]) / s->dx;
}

static double fdz(const OSim *s, const double *F, long i, long j, long k)
{
    return (F[at(s, i, j, k + 1)] - F[at(s, i, j, k)]) / s->dz;
}

/* Cole-Karkkainen half step of B in 2D (the paper uses it with beta = 1/8,
 * Secs. 2-3).  Reading: on square cells, each forward difference of E in
 * Faraday's law is replaced by the weighted mean, with weights (beta, 1 - 2 beta,
 * beta), of the same difference on the line itself and on its two neighbours
 * along the other in-plane axis; Ampere's law stays the Yee one.  Along a
 * mesh axis (transverse wave number zero) the operator is the Yee one. */
static void ck_b_half(OSim *s)
{
    const double h = 0.5 * s->dt, beta = 0.125, mid = 1.0 - 2.0 * beta;
    double *Ex = s->E[0], *Ey = s->E[1], *Ez = s->E[2];
    for (long k = 0; k < s->nz; k++)
        for (long i = 0; i < s->nx; i++) {
            long p = at(s, i, 0, k);
            double dzEy = mid * fdz(s, Ey, i, 0, k) + beta * (fdz(s, Ey, i - 1, 0, k) + fdz(s, Ey, i + 1, 0, k));
            double dzEx = mid * fdz(s, Ex, i, 0, k) + beta * (fdz(s, Ex, i - 1, 0, k) + fdz(s, Ex, i + 1, 0, k));
            double dxEz = mid * fdx(s, Ez, i, 0, k) + beta * (fdx(s, Ez, i, 0, k - 1) + fdx(s, Ez, i, 0, k + 1));
            double dxEy = mid * fdx(s, Ey, i, 0, k) + beta * (fdx(s, Ey, i, 0, k - 1) + fdx(s, Ey, i, 0, k + 1));
            s->B[0][p] -= h * (-dzEy);
            s->B[1][p] -= h * (dzEx - dxEz);
            s->B[2][p] -= h * dxEy;
        }
}

static void yee_b_half(OSim *s)
{
    if (s->solver == 1) {
        ck_b_half(s);
        return;
    }
    const double h = 0.5 * s->dt;
    double *Ex = s->E[0], *Ey = s->E[1], *Ez = s->E[2];
    for (long k = 0; k < s->nz; k++)
        for (long j = 0; j < s->ny; j++)
            for (long i = 0; i < s->nx; i++) {
                long p = at(s, i, j, k);
                double dyEz = (Ez[at(s, i, j + 1, k)] - Ez[p]) / s->dy;
                double dzEy = (Ey[at(s, i, j, k + 1)] - Ey[p]) / s->dz;
                double dzEx = (Ex[at(s, i, j, k + 1)] - Ex[p]) / s->dz;
                double dxEz = (Ez[at(s, i + 1, j, k)] - Ez[p]) / s->dx;
                double dxEy = (Ey[at(s, i + 1, j, k)] - Ey[p]) / s->dx;
                double dyEx = (Ex[at(s, i, j + 1, k)] - Ex[p]) / s->dy;
                s->B[0][p] -= h * (dyEz - dzEy);
                s->B[1][p] -= h * (dzEx - dxEz);
                s->B[2][p] -= h * (dxEy - dyEx);
            }
}

static void yee_e(OSim *s)
{
    const double dt = s->dt;
    double *Bx = s->B[0], *By = s->B[1], *Bz = s->B[2];
    for (long k = 0; k < s->nz; k++)
        for (long j = 0; j < s->ny; j++)
            for (long i = 0; i < s->nx; i++) {
                long p = at(s, i, j, k);
                double dyBz = (Bz[p] - Bz[at(s, i, j - 1, k)]) / s->dy;
                double dzBy = (By[p] - By[at(s, i, j, k - 1)]) / s->dz;
                double dzBx = (Bx[p] - Bx[at(s, i, j, k - 1)]) / s->dz;
                double dxBz = (Bz[p] - Bz[at(s, i - 1, j, k)]) / s->dx;
                double dxBy = (By[p] - By[at(s, i - 1, j, k)]) / s->dx;
                double dyBx = (Bx[p] - Bx[at(s, i, j - 1, k)]) / s->dy;
                s->E[0][p] += dt * (dyBz - dzBy - (s->J[0][p] + s->jbg[0]));
                s->E[1][p] += dt * (dzBx - dxBz - (s->J[1][p] + s->jbg[1]));
                s->E[2][p] += dt * (dxBy - dyBx - (s->J[2][p] + s->jbg[2]));
            }
}

void o_yee(OSim *s)
{
    yee_b_half(s);
    yee_e(s);
    yee_b_half(s);
}

/* ------------------------------------------- fields as seen (Sec. 2, 3) -- */

/* out = S_z in, S_z = -(1/4)(1,-2,1) along z, whose symbol is sin^2(kz dz/2) */
static void apply_sz(const OSim *s, const double *in, double *out)
{
    for (long k = 0; k < s->nz; k++)
        for (long j = 0; j < s->ny; j++)
            for (long i = 0; i < s->nx; i++) {
                long p = at(s, i, j, k);
                out[p] = -0.25 * (in[at(s, i, j, k - 1)] - 2.0 * in[p] + in[at(s, i, j, k + 1)]);
            }
}

/* one (w, 1-2w, w) pass along an axis (0 x, 1 y, 2 z) */
static void filter_pass(const OSim *s, int axis, double wt, const double *in, double *out)
{
    int ex = axis == 0, ey = axis == 1, ez = axis == 2;
    for (long k = 0; k < s->nz; k++)
        for (long j = 0; j < s->ny; j++)
            for (long i = 0; i < s->nx; i++) {
                long p = at(s, i, j, k);
                double lo = in[at(s, i - ex, j - ey, k - ez)];
                double hi = in[at(s, i + ex, j + ey, k + ez)];
                out[p] = wt * lo + (1.0 - 2.0 * wt) * in[p] + wt * hi;
            }
}

/* F <- Psi(S_z)^{-1} F along z.  Sec. 2 names this the inversion of the
 * denominator by tri-diagonal solves; written here as what it computes: for
 * every z column, the dense nz x nz matrix Psi(S_z) = sum_j c_j S_z^j (S_z the
 * periodic -(1/4)(1, -2, 1) matrix) is LU-factored with partial pivoting and
 * solved, which is exact up to rounding and obviously so. */
static void solve_psi_z(const OSim *s, const double *coef, double *F)
{
    const long n = s->nz;
    double *M = calloc((size_t)(n * n), sizeof(double));
    double *P = calloc((size_t)(n * n), sizeof(double));
    double *Q = calloc((size_t)(n * n), sizeof(double));
    double *col = malloc((size_t)n * sizeof(double));
    long *perm = malloc((size_t)n * sizeof(long));
    for (long r = 0; r < n; r++) {
        P[r * n + r] = 1.0;
        M[r * n + r] = coef[0];
    }
    for (int j = 1; j <= s->psi_deg; j++) {
        /* P <- S_z P, row r of S_z: -1/4 at r-1, 1/2 at r, -1/4 at r+1 (periodic) */
        for (long r = 0; r < n; r++)
            for (long c = 0; c < n; c++)
                Q[r * n + c] = -0.25 * P[wrap(r - 1, n) * n + c] + 0.5 * P[r * n + c] - 0.25 * P[wrap(r + 1, n) * n + c];
        memcpy(P, Q, (size_t)(n * n) * sizeof(double));
        for (long q = 0; q < n * n; q++) M[q] += coef[j] * P[q];
    }
    /* LU with partial pivoting, in place */
    for (long r = 0; r < n; r++) perm[r] = r;
    for (long c = 0; c < n; c++) {
        long piv = c;
        for (long r = c + 1; r < n; r++)
            if (fabs(M[r * n + c]) > fabs(M[piv * n + c])) piv = r;
        if (piv != c) {
            for (long q = 0; q < n; q++) {
                double t = M[c * n + q];
                M[c * n + q] = M[piv * n + q];
                M[piv * n + q] = t;
            }
            long t = perm[c];
            perm[c] = perm[piv];
            perm[piv] = t;
        }
        for (long r = c + 1; r < n; r++) {
            double f = M[r * n + c] / M[c * n + c];
            M[r * n + c] = f;
            for (long q = c + 1; q < n; q++) M[r * n + q] -= f * M[c * n + q];
        }
    }
    for (long j = 0; j < s->ny; j++)
        for (long i = 0; i < s->nx; i++) {
            for (long r = 0; r < n; r++) col[r] = F[at(s, i, j, perm[r])];
            for (long r = 0; r < n; r++)
                for (long q = 0; q < r; q++) col[r] -= M[r * n + q] * col[q];
            for (long r = n - 1; r >= 0; r--) {
                for (long q = r + 1; q < n; q++) col[r] -= M[r * n + q] * col[q];
                col[r] /= M[r * n + r];
            }
            for (long r = 0; r < n; r++) F[at(s, i, j, r)] = col[r];
        }
    free(M); free(P); free(Q); free(col); free(perm);
}

/* Psi(S_z) F = sum_j a_j S_z^j F, written as the power series (Sec. 2);
 * coef == NULL means the identity; with den, then Psi_den(S_z)^{-1} (the
 * ratio applied exactly).  Then the filter passes along z, x, y. */
static void seen_ratio(OSim *s, const double *coef, const double *den, const double *F, double *out)
{
    long nc = ncell(s);
    if (coef) {
        double *t = s->tmp, *t2 = s->tmp2;
        memcpy(t, F, nc * sizeof(double));
        for (long p = 0; p < nc; p++) out[p] = coef[0] * F[p];
        for (int j = 1; j <= s->psi_deg; j++) {
            apply_sz(s, t, t2);
            memcpy(t, t2, nc * sizeof(double));
            for (long p = 0; p < nc; p++) out[p] += coef[j] * t[p];
        }
    } else {
        memcpy(out, F, nc * sizeof(double));
    }
    if (den) solve_psi_z(s, den, out);
    static const int axes[3] = {2, 0, 1};
    for (int a = 0; a < 3; a++) {
        int axis = axes[a];
        if (axis == 1 && s->dims == 2) continue;
        for (int f = 0; f < s->nfilt; f++) {
            filter_pass(s, axis, s->filt[f], out, s->tmp);
            memcpy(out, s->tmp, nc * sizeof(double));
        }
    }
}

static void seen_one(OSim *s, const double *coef, const double *F, double *out)
{
    seen_ratio(s, coef, NULL, F, out);
}

/* Psi_E on both transverse E components; Psi_B on E_z and every B (Sec. 2).
 * correction 2: the full multiplier Psi_E / Psi_B on the transverse E
 * components only, the others filtered only (a variant Sec. 3 compares). */
void o_seen(OSim *s)
{
    if (s->correction == 2) {
        seen_ratio(s, s->psi_e, s->psi_b, s->E[0], s->Et[0]);
        seen_ratio(s, s->psi_e, s->psi_b, s->E[1], s->Et[1]);
        seen_one(s, NULL, s->E[2], s->Et[2]);
        for (int c = 0; c < 3; c++) seen_one(s, NULL, s->B[c], s->Bt[c]);
        return;
    }
    const double *pe = s->correction ? s->psi_e : NULL;
    const double *pb = s->correction ? s->psi_b : NULL;
    seen_one(s, pe, s->E[0], s->Et[0]);
    seen_one(s, pe, s->E[1], s->Et[1]);
    seen_one(s, pb, s->E[2], s->Et[2]);
    for (int c = 0; c < 3; c++) seen_one(s, pb, s->B[c], s->Bt[c]);
}

/* apply the seen-field operator with polynomial `which` (0 Psi_E, 1 Psi_B,
 * 2 identity, 3 the ratio Psi_E / Psi_B) to one plane; used by the
 * stencil-response tests */
void o_seen_plane(OSim *s, int which, const double *in, double *out)
{
    if (which == 3) {
        seen_ratio(s, s->psi_e, s->psi_b, in, out);
        return;
    }
    const double *coef = which == 0 ? s->psi_e : which == 1 ? s->psi_b : NULL;
    seen_one(s, coef, in, out);
}

/* -------------------------------------------------- B-spline shapes ------ */

/* centred B-spline of order o evaluated at t (cell units) */
double o_spline(int o, double t)
{
    double a = fabs(t);
    switch (o) {
    case 0:
        return (t >= -0.5 && t < 0.5) ? 1.0 : 0.0;
    case 1:
        return a < 1.0 ? 1.0 - a : 0.0;
    case 2:
        if (a < 0.5) return 0.75 - a * a;
        if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
        return 0.0;
    case 3:
        if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
        return 0.0;
    }
    return 0.0;
}

/* ------------------------------------------------------------ gather ----- */

/* value of plane F (staggering stag) on the Yee mesh, or, with avg, averaged
 * onto the integer node (i, j, k): the mean over the Yee locations half a cell
 * either side of the node along each staggered axis (y-invariant in 2D) */
static double node_value(const OSim *s, const double *F, const int *stag, int avg, long i, long j, long k)
{
    if (!avg) return F[at(s, i, j, k)];
    double sum = 0.0;
    int cnt = 0;
    for (long dk = -stag[2]; dk <= 0; dk++)
        for (long dj = s->dims == 3 ? -stag[1] : 0; dj <= 0; dj++)
            for (long di = -stag[0]; di <= 0; di++) {
                sum += F[at(s, i + di, j + dj, k + dk)];
                cnt++;
            }
    return sum / cnt;
}

/* interpolate plane F with per-axis orders ord[] at the point whose cell-unit
 * coordinates are c[] (c[1] ignored in 2D).  The samples sit at F's own Yee
 * locations (offsets stag[] / 2), or, with avg, at the integer nodes holding
 * node_value averages. */
static double interp(const OSim *s, const double *F, const int *stag, int avg, const int *ord, const double *c)
{
    long lo[3], hi[3];
    int pos[3];
    for (int a = 0; a < 3; a++) pos[a] = avg ? 0 : stag[a];
    for (int a = 0; a < 3; a++) {
        if (a == 1 && s->dims == 2) { lo[a] = hi[a] = 0; continue; }
        double shift = 0.5 * pos[a];
        double half = 0.5 * (ord[a] + 1);
        lo[a] = (long)floor(c[a] - shift - half);
        hi[a] = (long)floor(c[a] - shift + half);
    }
    double sum = 0.0;
    for (long k = lo[2]; k <= hi[2]; k++) {
        double wz = o_spline(ord[2], c[2] - k - 0.5 * pos[2]);
        if (wz == 0.0) continue;
        for (long j = lo[1]; j <= hi[1]; j++) {
            double wy = s->dims == 2 ? 1.0 : o_spline(ord[1], c[1] - j - 0.5 * pos[1]);
            if (wy == 0.0) continue;
            for (long i = lo[0]; i <= hi[0]; i++) {
                double wx = o_spline(ord[0], c[0] - i - 0.5 * pos[0]);
                if (wx == 0.0) continue;
                sum += wx * wy * wz * node_value(s, F, stag, avg, i, j, k);
            }
        }
    }
    return sum;
}

/* Galerkin: order l on axes where the component sits on integer nodes and
 * l-1 where it sits half a cell off (Eq. 3 scheme; Sec. 3 for E_z).
 * Uniform: order l on every axis from each component's own location (Eq. 4).
 * Momentum-conserving: the fields are first averaged from the Yee mesh to the
 * integer nodes, then interpolated with order l on every axis (Eq. 5). */
static void comp_orders(const OSim *s, const int *stag, int *ord)
{
    for (int a = 0; a < 3; a++) ord[a] = s->interp == 0 ? s->order - stag[a] : s->order;
}

void o_gather(const OSim *s, const double *pos, double *Eo, double *Bo)
{
    double c[3] = {pos[0] / s->dx, s->dims == 3 ? pos[1] / s->dy : 0.0, pos[2] / s->dz};
    const int avg = s->interp == 2;
    int ord[3];
    for (int comp = 0; comp < 3; comp++) {
        comp_orders(s, STAG_E[comp], ord);
        Eo[comp] = interp(s, s->Et[comp], STAG_E[comp], avg, ord, c);
        comp_orders(s, STAG_B[comp], ord);
        Bo[comp] = interp(s, s->Bt[comp], STAG_B[comp], avg, ord, c);
    }
}

/* ------------------------------------------------------------- Boris ----- */

void o_boris(double *u, const double *E, const double *B, double q, double m, double dt)
{
    double eps = q * dt / (2.0 * m);
    double um[3], t[3], sv[3], up[3], uq[3];
    for (int a = 0; a < 3; a++) um[a] = u[a] + eps * E[a];
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int a = 0; a < 3; a++) t[a] = eps * B[a] / gm;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int a = 0; a < 3; a++) sv[a] = 2.0 * t[a] / (1.0 + t2);
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    uq[0] = um[0] + (up[1] * sv[2] - up[2] * sv[1]);
    uq[1] = um[1] + (up[2] * sv[0] - up[0] * sv[2]);
    uq[2] = um[2] + (up[0] * sv[1] - up[1] * sv[0]);
    for (int a = 0; a < 3; a++) u[a] = uq[a] + eps * E[a];
}

/* ----------------------------------------------------- Esirkepov ------- */

#define MAXN 12

/* Add one particle's Esirkepov current for a move from p0 to p1 (absolute,
 * unwrapped: p1 = p0 + displacement).  vy is the y velocity used for J_y in
 * 2D3V.  Shapes are order-l B-splines on integer nodes. */
void o_deposit(OSim *s, const double *p0, const double *p1, double vy)
{
    const int l = s->order;
    const double d[3] = {s->dx, s->dy, s->dz};
    const double half = 0.5 * (l + 1);
    long lo[3] = {0, 0, 0};
    int cnt[3] = {1, 1, 1};
    double S0[3][MAXN], S1[3][MAXN], DS[3][MAXN];
    for (int a = 0; a < 3; a++) {
        if (a == 1 && s->dims == 2) { S0[a][0] = S1[a][0] = 1.0; DS[a][0] = 0.0; continue; }
        double c0 = p0[a] / d[a], c1 = p1[a] / d[a];
        double mn = c0 < c1 ? c0 : c1, mx = c0 < c1 ? c1 : c0;
        lo[a] = (long)floor(mn - half);
        long hi = (long)floor(mx + half);
        cnt[a] = (int)(hi - lo[a] + 1);
        for (int i = 0; i < cnt[a]; i++) {
            S0[a][i] = o_spline(l, c0 - (double)(lo[a] + i));
            S1[a][i] = o_spline(l, c1 - (double)(lo[a] + i));
            DS[a][i] = S1[a][i] - S0[a][i];
        }
    }
    const double qw = s->q * s->w;
    if (s->dims == 2) {
        const double dV = s->dx * s->dz;
        const double cx = -qw * s->dx / (s->dt * dV);
        const double cz = -qw * s->dz / (s->dt * dV);
        const double cy = qw * vy / dV;
        for (int k = 0; k < cnt[2]; k++) {          /* J_x: running sum along x */
            double acc = 0.0;
            for (int i = 0; i < cnt[0]; i++) {
                acc += DS[0][i] * (S0[2][k] + 0.5 * DS[2][k]);
                s->J[0][at(s, lo[0] + i, 0, lo[2] + k)] += cx * acc;
            }
        }
        for (int i = 0; i < cnt[0]; i++) {          /* J_z: running sum along z */
            double acc = 0.0;
            for (int k = 0; k < cnt[2]; k++) {
                acc += DS[2][k] * (S0[0][i] + 0.5 * DS[0][i]);
                s->J[2][at(s, lo[0] + i, 0, lo[2] + k)] += cz * acc;
            }
        }
        for (int k = 0; k < cnt[2]; k++)            /* J_y: out-of-plane */
            for (int i = 0; i < cnt[0]; i++) {
                double wy = S0[0][i] * S0[2][k] + 0.5 * DS[0][i] * S0[2][k]
                          + 0.5 * S0[0][i] * DS[2][k] + DS[0][i] * DS[2][k] / 3.0;
                s->J[1][at(s, lo[0] + i, 0, lo[2] + k)] += cy * wy;
            }
        return;
    }
    const double dV = s->dx * s->dy * s->dz;
    const double cf[3] = {-qw * s->dx / (s->dt * dV), -qw * s->dy / (s->dt * dV),
                          -qw * s->dz / (s->dt * dV)};
    /* W_a = DS_a * (S0_b S0_c + DS_b S0_c / 2 + S0_b DS_c / 2 + DS_b DS_c / 3) */
    for (int a = 0; a < 3; a++) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        int idx[3];
        for (idx[b] = 0; idx[b] < cnt[b]; idx[b]++)
            for (idx[c] = 0; idx[c] < cnt[c]; idx[c]++) {
                double sb0 = S0[b][idx[b]], dsb = DS[b][idx[b]];
                double sc0 = S0[c][idx[c]], dsc = DS[c][idx[c]];
                double tr = sb0 * sc0 + 0.5 * dsb * sc0 + 0.5 * sb0 * dsc + dsb * dsc / 3.0;
                double acc = 0.0;
                for (idx[a] = 0; idx[a] < cnt[a]; idx[a]++) {
                    acc += DS[a][idx[a]] * tr;
                    s->J[a][at(s, lo[0] + idx[0], lo[1] + idx[1], lo[2] + idx[2])] += cf[a] * acc;
                }
            }
    }
}

/* ------------------------------------------------------------ step ------ */

static double wrap_pos(double x, double L)
{
    if (x >= L) x -= L;
    if (x < 0.0) {
        x += L;
        if (x >= L) x -= L;
    }
    return x;
}

void o_push_deposit(OSim *s)
{
    long nc = ncell(s);
    for (int c = 0; c < 3; c++) memset(s->J[c], 0, nc * sizeof(double));
    const double L[3] = {s->nx * s->dx, s->ny * s->dy, s->nz * s->dz};
    const double d[3] = {s->dx, s->dy, s->dz};
    for (long p = 0; p < s->np; p++) {
        double p0[3] = {s->x[0][p], s->dims == 3 ? s->x[1][p] : 0.0, s->x[2][p]};
        double E[3], B[3];
        o_gather(s, p0, E, B);
        double u[3] = {s->u[0][p], s->u[1][p], s->u[2][p]};
        o_boris(u, E, B, s->q, s->m, s->dt);
        double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double p1[3];
        for (int a = 0; a < 3; a++) {
            if (a == 1 && s->dims == 2) { p1[a] = 0.0; continue; }
            p1[a] = p0[a] + s->dt * u[a] / g;
            if (fabs(p1[a] - p0[a]) >= d[a]) s->status = 1;
        }
        o_deposit(s, p0, p1, u[1] / g);
        for (int a = 0; a < 3; a++) {
            s->u[a][p] = u[a];
            if (a == 1 && s->dims == 2) continue;
            s->x[a][p] = wrap_pos(p1[a], L[a]);
        }
    }
}

void o_step(OSim *s, int nsteps)
{
    for (int n = 0; n < nsteps; n++) {
        o_yee(s);
        o_seen(s);
        o_push_deposit(s);
    }
}

/* ------------------------------------------------------- diagnostics ---- */

/* charge density on integer nodes with the order-l shape */
void o_rho(const OSim *s, double *rho)
{
    long nc = ncell(s);
    memset(rho, 0, nc * sizeof(double));
    const double dV = s->dims == 2 ? s->dx * s->dz : s->dx * s->dy * s->dz;
    static const int zero[3] = {0, 0, 0};
    int ord[3] = {s->order, s->order, s->order};
    for (long p = 0; p < s->np; p++) {
        double c[3] = {s->x[0][p] / s->dx, s->dims == 3 ? s->x[1][p] / s->dy : 0.0, s->x[2][p] / s->dz};
        long lo[3], hi[3];
        for (int a = 0; a < 3; a++) {
            if (a == 1 && s->dims == 2) { lo[a] = hi[a] = 0; continue; }
            lo[a] = (long)floor(c[a] - 0.5 * (ord[a] + 1));
            hi[a] = (long)floor(c[a] + 0.5 * (ord[a] + 1));
        }
        for (long k = lo[2]; k <= hi[2]; k++)
            for (long j = lo[1]; j <= hi[1]; j++)
                for (long i = lo[0]; i <= hi[0]; i++) {
                    double wgt = o_spline(ord[0], c[0] - i - 0.5 * zero[0]) *
                                 (s->dims == 2 ? 1.0 : o_spline(ord[1], c[1] - j)) *
                                 o_spline(ord[2], c[2] - k);
                    rho[at(s, i, j, k)] += s->q * s->w * wgt / dV;
                }
    }
}

/* discrete divergence of a field with E's staggering, at integer nodes */
void o_div(const OSim *s, double *const F[3], double *out)
{
    for (long k = 0; k < s->nz; k++)
        for (long j = 0; j < s->ny; j++)
            for (long i = 0; i < s->nx; i++) {
                long p = at(s, i, j, k);
                double v = (F[0][p] - F[0][at(s, i - 1, j, k)]) / s->dx
                         + (F[2][p] - F[2][at(s, i, j, k - 1)]) / s->dz;
                if (s->dims == 3) v += (F[1][p] - F[1][at(s, i, j - 1, k)]) / s->dy;
                out[p] = v;
            }
}

/* ================================================================ adjoint
 *
 * Reverse mode of one oracle step, with exact transposes.  The step maps
 * (E, B, J, x, u) to (E1, B2, J', x', u') through
 *   B1 = B - h Cf E,  E1 = E + dt (Cb B1 - J - Jbg),  B2 = B1 - h Cf E1   (h = dt/2)
 *   Et = M_E E1, Bt = M_B B2           (Psi series then filter passes; symmetric)
 *   per particle: gather at x, Boris, x' = x + dt u'/gamma', Esirkepov J'
 * with Cb = Cf^T on the periodic mesh.  Given the adjoints of the outputs,
 * o_adj_step overwrites them with the adjoints of the inputs and adds
 * dL/da_j = sum_{c in x,y} <lambda_Et_c, F S_z^j E1_c> to grad[j].
 * The tape of the step is E1, B2 (after its Yee update) and the particle
 * state x, u before its push.
 */

double o_dspline(int o, double t)
{
    double a = fabs(t), sg = t < 0.0 ? -1.0 : 1.0;
    switch (o) {
    case 0:
        return 0.0;
    case 1:
        return a < 1.0 ? -sg : 0.0;
    case 2:
        if (a < 0.5) return -2.0 * t;
        if (a < 1.5) return -sg * (1.5 - a);
        return 0.0;
    case 3:
        if (a < 1.0) return -2.0 * t + 1.5 * t * a;
        if (a < 2.0) return -0.5 * sg * (2.0 - a) * (2.0 - a);
        return 0.0;
    }
    return 0.0;
}

/* out = Cf F (forward-difference curl, E locations -> B locations) */
static void curl_f(const OSim *s, double *const F[3], double *out[3])
{
    for (long k = 0; k < s->nz; k++)
        for (long j = 0; j < s->ny; j++)
            for (long i = 0; i < s->nx; i++) {
                long p = at(s, i, j, k);
                double dyFz = (F[2][at(s, i, j + 1, k)] - F[2][p]) / s->dy;
                double dzFy = (F[1][at(s, i, j, k + 1)] - F[1][p]) / s->dz;
                double dzFx = (F[0][at(s, i, j, k + 1)] - F[0][p]) / s->dz;
                double dxFz = (F[2][at(s, i + 1, j, k)] - F[2][p]) / s->dx;
                double dxFy = (F[1][at(s, i + 1, j, k)] - F[1][p]) / s->dx;
                double dyFx = (F[0][at(s, i, j + 1, k)] - F[0][p]) / s->dy;
                out[0][p] = dyFz - dzFy;
                out[1][p] = dzFx - dxFz;
                out[2][p] = dxFy - dyFx;
            }
}

/* out = Cb F (backward-difference curl, B locations -> E locations) */
static void curl_b(const OSim *s, double *const F[3], double *out[3])
{
    for (long k = 0; k < s->nz; k++)
        for (long j = 0; j < s->ny; j++)
            for (long i = 0; i < s->nx; i++) {
                long p = at(s, i, j, k);
                double dyFz = (F[2][p] - F[2][at(s, i, j - 1, k)]) / s->dy;
                double dzFy = (F[1][p] - F[1][at(s, i, j, k - 1)]) / s->dz;
                double dzFx = (F[0][p] - F[0][at(s, i, j, k - 1)]) / s->dz;
                double dxFz = (F[2][p] - F[2][at(s, i - 1, j, k)]) / s->dx;
                double dxFy = (F[1][p] - F[1][at(s, i - 1, j, k)]) / s->dx;
                double dyFx = (F[0][p] - F[0][at(s, i, j - 1, k)]) / s->dy;
                out[0][p] = dyFz - dzFy;
                out[1][p] = dzFx - dxFz;
                out[2][p] = dxFy - dyFx;
            }
}

/* transpose of Faraday's curl: the backward-difference curl for Yee; for the
 * Cole-Karkkainen solver every backward difference is averaged across its
 * direction with (beta, 1 - 2 beta, beta) (the transpose of an average of
 * forward differences, the average being symmetric) */
static void curl_faraday_t(const OSim *s, double *const F[3], double *out[3])
{
    if (s->solver != 1) {
        curl_b(s, F, out);
        return;
    }
    const double beta = 0.125, mid = 1.0 - 2.0 * beta;
    for (long k = 0; k < s->nz; k++)
        for (long i = 0; i < s->nx; i++) {
            long p = at(s, i, 0, k);
            double dz[2], dx[2];
            for (int c = 0; c < 2; c++) {
                const double *G = c == 0 ? F[1] : F[0];   /* dz of Fy, dz of Fx */
                double m0 = (G[at(s, i, 0, k)] - G[at(s, i, 0, k - 1)]) / s->dz;
                double mm = (G[at(s, i - 1, 0, k)] - G[at(s, i - 1, 0, k - 1)]) / s->dz;
                double mp = (G[at(s, i + 1, 0, k)] - G[at(s, i + 1, 0, k - 1)]) / s->dz;
                dz[c] = mid * m0 + beta * (mm + mp);
            }
            for (int c = 0; c < 2; c++) {
                const double *G = c == 0 ? F[2] : F[1];   /* dx of Fz, dx of Fy */
                double m0 = (G[at(s, i, 0, k)] - G[at(s, i - 1, 0, k)]) / s->dx;
                double mm = (G[at(s, i, 0, k - 1)] - G[at(s, i - 1, 0, k - 1)]) / s->dx;
                double mp = (G[at(s, i, 0, k + 1)] - G[at(s, i - 1, 0, k + 1)]) / s->dx;
                dx[c] = mid * m0 + beta * (mm + mp);
            }
            out[0][p] = -dz[0];
            out[1][p] = dz[1] - dx[0];
            out[2][p] = dx[1];
        }
}

/* adjoint of the gather of one component: scatter w * lv into lF and add
 * d(value)/d(position) * lv to lpos (physical units) */
static void interp_adj(const OSim *s, const double *F, double *lF, const int *stag, const int *ord,
                       const double *c, double lv, double *lpos)
{
    long lo[3], hi[3];
    const double d[3] = {s->dx, s->dy, s->dz};
    for (int a = 0; a < 3; a++) {
        if (a == 1 && s->dims == 2) { lo[a] = hi[a] = 0; continue; }
        double shift = 0.5 * stag[a];
        double half = 0.5 * (ord[a] + 1);
        lo[a] = (long)floor(c[a] - shift - half);
        hi[a] = (long)floor(c[a] - shift + half);
    }
    for (long k = lo[2]; k <= hi[2]; k++) {
        double tz = c[2] - k - 0.5 * stag[2];
        double wz = o_spline(ord[2], tz), dwz = o_dspline(ord[2], tz);
        for (long j = lo[1]; j <= hi[1]; j++) {
            double ty = c[1] - j - 0.5 * stag[1];
            double wy = s->dims == 2 ? 1.0 : o_spline(ord[1], ty);
            double dwy = s->dims == 2 ? 0.0 : o_dspline(ord[1], ty);
            for (long i = lo[0]; i <= hi[0]; i++) {
                double tx = c[0] - i - 0.5 * stag[0];
                double wx = o_spline(ord[0], tx), dwx = o_dspline(ord[0], tx);
                long p = at(s, i, j, k);
                lF[p] += wx * wy * wz * lv;
                double fv = F[p] * lv;
                lpos[0] += dwx * wy * wz * fv / d[0];
                if (s->dims == 3) lpos[1] += wx * dwy * wz * fv / d[1];
                lpos[2] += wx * wy * dwz * fv / d[2];
            }
        }
    }
}

/* reverse of the Boris push: given lun = dL/du_new, return lu (= dL/du_old),
 * and add to lE, lB */
void o_boris_adj(const double *u, const double *E, const double *B, double q, double m, double dt,
                 const double *lun, double *lu, double *lE, double *lB)
{
    double eps = q * dt / (2.0 * m);
    double um[3], t[3], sv[3], up[3];
    for (int a = 0; a < 3; a++) um[a] = u[a] + eps * E[a];
    double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int a = 0; a < 3; a++) t[a] = eps * B[a] / g;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double f = 2.0 / (1.0 + t2);
    for (int a = 0; a < 3; a++) sv[a] = f * t[a];
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    /* un = uq + eps E;  uq = um + up x s */
    double luq[3], lum[3], lup[3], ls[3], lt[3];
    for (int a = 0; a < 3; a++) { luq[a] = lun[a]; lE[a] += eps * lun[a]; lum[a] = luq[a]; }
    /* d(up x s): lup = s x luq ; ls = luq x up */
    lup[0] = sv[1] * luq[2] - sv[2] * luq[1];
    lup[1] = sv[2] * luq[0] - sv[0] * luq[2];
    lup[2] = sv[0] * luq[1] - sv[1] * luq[0];
    ls[0] = luq[1] * up[2] - luq[2] * up[1];
    ls[1] = luq[2] * up[0] - luq[0] * up[2];
    ls[2] = luq[0] * up[1] - luq[1] * up[0];
    /* up = um + um x t: lum += lup + t x lup ; lt = lup x um */
    lum[0] += lup[0] + (t[1] * lup[2] - t[2] * lup[1]);
    lum[1] += lup[1] + (t[2] * lup[0] - t[0] * lup[2]);
    lum[2] += lup[2] + (t[0] * lup[1] - t[1] * lup[0]);
    lt[0] = lup[1] * um[2] - lup[2] * um[1];
    lt[1] = lup[2] * um[0] - lup[0] * um[2];
    lt[2] = lup[0] * um[1] - lup[1] * um[0];
    /* s = f t, f = 2 / (1 + t.t) */
    double lf = ls[0] * t[0] + ls[1] * t[1] + ls[2] * t[2];
    double lt2 = -lf * f * f / 2.0;
    for (int a = 0; a < 3; a++) lt[a] += f * ls[a] + 2.0 * t[a] * lt2;
    /* t = eps B / g */
    double lg = -(t[0] * lt[0] + t[1] * lt[1] + t[2] * lt[2]) / g;
    for (int a = 0; a < 3; a++) lB[a] += eps * lt[a] / g;
    /* g = sqrt(1 + um.um) */
    for (int a = 0; a < 3; a++) lum[a] += lg * um[a] / g;
    /* um = u + eps E */
    for (int a = 0; a < 3; a++) { lu[a] = lum[a]; lE[a] += eps * lum[a]; }
}

/* reverse of o_deposit: given lJ on the grid, add dL/dp0, dL/dp1 (physical
 * units) and return dL/dvy (2D J_y) */
double o_deposit_adj(const OSim *s, const double *p0, const double *p1, double vy, double *const lJ[3],
                     double *lp0, double *lp1)
{
    const int l = s->order;
    const double d[3] = {s->dx, s->dy, s->dz};
    const double half = 0.5 * (l + 1);
    long lo[3] = {0, 0, 0};
    int cnt[3] = {1, 1, 1};
    double S0[3][MAXN], S1[3][MAXN], DS[3][MAXN], D0[3][MAXN], D1[3][MAXN];
    double L0[3][MAXN], L1[3][MAXN];  /* dL/dS0, dL/dS1 */
    double c0[3], c1[3];
    for (int a = 0; a < 3; a++) {
        for (int i = 0; i < MAXN; i++) L0[a][i] = L1[a][i] = 0.0;
        if (a == 1 && s->dims == 2) { S0[a][0] = S1[a][0] = 1.0; DS[a][0] = 0.0; continue; }
        c0[a] = p0[a] / d[a];
        c1[a] = p1[a] / d[a];
        double mn = c0[a] < c1[a] ? c0[a] : c1[a], mx = c0[a] < c1[a] ? c1[a] : c0[a];
        lo[a] = (long)floor(mn - half);
        long hi = (long)floor(mx + half);
        cnt[a] = (int)(hi - lo[a] + 1);
        for (int i = 0; i < cnt[a]; i++) {
            double t0 = c0[a] - (double)(lo[a] + i), t1 = c1[a] - (double)(lo[a] + i);
            S0[a][i] = o_spline(l, t0);
            S1[a][i] = o_spline(l, t1);
            D0[a][i] = o_dspline(l, t0);
            D1[a][i] = o_dspline(l, t1);
            DS[a][i] = S1[a][i] - S0[a][i];
        }
    }
    const double qw = s->q * s->w;
    double lvy = 0.0;
    if (s->dims == 2) {
        const double dV = s->dx * s->dz;
        const double cx = -qw * s->dx / (s->dt * dV);
        const double cz = -qw * s->dz / (s->dt * dV);
        const double cy = qw * vy / dV;
        /* J_x(i) = cx sum_{i'<=i} Wx(i'), Wx(i,k) = DSx(i) (S0z(k) + DSz(k)/2) */
        for (int k = 0; k < cnt[2]; k++) {
            double acc = 0.0;
            for (int i = cnt[0] - 1; i >= 0; i--) {
                acc += cx * lJ[0][at(s, lo[0] + i, 0, lo[2] + k)];   /* lWx(i,k) */
                double az = 0.5 * (S0[2][k] + S1[2][k]);
                L1[0][i] += acc * az;
                L0[0][i] -= acc * az;
                L0[2][k] += acc * 0.5 * DS[0][i];
                L1[2][k] += acc * 0.5 * DS[0][i];
            }
        }
        for (int i = 0; i < cnt[0]; i++) {
            double acc = 0.0;
            for (int k = cnt[2] - 1; k >= 0; k--) {
                acc += cz * lJ[2][at(s, lo[0] + i, 0, lo[2] + k)];   /* lWz(i,k) */
                double ax = 0.5 * (S0[0][i] + S1[0][i]);
                L1[2][k] += acc * ax;
                L0[2][k] -= acc * ax;
                L0[0][i] += acc * 0.5 * DS[2][k];
                L1[0][i] += acc * 0.5 * DS[2][k];
            }
        }
        for (int k = 0; k < cnt[2]; k++)
            for (int i = 0; i < cnt[0]; i++) {
                double lj = lJ[1][at(s, lo[0] + i, 0, lo[2] + k)];
                double wy = S0[0][i] * S0[2][k] / 3.0 + S1[0][i] * S0[2][k] / 6.0 + S0[0][i] * S1[2][k] / 6.0
                          + S1[0][i] * S1[2][k] / 3.0;
                lvy += qw / dV * wy * lj;
                double lw = cy * lj;
                L0[0][i] += lw * (S0[2][k] / 3.0 + S1[2][k] / 6.0);
                L1[0][i] += lw * (S0[2][k] / 6.0 + S1[2][k] / 3.0);
                L0[2][k] += lw * (S0[0][i] / 3.0 + S1[0][i] / 6.0);
                L1[2][k] += lw * (S0[0][i] / 6.0 + S1[0][i] / 3.0);
            }
    } else {
        const double dV = s->dx * s->dy * s->dz;
        for (int a = 0; a < 3; a++) {
            const double cf = -qw * d[a] / (s->dt * dV);
            int b = (a + 1) % 3, c = (a + 2) % 3;
            int idx[3];
            for (idx[b] = 0; idx[b] < cnt[b]; idx[b]++)
                for (idx[c] = 0; idx[c] < cnt[c]; idx[c]++) {
                    const int ib = idx[b], ic = idx[c];
                    /* tr = S0b S0c/3 + S1b S0c/6 + S0b S1c/6 + S1b S1c/3 */
                    double tr = S0[b][ib] * S0[c][ic] / 3.0 + S1[b][ib] * S0[c][ic] / 6.0
                              + S0[b][ib] * S1[c][ic] / 6.0 + S1[b][ib] * S1[c][ic] / 3.0;
                    double acc = 0.0, ltr = 0.0;
                    for (idx[a] = cnt[a] - 1; idx[a] >= 0; idx[a]--) {
                        acc += cf * lJ[a][at(s, lo[0] + idx[0], lo[1] + idx[1], lo[2] + idx[2])];
                        L1[a][idx[a]] += acc * tr;
                        L0[a][idx[a]] -= acc * tr;
                        ltr += acc * DS[a][idx[a]];
                    }
                    L0[b][ib] += ltr * (S0[c][ic] / 3.0 + S1[c][ic] / 6.0);
                    L1[b][ib] += ltr * (S0[c][ic] / 6.0 + S1[c][ic] / 3.0);
                    L0[c][ic] += ltr * (S0[b][ib] / 3.0 + S1[b][ib] / 6.0);
                    L1[c][ic] += ltr * (S0[b][ib] / 6.0 + S1[b][ib] / 3.0);
                }
        }
    }
    for (int a = 0; a < 3; a++) {
        if (a == 1 && s->dims == 2) continue;
        for (int i = 0; i < cnt[a]; i++) {
            lp0[a] += L0[a][i] * D0[a][i] / d[a];
            lp1[a] += L1[a][i] * D1[a][i] / d[a];
        }
    }
    return lvy;
}

void o_adj_step(OSim *s, double *const E1[3], double *const B2[3], double *const x0[3], double *const u0[3],
                double *lE[3], double *lB[3], double *lJ[3], double *lx[3], double *lu[3],
                double *lEt[3], double *lBt[3], double *grad)
{
    const long nc = ncell(s);
    const double h = 0.5 * s->dt;
    /* recompute the seen fields of this step */
    for (int c = 0; c < 3; c++) {
        memcpy(s->E[c], E1[c], nc * sizeof(double));
        memcpy(s->B[c], B2[c], nc * sizeof(double));
        memset(lEt[c], 0, nc * sizeof(double));
        memset(lBt[c], 0, nc * sizeof(double));
    }
    o_seen(s);
    /* particles */
    int ord[3];
    const double d[3] = {s->dx, s->dy, s->dz};
    for (long p = 0; p < s->np; p++) {
        double p0[3] = {x0[0][p], s->dims == 3 ? x0[1][p] : 0.0, x0[2][p]};
        double E[3], B[3];
        o_gather(s, p0, E, B);
        double u[3] = {u0[0][p], u0[1][p], u0[2][p]};
        double un[3] = {u[0], u[1], u[2]};
        o_boris(un, E, B, s->q, s->m, s->dt);
        double g = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
        double p1[3];
        for (int a = 0; a < 3; a++) p1[a] = (a == 1 && s->dims == 2) ? 0.0 : p0[a] + s->dt * un[a] / g;
        double lp0[3] = {0, 0, 0}, lp1[3] = {lx[0][p], s->dims == 3 ? lx[1][p] : 0.0, lx[2][p]};
        double lvy = o_deposit_adj(s, p0, p1, un[1] / g, lJ, lp0, lp1);
        /* move: p1 = p0 + dt v(un);  J_y used vy = un_y / g */
        double lv[3] = {0, 0, 0};
        for (int a = 0; a < 3; a++) {
            if (a == 1 && s->dims == 2) continue;
            lp0[a] += lp1[a];
            lv[a] += s->dt * lp1[a];
        }
        if (s->dims == 2) lv[1] += lvy;
        double un_dot_lv = un[0] * lv[0] + un[1] * lv[1] + un[2] * lv[2];
        double lun[3];
        for (int a = 0; a < 3; a++) lun[a] = lu[a][p] + lv[a] / g - un[a] * un_dot_lv / (g * g * g);
        double luo[3], lEp[3] = {0, 0, 0}, lBp[3] = {0, 0, 0};
        o_boris_adj(u, E, B, s->q, s->m, s->dt, lun, luo, lEp, lBp);
        /* gather */
        double c[3] = {p0[0] / d[0], s->dims == 3 ? p0[1] / d[1] : 0.0, p0[2] / d[2]};
        for (int comp = 0; comp < 3; comp++) {
            comp_orders(s, STAG_E[comp], ord);
            interp_adj(s, s->Et[comp], lEt[comp], STAG_E[comp], ord, c, lEp[comp], lp0);
            comp_orders(s, STAG_B[comp], ord);
            interp_adj(s, s->Bt[comp], lBt[comp], STAG_B[comp], ord, c, lBp[comp], lp0);
        }
        for (int a = 0; a < 3; a++) {
            lu[a][p] = luo[a];
            if (a == 1 && s->dims == 2) continue;
            lx[a][p] = lp0[a];
        }
    }
    /* seen fields: lE1 += M_E lEt, lB2 += M_B lBt; gradient of the Psi_E coefficients */
    const double *pe = s->correction ? s->psi_e : NULL;
    const double *pb = s->correction ? s->psi_b : NULL;
    double *t = s->tmp, *t2 = s->tmp2;
    double *buf = s->Et[0];   /* the recomputed seen fields are no longer needed */
    for (int c = 0; c < 3; c++) {
        seen_one(s, c < 2 ? pe : pb, lEt[c], buf);
        for (long q = 0; q < nc; q++) lE[c][q] += buf[q];
        seen_one(s, pb, lBt[c], buf);
        for (long q = 0; q < nc; q++) lB[c][q] += buf[q];
    }
    if (s->correction && grad) {
        for (int c = 0; c < 2; c++) {
            /* F lEt (filter only), then S_z^j, dotted with E1 */
            seen_one(s, NULL, lEt[c], buf);
            memcpy(t, buf, nc * sizeof(double));
            for (int j = 0; j <= s->psi_deg; j++) {
                if (j > 0) {
                    apply_sz(s, t, t2);
                    memcpy(t, t2, nc * sizeof(double));
                }
                double acc = 0.0;
                for (long q = 0; q < nc; q++) acc += t[q] * E1[c][q];
                grad[j] += acc;
            }
        }
    }
    /* Yee reverse */
    double *w0 = s->Et[0], *w1 = s->Et[1], *w2 = s->Et[2];
    double *cw[3] = {w0, w1, w2};
    /* B2 = B1 - h Cf E1  ->  lB1 = lB2 ;  lE1 -= h Cf^T lB2 (Cf^T = Cb for Yee) */
    curl_faraday_t(s, lB, cw);
    for (int c = 0; c < 3; c++)
        for (long q = 0; q < nc; q++) lE[c][q] -= h * cw[c][q];
    /* E1 = E + dt (Cb B1 - J) -> lB1 += dt Cf lE1 ; lJ = -dt lE1 ; lE = lE1 */
    curl_f(s, lE, cw);
    for (int c = 0; c < 3; c++)
        for (long q = 0; q < nc; q++) {
            lB[c][q] += s->dt * cw[c][q];
            lJ[c][q] = -s->dt * lE[c][q];
        }
    /* B1 = B - h Cf E -> lB = lB1 ; lE -= h Cf^T lB1 */
    curl_faraday_t(s, lB, cw);
    for (int c = 0; c < 3; c++)
        for (long q = 0; q < nc; q++) lE[c][q] -= h * cw[c][q];
}
