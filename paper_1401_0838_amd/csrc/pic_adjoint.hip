// Reverse-mode (adjoint) kernels of the PIC step, for gradients of the
// late-time transverse field energy with respect to the Psi_E coefficients
// (Sec. 2 defines Psi_E; its coefficients are what gets tuned).
//
// The forward step maps (E, B, J, particles) through
//   Yee:  B1 = B - h Cf E,  E1 = E + dt (Cb B1 - J - J_bg),  B2 = B1 - h Cf E1
//   seen: Et = M_E E1, Bt = M_B B2   (Psi(S_z) composed with the filter; symmetric)
//   particles: gather at x, Boris, move, Esirkepov deposit of J'
// and, on the periodic Yee mesh, Cb = Cf^T.  Each kernel below is the exact
// transpose of its forward counterpart:
//   k_adj_particles  per tile: recompute the particle's forward step, then the
//                    reverse of deposit, move, Boris and gather; the adjoint
//                    of the seen fields is scattered into an LDS window
//   k_adj_seen_2d    2D: the transposed seen-field stencils in LDS, fused with
//                    dW/da_j += <S_z^j F lambda_Et_c, E1_c>, c in {x, y}
//   k_adj_yee_2d     2D: the three transposed Yee sweeps in one LDS pass
//   k_pass, k_adj_grad, k_adj_yee_e/_b   the same in 3D as per-cell passes
// Positions and their adjoints are in cell units (offsets).
#include <hip/hip_runtime.h>

#include "pic_device.h"
#include "pic_internal.h"

namespace {

using namespace pic;

// byte offset of the double accumulation planes after 9 planes of R
__host__ __device__ inline size_t adj_lf_offset(size_t wc, size_t rsize) { return (9 * wc * rsize + 7) & ~(size_t)7; }

// derivatives of the Shape weights with respect to the in-cell offset
// Blocks add their gradient partial sums to one of PIC_GRAD_COPIES copies of
// the gradient (by block index), so that a few blocks, not all, meet at each
// address; the host sums the copies.
__device__ __forceinline__ int grad_copy() { return 16 * (int)(blockIdx.x & (PIC_GRAD_COPIES - 1)); }

template <int L, class R> struct DShape;

template <class R> struct DShape<1, R> {
    static __device__ __forceinline__ void integer(R, R *w) { w[0] = R(-1); w[1] = R(1); }
    static __device__ __forceinline__ void half(R, R *w) { w[0] = R(0); }
};

template <class R> struct DShape<3, R> {
    static __device__ __forceinline__ void integer(R d, R *w)
    {
        R e = R(1) - d;
        w[0] = R(-0.5) * e * e;
        w[1] = R(-2) * d + R(1.5) * d * d;
        w[2] = R(2) * e - R(1.5) * e * e;
        w[3] = R(0.5) * d * d;
    }
    static __device__ __forceinline__ void half(R d, R *w)
    {
        w[0] = -(R(1) - d);
        w[1] = R(-2) * (d - R(0.5));
        w[2] = d;
    }
};

__device__ __forceinline__ void gadd(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void gadd(double *p, double v) { unsafeAtomicAdd(p, v); }

// window of seen fields (read), adjoint current (read) and adjoint seen fields
// (accumulate).  The accumulation is in double whatever R is: LDS atomic adds
// of doubles run at several times the rate of float ones on this chip.
template <class R> struct AdjLds {
    const R *F;    // 6 planes
    const R *LJ;   // 3 planes
    double *LF;    // 6 planes
    int wx, wxy, wc;
    __device__ __forceinline__ int at(int x, int y, int z) const { return z * wxy + y * wx + x; }
    __device__ __forceinline__ R f(int c, int x, int y, int z) const { return F[c * wc + at(x, y, z)]; }
    __device__ __forceinline__ R lj(int c, int x, int y, int z) const { return LJ[c * wc + at(x, y, z)]; }
    __device__ __forceinline__ void addf(int c, int x, int y, int z, R v)
    {
        unsafeAtomicAdd(&LF[c * wc + at(x, y, z)], (double)v);
    }
};

template <class R> struct AdjGlb {
    const R *F[6];
    const R *LJ[3];
    R *LF[6];
    int o[3], n[3];
    __device__ __forceinline__ int at(int x, int y, int z) const
    {
        int gx = (o[0] + x) % n[0], gy = (o[1] + y) % n[1], gz = (o[2] + z) % n[2];
        return (gz * n[1] + gy) * n[0] + gx;
    }
    __device__ __forceinline__ R f(int c, int x, int y, int z) const { return F[c][at(x, y, z)]; }
    __device__ __forceinline__ R lj(int c, int x, int y, int z) const { return LJ[c][at(x, y, z)]; }
    __device__ __forceinline__ void addf(int c, int x, int y, int z, R v) { gadd(&LF[c][at(x, y, z)], v); }
};

template <int SX, int SY, int SZ, int DIM, int L, class R, class Win>
__device__ __forceinline__ R interp_f(const Win &W, int comp, const int *lc, const R (*wi)[L + 1], const R (*wh)[L])
{
    constexpr int H = (L - 1) / 2;
    constexpr int NX = L + 1 - SX, NZ = L + 1 - SZ, NY = DIM == 3 ? L + 1 - SY : 1;
    R s = R(0);
#pragma unroll
    for (int kz = 0; kz < NZ; kz++) {
        R wz;
        if constexpr (SZ) wz = wh[2][kz]; else wz = wi[2][kz];
#pragma unroll
        for (int ky = 0; ky < NY; ky++) {
            R wy = R(1);
            if constexpr (DIM == 3) { if constexpr (SY) wy = wh[1][ky]; else wy = wi[1][ky]; }
            R row = R(0);
#pragma unroll
            for (int kx = 0; kx < NX; kx++) {
                R wx;
                if constexpr (SX) wx = wh[0][kx]; else wx = wi[0][kx];
                row += wx * W.f(comp, lc[0] - H + kx, DIM == 3 ? lc[1] - H + ky : 0, lc[2] - H + kz);
            }
            s += wy * wz * row;
        }
    }
    return s;
}

// adjoint of one gathered component: scatter w * lv, accumulate d/doffset
template <int SX, int SY, int SZ, int DIM, int L, class R, class Win>
__device__ __forceinline__ void interp_adj(Win &W, int comp, const int *lc, const R (*wi)[L + 1], const R (*wh)[L],
                                           const R (*dwi)[L + 1], const R (*dwh)[L], R lv, R *lo)
{
    constexpr int H = (L - 1) / 2;
    constexpr int NX = L + 1 - SX, NZ = L + 1 - SZ, NY = DIM == 3 ? L + 1 - SY : 1;
#pragma unroll
    for (int kz = 0; kz < NZ; kz++) {
        R wz, dwz;
        if constexpr (SZ) { wz = wh[2][kz]; dwz = dwh[2][kz]; } else { wz = wi[2][kz]; dwz = dwi[2][kz]; }
#pragma unroll
        for (int ky = 0; ky < NY; ky++) {
            R wy = R(1), dwy = R(0);
            if constexpr (DIM == 3) {
                if constexpr (SY) { wy = wh[1][ky]; dwy = dwh[1][ky]; } else { wy = wi[1][ky]; dwy = dwi[1][ky]; }
            }
#pragma unroll
            for (int kx = 0; kx < NX; kx++) {
                R wx, dwx;
                if constexpr (SX) { wx = wh[0][kx]; dwx = dwh[0][kx]; } else { wx = wi[0][kx]; dwx = dwi[0][kx]; }
                const int x = lc[0] - H + kx, y = DIM == 3 ? lc[1] - H + ky : 0, z = lc[2] - H + kz;
                W.addf(comp, x, y, z, wx * wy * wz * lv);
                const R fv = W.f(comp, x, y, z) * lv;
                lo[0] += dwx * wy * wz * fv;
                if constexpr (DIM == 3) lo[1] += wx * dwy * wz * fv;
                lo[2] += wx * wy * dwz * fv;
            }
        }
    }
}

// Order-l interpolation on every axis from window cells b[a] .. b[a] + L
// (Uniform scheme), and its adjoint: scatter w * lv, accumulate d/doffset.
template <int DIM, int L, class R, class Win>
__device__ __forceinline__ R interp_fl(const Win &W, int comp, const int *b, const R *const *w)
{
    constexpr int NY = DIM == 3 ? L + 1 : 1;
    R s = R(0);
#pragma unroll
    for (int kz = 0; kz <= L; kz++)
#pragma unroll
        for (int ky = 0; ky < NY; ky++) {
            R row = R(0);
#pragma unroll
            for (int kx = 0; kx <= L; kx++) row += w[0][kx] * W.f(comp, b[0] + kx, DIM == 3 ? b[1] + ky : 0, b[2] + kz);
            s += (DIM == 3 ? w[1][ky] : R(1)) * w[2][kz] * row;
        }
    return s;
}

template <int DIM, int L, class R, class Win>
__device__ __forceinline__ void interp_adjl(Win &W, int comp, const int *b, const R *const *w, const R *const *dw,
                                            R lv, R *lo)
{
    constexpr int NY = DIM == 3 ? L + 1 : 1;
#pragma unroll
    for (int kz = 0; kz <= L; kz++)
#pragma unroll
        for (int ky = 0; ky < NY; ky++) {
            const R wy = DIM == 3 ? w[1][ky] : R(1), dwy = DIM == 3 ? dw[1][ky] : R(0);
#pragma unroll
            for (int kx = 0; kx <= L; kx++) {
                const int x = b[0] + kx, y = DIM == 3 ? b[1] + ky : 0, z = b[2] + kz;
                W.addf(comp, x, y, z, w[0][kx] * wy * w[2][kz] * lv);
                const R fv = W.f(comp, x, y, z) * lv;
                lo[0] += dw[0][kx] * wy * w[2][kz] * fv;
                if constexpr (DIM == 3) lo[1] += w[0][kx] * dwy * w[2][kz] * fv;
                lo[2] += w[0][kx] * wy * dw[2][kz] * fv;
            }
        }
}

// Uniform weights of one particle: integer-node weights wi from window cell
// bi, and for half-staggered samples the weights wu of the coordinate shifted
// by half a cell from window cell bu (one lower when the offset is below 1/2)
template <int DIM, int L, class R> struct UniformW {
    R wi[3][L + 1], wu[3][L + 1], dwi[3][L + 1], dwu[3][L + 1];
    int bi[3], bu[3];
    __device__ __forceinline__ UniformW(const int *lc, const R *off)
    {
        constexpr int H = (L - 1) / 2;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            bi[a] = bu[a] = lc[a] - H;
            if (DIM == 2 && a == 1) continue;
            const bool up = off[a] >= R(0.5);
            const R sh = up ? off[a] - R(0.5) : off[a] + R(0.5);
            bu[a] -= up ? 0 : 1;
            Shape<L, R>::integer(off[a], wi[a]);
            DShape<L, R>::integer(off[a], dwi[a]);
            Shape<L, R>::integer(sh, wu[a]);
            DShape<L, R>::integer(sh, dwu[a]);
        }
    }
    // component with staggering (SX, SY, SZ): its window start, weights and derivatives
    template <int SX, int SY, int SZ>
    __device__ __forceinline__ void pick(int *b, const R **w, const R **dw) const
    {
        b[0] = SX ? bu[0] : bi[0]; b[1] = SY ? bu[1] : bi[1]; b[2] = SZ ? bu[2] : bi[2];
        w[0] = SX ? wu[0] : wi[0]; w[1] = SY ? wu[1] : wi[1]; w[2] = SZ ? wu[2] : wi[2];
        dw[0] = SX ? dwu[0] : dwi[0]; dw[1] = SY ? dwu[1] : dwi[1]; dw[2] = SZ ? dwu[2] : dwi[2];
    }
    template <int SX, int SY, int SZ, class Win>
    __device__ __forceinline__ R f(const Win &W, int comp) const
    {
        int b[3];
        const R *w[3], *dw[3];
        pick<SX, SY, SZ>(b, w, dw);
        return interp_fl<DIM, L, R>(W, comp, b, w);
    }
    template <int SX, int SY, int SZ, class Win>
    __device__ __forceinline__ void adj(Win &W, int comp, R lv, R *lo) const
    {
        int b[3];
        const R *w[3], *dw[3];
        pick<SX, SY, SZ>(b, w, dw);
        interp_adjl<DIM, L, R>(W, comp, b, w, dw, lv, lo);
    }
};

// Reverse of one particle's step.  loff / lu hold the adjoints of the new
// offset / momentum on entry and of the old ones on exit.  IP: gather scheme
// (Galerkin or Uniform).
template <int DIM, int L, class R, int IP, class Win>
__device__ __forceinline__ void adjoint_particle(Win &W, const int *lc, const R *off, const R *u, R *loff, R *lu,
                                                 const R *dtd, R qdt2m, const R *cdr, R cyr)
{
    constexpr int H = (L - 1) / 2;
    R wi[3][L + 1], wh[3][L], dwi[3][L + 1], dwh[3][L];
    R E[3], B[3];
    // staggering: Ex(1,0,0) Ey(0,1,0) Ez(0,0,1) Bx(0,1,1) By(1,0,1) Bz(1,1,0)
    // (unused, and so removed by the compiler, with the Galerkin gather)
    const UniformW<DIM, L, R> uw(lc, off);
    if constexpr (IP == GATHER_UNIFORM) {
        E[0] = uw.template f<1, 0, 0>(W, 0);
        E[1] = uw.template f<0, 1, 0>(W, 1);
        E[2] = uw.template f<0, 0, 1>(W, 2);
        B[0] = uw.template f<0, 1, 1>(W, 3);
        B[1] = uw.template f<1, 0, 1>(W, 4);
        B[2] = uw.template f<1, 1, 0>(W, 5);
    } else {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (DIM == 2 && a == 1) continue;
            Shape<L, R>::integer(off[a], wi[a]);
            Shape<L, R>::half(off[a], wh[a]);
            DShape<L, R>::integer(off[a], dwi[a]);
            DShape<L, R>::half(off[a], dwh[a]);
        }
        E[0] = interp_f<1, 0, 0, DIM, L, R>(W, 0, lc, wi, wh);
        E[1] = interp_f<0, 1, 0, DIM, L, R>(W, 1, lc, wi, wh);
        E[2] = interp_f<0, 0, 1, DIM, L, R>(W, 2, lc, wi, wh);
        B[0] = interp_f<0, 1, 1, DIM, L, R>(W, 3, lc, wi, wh);
        B[1] = interp_f<1, 0, 1, DIM, L, R>(W, 4, lc, wi, wh);
        B[2] = interp_f<1, 1, 0, DIM, L, R>(W, 5, lc, wi, wh);
    }
    // Boris and move, recomputed with the forward kernel's own routines
    R un[3];
    BorisTrace<R> bt;
    boris_push<R>(u, E, B, qdt2m, un, bt);
    const R *um = bt.um, *t = bt.t, *sv = bt.sv, *up = bt.up;
    const R igm = bt.igm, f = bt.f;
    int dc[3], err = 0;
    R offn[3];
    const R ig = move_cells<DIM, R>(off, un, dtd, dc, offn, err);
    // Esirkepov reverse
    R S0[3][L + 2], S1[3][L + 2], D0[3][L + 2], D1[3][L + 2], lS0[3][L + 2], lS1[3][L + 2];
    int base[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
        for (int i = 0; i < L + 2; i++) { lS0[a][i] = R(0); lS1[a][i] = R(0); }
        if (DIM == 2 && a == 1) { base[a] = 0; continue; }
        R w0[L + 1], w1[L + 1], d0[L + 1], d1[L + 1];
        Shape<L, R>::integer(off[a], w0);
        Shape<L, R>::integer(offn[a], w1);
        DShape<L, R>::integer(off[a], d0);
        DShape<L, R>::integer(offn[a], d1);
        const int mn = dc[a] < 0 ? -1 : 0;
        const bool sh0 = mn < 0, sh1 = dc[a] > 0;
        base[a] = lc[a] + mn - H;
#pragma unroll
        for (int i = 0; i < L + 2; i++) {
            const int jl = i >= 1 ? i - 1 : 0, jh = i < L + 1 ? i : L;
            const bool okl = i >= 1, okh = i < L + 1;
            S0[a][i] = sh0 ? (okl ? w0[jl] : R(0)) : (okh ? w0[jh] : R(0));
            D0[a][i] = sh0 ? (okl ? d0[jl] : R(0)) : (okh ? d0[jh] : R(0));
            S1[a][i] = sh1 ? (okl ? w1[jl] : R(0)) : (okh ? w1[jh] : R(0));
            D1[a][i] = sh1 ? (okl ? d1[jl] : R(0)) : (okh ? d1[jh] : R(0));
        }
    }
    R lvy = R(0);
    if constexpr (DIM == 2) {
#pragma unroll
        for (int k = 0; k < L + 2; k++) {
            const R az = R(0.5) * (S0[2][k] + S1[2][k]);
            R acc = R(0);
#pragma unroll
            for (int i = L; i >= 0; i--) {
                acc += cdr[0] * W.lj(0, base[0] + i, 0, base[2] + k);
                lS1[0][i] += acc * az;
                lS0[0][i] -= acc * az;
                const R tt = R(0.5) * acc * (S1[0][i] - S0[0][i]);
                lS0[2][k] += tt;
                lS1[2][k] += tt;
            }
        }
#pragma unroll
        for (int i = 0; i < L + 2; i++) {
            const R ax = R(0.5) * (S0[0][i] + S1[0][i]);
            R acc = R(0);
#pragma unroll
            for (int k = L; k >= 0; k--) {
                acc += cdr[2] * W.lj(2, base[0] + i, 0, base[2] + k);
                lS1[2][k] += acc * ax;
                lS0[2][k] -= acc * ax;
                const R tt = R(0.5) * acc * (S1[2][k] - S0[2][k]);
                lS0[0][i] += tt;
                lS1[0][i] += tt;
            }
        }
        const R vy = un[1] * ig;
#pragma unroll
        for (int k = 0; k < L + 2; k++)
#pragma unroll
            for (int i = 0; i < L + 2; i++) {
                const R lj = W.lj(1, base[0] + i, 0, base[2] + k);
                const R wy = R(1.0 / 3.0) * S0[0][i] * S0[2][k] + R(1.0 / 6.0) * S1[0][i] * S0[2][k]
                           + R(1.0 / 6.0) * S0[0][i] * S1[2][k] + R(1.0 / 3.0) * S1[0][i] * S1[2][k];
                lvy += cyr * wy * lj;
                const R lw = cyr * vy * lj;
                lS0[0][i] += lw * (R(1.0 / 3.0) * S0[2][k] + R(1.0 / 6.0) * S1[2][k]);
                lS1[0][i] += lw * (R(1.0 / 6.0) * S0[2][k] + R(1.0 / 3.0) * S1[2][k]);
                lS0[2][k] += lw * (R(1.0 / 3.0) * S0[0][i] + R(1.0 / 6.0) * S1[0][i]);
                lS1[2][k] += lw * (R(1.0 / 6.0) * S0[0][i] + R(1.0 / 3.0) * S1[0][i]);
            }
    } else {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
#pragma unroll
            for (int ib = 0; ib < L + 2; ib++)
#pragma unroll
                for (int ic = 0; ic < L + 2; ic++) {
                    const R tr = R(1.0 / 3.0) * S0[b][ib] * S0[c][ic] + R(1.0 / 6.0) * S1[b][ib] * S0[c][ic]
                               + R(1.0 / 6.0) * S0[b][ib] * S1[c][ic] + R(1.0 / 3.0) * S1[b][ib] * S1[c][ic];
                    R acc = R(0), ltr = R(0);
#pragma unroll
                    for (int ia = L; ia >= 0; ia--) {
                        int nd[3];
                        nd[a] = base[a] + ia;
                        nd[b] = base[b] + ib;
                        nd[c] = base[c] + ic;
                        acc += cdr[a] * W.lj(a, nd[0], nd[1], nd[2]);
                        lS1[a][ia] += acc * tr;
                        lS0[a][ia] -= acc * tr;
                        ltr += acc * (S1[a][ia] - S0[a][ia]);
                    }
                    lS0[b][ib] += ltr * (R(1.0 / 3.0) * S0[c][ic] + R(1.0 / 6.0) * S1[c][ic]);
                    lS1[b][ib] += ltr * (R(1.0 / 6.0) * S0[c][ic] + R(1.0 / 3.0) * S1[c][ic]);
                    lS0[c][ic] += ltr * (R(1.0 / 3.0) * S0[b][ib] + R(1.0 / 6.0) * S1[b][ib]);
                    lS1[c][ic] += ltr * (R(1.0 / 6.0) * S0[b][ib] + R(1.0 / 3.0) * S1[b][ib]);
                }
        }
    }
    // shapes -> offsets; move reverse
    R lo[3] = {R(0), R(0), R(0)}, lv[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (DIM == 2 && a == 1) continue;
        R l0 = R(0), l1 = R(0);
#pragma unroll
        for (int i = 0; i < L + 2; i++) { l0 += lS0[a][i] * D0[a][i]; l1 += lS1[a][i] * D1[a][i]; }
        const R lx1 = loff[a] + l1;
        lo[a] = l0 + lx1;
        lv[a] = dtd[a] * lx1;
    }
    if constexpr (DIM == 2) lv[1] += lvy;
    const R udl = un[0] * lv[0] + un[1] * lv[1] + un[2] * lv[2];
    R lun[3];
#pragma unroll
    for (int a = 0; a < 3; a++) lun[a] = lu[a] + lv[a] * ig - un[a] * udl * ig * ig * ig;
    // Boris reverse
    R lE[3], lB[3], lum[3], lup[3], ls[3], lt[3];
#pragma unroll
    for (int a = 0; a < 3; a++) { lE[a] = qdt2m * lun[a]; lum[a] = lun[a]; }
    lup[0] = sv[1] * lun[2] - sv[2] * lun[1];
    lup[1] = sv[2] * lun[0] - sv[0] * lun[2];
    lup[2] = sv[0] * lun[1] - sv[1] * lun[0];
    ls[0] = lun[1] * up[2] - lun[2] * up[1];
    ls[1] = lun[2] * up[0] - lun[0] * up[2];
    ls[2] = lun[0] * up[1] - lun[1] * up[0];
    lum[0] += lup[0] + (t[1] * lup[2] - t[2] * lup[1]);
    lum[1] += lup[1] + (t[2] * lup[0] - t[0] * lup[2]);
    lum[2] += lup[2] + (t[0] * lup[1] - t[1] * lup[0]);
    lt[0] = lup[1] * um[2] - lup[2] * um[1];
    lt[1] = lup[2] * um[0] - lup[0] * um[2];
    lt[2] = lup[0] * um[1] - lup[1] * um[0];
    const R lf = ls[0] * t[0] + ls[1] * t[1] + ls[2] * t[2];
    const R lt2 = -lf * f * f * R(0.5);
#pragma unroll
    for (int a = 0; a < 3; a++) lt[a] += f * ls[a] + R(2) * t[a] * lt2;
    // t = qdt2m B igm, igm = (1 + um.um)^(-1/2)
    const R lg = -(t[0] * lt[0] + t[1] * lt[1] + t[2] * lt[2]) * igm;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lB[a] = qdt2m * lt[a] * igm;
        lum[a] += lg * um[a] * igm;
        lE[a] += qdt2m * lum[a];
        lu[a] = lum[a];
    }
    // gather reverse
    if constexpr (IP == GATHER_UNIFORM) {
        uw.template adj<1, 0, 0>(W, 0, lE[0], lo);
        uw.template adj<0, 1, 0>(W, 1, lE[1], lo);
        uw.template adj<0, 0, 1>(W, 2, lE[2], lo);
        uw.template adj<0, 1, 1>(W, 3, lB[0], lo);
        uw.template adj<1, 0, 1>(W, 4, lB[1], lo);
        uw.template adj<1, 1, 0>(W, 5, lB[2], lo);
    } else {
        interp_adj<1, 0, 0, DIM, L, R>(W, 0, lc, wi, wh, dwi, dwh, lE[0], lo);
        interp_adj<0, 1, 0, DIM, L, R>(W, 1, lc, wi, wh, dwi, dwh, lE[1], lo);
        interp_adj<0, 0, 1, DIM, L, R>(W, 2, lc, wi, wh, dwi, dwh, lE[2], lo);
        interp_adj<0, 1, 1, DIM, L, R>(W, 3, lc, wi, wh, dwi, dwh, lB[0], lo);
        interp_adj<1, 0, 1, DIM, L, R>(W, 4, lc, wi, wh, dwi, dwh, lB[1], lo);
        interp_adj<1, 1, 0, DIM, L, R>(W, 5, lc, wi, wh, dwi, dwh, lB[2], lo);
    }
#pragma unroll
    for (int a = 0; a < 3; a++) loff[a] = lo[a];
}

template <int DIM, int L, class R, int IP>
__global__ void __launch_bounds__(256) k_adj_particles(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                       int nwork, int wmx, int wmy, int wmz)
{
    constexpr int JL = (L + 1) / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, bs = blockDim.x;
    const int wcmax = wmx * wmy * wmz;
    for (int item = blockIdx.x; item < nwork; item += gridDim.x) {
        const int inst = work[item].x, tile = work[item].y;
        const InstDesc &D = Dt[inst];
        const int p0 = D.tstart[tile], p1 = D.tstart[tile + 1];
        if (p1 <= p0) continue;
        int lo[3], o[3], wn[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = D.tbox[tile * 6 + a];
            const int ext = D.tbox[tile * 6 + 3 + a];
            if (DIM == 2 && a == 1) { o[a] = 0; wn[a] = 1; continue; }
            o[a] = wrapi(lo[a] - JL, D.n[a]);
            wn[a] = ext + L + 2;
        }
        const bool fits = wn[0] <= wmx && wn[1] <= wmy && wn[2] <= wmz;
        const int wc = wn[0] * wn[1] * wn[2];
        R *sF = reinterpret_cast<R *>(smem);
        R *sLJ = sF + 6 * wcmax;
        double *sLF = reinterpret_cast<double *>(smem + adj_lf_offset(wcmax, sizeof(R)));
        const int nn[3] = {D.n[0], D.n[1], D.n[2]};
        if (fits) {
            const gp<const R> src[6] = {G<R>((const void *)D.Et[0]), G<R>((const void *)D.Et[1]),
                                        G<R>((const void *)D.Et[2]), G<R>((const void *)D.Bt[0]),
                                        G<R>((const void *)D.Bt[1]), G<R>((const void *)D.Bt[2])};
            const gp<const R> lsrc[3] = {G<R>((const void *)D.lJ[0]), G<R>((const void *)D.lJ[1]),
                                         G<R>((const void *)D.lJ[2])};
            auto addr = [&](int c) { return window_cell(c, wn, o, nn); };
            stage<2, 6, R, R>(sF, wc, src, wc, addr, IdentityIx{}, PlainCv{});
            stage<2, 3, R, R>(sLJ, wc, lsrc, wc, addr, IdentityIx{}, PlainCv{});
            for (int c = tid; c < 6 * wc; c += bs) sLF[c] = 0.0;
        }
        __syncthreads();
        const R dtd[3] = {(R)D.dtd[0], (R)D.dtd[1], (R)D.dtd[2]};
        const R cdr[3] = {(R)D.cdep_r[0], (R)D.cdep_r[1], (R)D.cdep_r[2]};
        const R qdt2m = (R)D.qdt2m, cyr = (R)D.cy2d_r;
        AdjLds<R> lw{sF, sLJ, sLF, wn[0], wn[0] * wn[1], wc};
        AdjGlb<R> gw;
        if (!fits) {
            for (int k = 0; k < 3; k++) {
                gw.F[k] = (const R *)D.Et[k]; gw.F[3 + k] = (const R *)D.Bt[k];
                gw.LJ[k] = (const R *)D.lJ[k];
                gw.LF[k] = (R *)D.lEt[k]; gw.LF[3 + k] = (R *)D.lBt[k];
                gw.o[k] = o[k]; gw.n[k] = D.n[k];
            }
        }
        const gp<const unsigned> pidx = G<unsigned>((const void *)D.pidx);
        const gp<const R> pu[3] = {G<R>((const void *)D.pu[0]), G<R>((const void *)D.pu[1]), G<R>((const void *)D.pu[2])};
        const gp<const R> po[3] = {G<R>((const void *)D.poff[0]), G<R>((const void *)D.poff[1]),
                                   G<R>((const void *)D.poff[2])};
        const gp<R> plu[3] = {G<R>(D.lu[0]), G<R>(D.lu[1]), G<R>(D.lu[2])};
        const gp<R> plo[3] = {G<R>(D.loff[0]), G<R>(D.loff[1]), G<R>(D.loff[2])};
        // the next particle's state is loaded while this one is reversed (its
        // index clamped to the tile's last particle, so every load is valid)
        unsigned nidx = 0;
        R nu[3], nlu[3], noff[3], nloff[3];
        // (streamed state: non-temporal loads and stores, as in the forward kernel)
        auto fetch = [&](int q) {
            nidx = __builtin_nontemporal_load(&pidx[q]);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                nu[a] = __builtin_nontemporal_load(&pu[a][q]);
                nlu[a] = __builtin_nontemporal_load(&plu[a][q]);
                if (DIM == 2 && a == 1) { noff[a] = R(0); nloff[a] = R(0); continue; }
                noff[a] = __builtin_nontemporal_load(&po[a][q]);
                nloff[a] = __builtin_nontemporal_load(&plo[a][q]);
            }
        };
        if (p0 + tid < p1) fetch(p0 + tid);
        for (int p = p0 + tid; p < p1; p += bs) {
            int c[3];
            unpack_cell<DIM>(nidx, c);
            int lc[3];
            R off[3], u[3], loff[3], lu[3];
#pragma unroll
            for (int a = 0; a < 3; a++) {
                u[a] = nu[a];
                lu[a] = nlu[a];
                off[a] = noff[a];
                loff[a] = nloff[a];
                if (DIM == 2 && a == 1) { lc[a] = 0; continue; }
                int rel = c[a] - lo[a];
                rel += rel < 0 ? nn[a] : 0;
                lc[a] = rel + JL;
            }
            fetch(min(p + bs, p1 - 1));
            if (fits) adjoint_particle<DIM, L, R, IP>(lw, lc, off, u, loff, lu, dtd, qdt2m, cdr, cyr);
            else adjoint_particle<DIM, L, R, IP>(gw, lc, off, u, loff, lu, dtd, qdt2m, cdr, cyr);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                __builtin_nontemporal_store(lu[a], &plu[a][p]);
                if (!(DIM == 2 && a == 1)) __builtin_nontemporal_store(loff[a], &plo[a][p]);
            }
        }
        __syncthreads();
        if (fits) {
            const gp<R> dst[6] = {G<R>(D.lEt[0]), G<R>(D.lEt[1]), G<R>(D.lEt[2]),
                                  G<R>(D.lBt[0]), G<R>(D.lBt[1]), G<R>(D.lBt[2])};
            for (int c = tid; c < wc; c += bs) {
                const int g = window_cell(c, wn, o, nn);
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    const double v = sLF[k * wc + c];
                    if (v != 0.0) gatomic_add(dst[k] + g, (R)v);
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ stencil passes
enum { PL_T1 = 1, PL_T2 = 2, PL_LSEEN = 4, PL_LEB = 5 };

__device__ __forceinline__ void *plane(const InstDesc &D, int sel, int comp)
{
    switch (sel) {
    case PL_T1: return D.T1[comp];
    case PL_T2: return D.T2[comp];
    case PL_LSEEN: return comp < 3 ? D.lEt[comp] : D.lBt[comp - 3];
    default: return comp < 3 ? D.lE[comp] : D.lB[comp - 3];
    }
}

// AXIS 2 with filter_only = 0 uses the per-component correction taps;
// filter_only = 1 uses the filter taps alone.  accumulate adds into dst.
template <int AXIS, class R>
__global__ void __launch_bounds__(256) k_pass(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                              int src_sel, int dst_sel, int filter_only, int accumulate)
{
    const InstDesc &D = Dt[work[blockIdx.x].x];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    const int comp = blockIdx.y;
    if (cell >= D.ncell) return;
    const R *src = (const R *)plane(D, src_sel, comp);
    R *dst = (R *)plane(D, dst_sel, comp);
    const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
    const int i = cell % nx, r = cell / nx, j = r % ny, k = r / ny;
    R acc = R(0);
    if constexpr (AXIS == 2) {
        const double *tap = filter_only ? D.tzf : D.tz[comp < 2 ? 0 : 1];
        const int h = filter_only ? D.hzf : D.hz;
        const int rowoff = i + j * nx, pl = nx * ny;
        for (int t = -h; t <= h; t++) {
            int kk = k + t;
            kk = ((kk % nz) + nz) % nz;
            acc += (R)tap[t + h] * src[rowoff + kk * pl];
        }
    } else if constexpr (AXIS == 0) {
        const int h = D.hx, rowbase = cell - i;
        for (int t = -h; t <= h; t++) {
            int ii = i + t;
            ii = ((ii % nx) + nx) % nx;
            acc += (R)D.tx[t + h] * src[rowbase + ii];
        }
    } else {
        const int h = D.hy, base = i + k * ny * nx;
        for (int t = -h; t <= h; t++) {
            int jj = j + t;
            jj = ((jj % ny) + ny) % ny;
            acc += (R)D.ty[t + h] * src[base + jj * nx];
        }
    }
    if (accumulate) dst[cell] += acc;
    else dst[cell] = acc;
}

// dW/da_j += <S_z^j Lambda_c, E1_c> with Lambda_c = F lambda_Et_c (c = blockIdx.y in {0,1})
template <class R>
__global__ void __launch_bounds__(256) k_adj_grad(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                  int lam_sel)
{
    const InstDesc &D = Dt[work[blockIdx.x].x];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    const int comp = blockIdx.y;
    double v[9];
    for (int j = 0; j < 9; j++) v[j] = 0.0;
    if (cell < D.ncell) {
        const R *lam = (const R *)plane(D, lam_sel, comp);
        const double e1 = (double)((const R *)D.E[0][comp])[cell];
        const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
        const int i = cell % nx, r = cell / nx, j0 = r % ny, k = r / ny;
        const int rowoff = i + j0 * nx, pl = nx * ny;
        for (int j = 0; j <= D.psi_deg; j++) {
            double s = 0.0;
            for (int t = -j; t <= j; t++) {
                int kk = k + t;
                kk = ((kk % nz) + nz) % nz;
                s += D.sj[j][8 + t] * (double)lam[rowoff + kk * pl];
            }
            v[j] = s * e1;
        }
    }
    for (int j = 0; j < 9; j++) {
        if (j > D.psi_deg) break;
        const double w = wave_sum(v[j]);
        if ((threadIdx.x & 63) == 0 && w != 0.0) unsafeAtomicAdd(&D.grad[grad_copy() + j], w);
    }
}

// lambda_E -= h Cb lambda_B  (backward differences, B locations -> E locations)
template <int DIM, class R>
__global__ void __launch_bounds__(256) k_adj_yee_e(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work)
{
    const InstDesc &D = Dt[work[blockIdx.x].x];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    if (cell >= D.ncell) return;
    const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
    const int i = cell % nx, r = cell / nx, j = r % ny, k = r / ny;
    const int im = (i == 0 ? nx - 1 : i - 1) + (j + k * ny) * nx;
    const int km = i + (j + (k == 0 ? nz - 1 : k - 1) * ny) * nx;
    const R *Bx = (const R *)D.lB[0], *By = (const R *)D.lB[1], *Bz = (const R *)D.lB[2];
    const R idx = R(1) / (R)D.d[0], idz = R(1) / (R)D.d[2], h = R(0.5) * (R)D.dt;
    const R bx = Bx[cell], by = By[cell], bz = Bz[cell];
    R dyBz = R(0), dyBx = R(0);
    if constexpr (DIM == 3) {
        const int jm = i + ((j == 0 ? ny - 1 : j - 1) + k * ny) * nx;
        const R idy = R(1) / (R)D.d[1];
        dyBz = (bz - Bz[jm]) * idy;
        dyBx = (bx - Bx[jm]) * idy;
    }
    ((R *)D.lE[0])[cell] -= h * (dyBz - (by - By[km]) * idz);
    ((R *)D.lE[1])[cell] -= h * ((bx - Bx[km]) * idz - (bz - Bz[im]) * idx);
    ((R *)D.lE[2])[cell] -= h * ((by - By[im]) * idx - dyBx);
}

// lambda_B += dt Cf lambda_E (forward differences);  lambda_J = -dt lambda_E
template <int DIM, class R>
__global__ void __launch_bounds__(256) k_adj_yee_b(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work)
{
    const InstDesc &D = Dt[work[blockIdx.x].x];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    if (cell >= D.ncell) return;
    const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
    const int i = cell % nx, r = cell / nx, j = r % ny, k = r / ny;
    const int ip = (i + 1 == nx ? 0 : i + 1) + (j + k * ny) * nx;
    const int kp = i + (j + (k + 1 == nz ? 0 : k + 1) * ny) * nx;
    const R *Ex = (const R *)D.lE[0], *Ey = (const R *)D.lE[1], *Ez = (const R *)D.lE[2];
    const R idx = R(1) / (R)D.d[0], idz = R(1) / (R)D.d[2], dt = (R)D.dt;
    const R ex = Ex[cell], ey = Ey[cell], ez = Ez[cell];
    R dyEz = R(0), dyEx = R(0);
    if constexpr (DIM == 3) {
        const int jp = i + ((j + 1 == ny ? 0 : j + 1) + k * ny) * nx;
        const R idy = R(1) / (R)D.d[1];
        dyEz = (Ez[jp] - ez) * idy;
        dyEx = (Ex[jp] - ex) * idy;
    }
    ((R *)D.lB[0])[cell] += dt * (dyEz - (Ey[kp] - ey) * idz);
    ((R *)D.lB[1])[cell] += dt * ((Ex[kp] - ex) * idz - (Ez[ip] - ez) * idx);
    ((R *)D.lB[2])[cell] += dt * ((Ey[ip] - ey) * idx - dyEx);
    ((R *)D.lJ[0])[cell] = -dt * ex;
    ((R *)D.lJ[1])[cell] = -dt * ey;
    ((R *)D.lJ[2])[cell] = -dt * ez;
}

// loss W and its gradient seed lambda_E = dV (Ex, Ey, 0), lambda_B = dV (Bx, By, 0)
template <class R>
__global__ void __launch_bounds__(256) k_adj_seed(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work, int par)
{
    const InstDesc &D = Dt[work[blockIdx.x].x];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    double w = 0.0;
    if (cell < D.ncell) {
        const R dV = (R)D.dV;
        for (int c = 0; c < 3; c++) {
            const R e = ((const R *)D.E[par][c])[cell], b = ((const R *)D.B[par][c])[cell];
            ((R *)D.lE[c])[cell] = c < 2 ? dV * e : R(0);
            ((R *)D.lB[c])[cell] = c < 2 ? dV * b : R(0);
            ((R *)D.lJ[c])[cell] = R(0);
            ((R *)D.lEt[c])[cell] = R(0);
            ((R *)D.lBt[c])[cell] = R(0);
            if (c < 2) w += 0.5 * D.dV * ((double)e * e + (double)b * b);
        }
    }
    w = wave_sum(w);
    if ((threadIdx.x & 63) == 0 && w != 0.0) unsafeAtomicAdd(D.loss, w);
}

template <class R>
__global__ void __launch_bounds__(256) k_adj_seed_particles(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work)
{
    const InstDesc &D = Dt[work[blockIdx.x].x];
    const long long p = (long long)work[blockIdx.x].y * PIC_PART_CHUNK + threadIdx.x;
    if (p >= D.np) return;
    for (int a = 0; a < 3; a++) {
        ((R *)D.lu[a])[p] = R(0);
        if (D.loff[a]) ((R *)D.loff[a])[p] = R(0);
    }
}

template <class R>
__global__ void __launch_bounds__(256) k_zero_lseen(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work)
{
    const InstDesc &D = Dt[work[blockIdx.x].x];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    if (cell >= D.ncell) return;
    for (int c = 0; c < 3; c++) { ((R *)D.lEt[c])[cell] = R(0); ((R *)D.lBt[c])[cell] = R(0); }
}

// ------------------------------------------------------------ fused 2D kernels
// Adjoint of the fields as seen by the particles, 2D, one (64 x TZ) tile of one
// component per block.  GRAD (components x, y): Lambda = F lambda_Et (filter
// passes only), then lambda_E + sum_j a_j S_z^j Lambda
// (= lambda_E + Psi_E(S_z) F lambda_Et) and dW/da_j += <S_z^j Lambda, E1>.
// Otherwise (E_z and all of B): lambda + Psi_B(S_z) F lambda_t with the
// combined taps.  The sums go to the scratch planes T1: the reverse Yee kernel
// reads them with halos and writes lambda_E, lambda_B.
// The window (tile plus the z halo deg + hz and the x halo hx) is staged in LDS
// with waves on rows and lanes on columns; the x filter runs on every staged
// row, four neighbouring output columns per thread; then each wave walks down
// its TZ / 4 output rows of each column in registers: the z pass, and for GRAD
// the S_z^j stencils on the z-filtered column.  Stencils on different axes of
// the periodic grid commute, so x first is the same operator.  HZ (half-width
// of the z pass), HX and DEG >= 0 are compile-time widths (loops unrolled,
// taps in registers); -1 reads the descriptor.
#define ADJ_TX 64
template <class R, int TZ, bool GRAD, int HZ, int HX, int DEG>
__device__ __forceinline__ void adj_seen_body(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work, int comp)
{
    constexpr int NW = PIC_FIELD_CHUNK / 64, RB = TZ / NW;
    static_assert(TZ % NW == 0, "the four waves split the output rows");
    extern __shared__ __align__(16) unsigned char smem[];
    const int inst = work[blockIdx.x].x, t = work[blockIdx.x].y;
    const InstDesc &D = Dt[inst];
    const int nx = D.n[0], nz = D.n[2];
    const int ntx = (nx + ADJ_TX - 1) / ADJ_TX;
    const int x0 = (t % ntx) * ADJ_TX, z0 = (t / ntx) * TZ;
    const int hx = HX >= 0 ? HX : D.hx;
    const int deg = GRAD ? (DEG >= 0 ? DEG : D.psi_deg) : 0;
    const int hz = HZ >= 0 ? HZ : (GRAD ? D.hzf : D.hz);
    const int ez = deg + hz;                    // z halo of the window
    const int wx = ADJ_TX + 2 * hx, wz = TZ + 2 * ez;
    R *win = reinterpret_cast<R *>(smem);       // wz x wx: lambda_t with halos
    R *mid = win + wx * wz;                     // wz x 64: after the x filter
    R *tz = mid + ADJ_TX * wz;
    R *tx = tz + 2 * PIC_MAX_HZ + 1;
    __shared__ double red[9][NW];
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int zr = wave * RB;                   // this wave's first output row
    const int gx = x0 + lane;
    // what the last phase reads at its own cells, loaded first (rows and
    // columns clamped into the grid) so that its latency overlaps the window's
    const gp<const R> own = G<R>((const void *)(comp < 3 ? D.lE[comp] : D.lB[comp - 3]));
    R pown[RB], pe1[RB];
    {
        const gp<const R> e1p = G<R>((const void *)D.E[0][comp < 3 ? comp : 0]);
        const int gxc = min(gx, nx - 1);
#pragma unroll
        for (int j = 0; j < RB; j++) {
            const int g = min(z0 + zr + j, nz - 1) * nx + gxc;
            pown[j] = own[g];
            pe1[j] = GRAD ? e1p[g] : R(0);
        }
    }
    const double *tzs = GRAD ? D.tzf : D.tz[comp < 2 ? 0 : 1];
    constexpr int NTZ = HZ >= 0 ? 2 * HZ + 1 : 1, NTX = HX >= 0 ? 2 * HX + 1 : 1;
    R rz[NTZ], rx[NTX];
    if constexpr (HZ >= 0) {
#pragma unroll
        for (int k = 0; k < NTZ; k++) rz[k] = (R)tzs[k];
    } else {
        for (int i = threadIdx.x; i <= 2 * hz; i += blockDim.x) tz[i] = (R)tzs[i];
    }
    if constexpr (HX >= 0) {
#pragma unroll
        for (int k = 0; k < NTX; k++) rx[k] = (R)D.tx[k];
    } else {
        for (int i = threadIdx.x; i <= 2 * hx; i += blockDim.x) tx[i] = (R)D.tx[i];
    }
    const gp<const R> src = G<R>((const void *)(comp < 3 ? D.lEt[comp] : D.lBt[comp - 3]));
    // staging: column a = lane, column b = 64 + lane for the right halo (lane < 2 hx)
    const bool hasb = lane < 2 * hx;
    const int gxa = wrap_near(x0 - hx + lane, nx);
    const int gxb = hasb ? wrap_near(x0 - hx + ADJ_TX + lane, nx) : gxa;
    // rows per wave: the whole window in one round when its height is a constant
    constexpr int WZC = (HZ >= 0 && (!GRAD || DEG >= 0)) ? TZ + 2 * ((GRAD ? DEG : 0) + HZ) : 0;
    constexpr int U = WZC > 0 ? (WZC + NW - 1) / NW : 4;
    for (int r0 = wave; r0 < wz; r0 += U * NW) {
        R va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int row = min(r0 + u * NW, wz - 1);
            const int base = wrap_near(z0 - ez + row, nz) * nx;
            va[u] = src[base + gxa];
            vb[u] = src[base + gxb];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int row = r0 + u * NW;
            if (row < wz) {
                win[row * wx + lane] = va[u];
                if (hasb) win[row * wx + ADJ_TX + lane] = vb[u];
            }
        }
    }
    __syncthreads();
    // x filter: item (row r, output columns [4 q, 4 q + 4)) of wz x 16 items
    constexpr int XQ = 4, NQ = ADJ_TX / XQ;
    for (int it = threadIdx.x; it < wz * NQ; it += blockDim.x) {
        const int r = it / NQ, c0 = (it % NQ) * XQ;
        const R *w = win + r * wx + c0;
        R *o = mid + r * ADJ_TX + c0;
        if constexpr (HX >= 0) {
            R v[XQ + 2 * HX];
#pragma unroll
            for (int k = 0; k < XQ + 2 * HX; k++) v[k] = w[k];
#pragma unroll
            for (int q = 0; q < XQ; q++) {
                R acc = R(0);
#pragma unroll
                for (int k = 0; k < NTX; k++) acc += rx[k] * v[q + k];
                o[q] = acc;
            }
        } else {
            for (int q = 0; q < XQ; q++) {
                R acc = R(0);
                for (int k = 0; k <= 2 * hx; k++) acc += tx[k] * w[q + k];
                o[q] = acc;
            }
        }
    }
    __syncthreads();
    // z: output row zr + j of this column takes mid rows zr + j .. zr + j + 2 ez
    gp<R> dst = G<R>(D.T1[comp]);
    const R *m = mid + zr * ADJ_TX + lane;
    constexpr int NJ = GRAD ? (DEG >= 0 ? DEG + 1 : 9) : 1;
    R gpart[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j++) gpart[j] = R(0);
    R out[RB];
    if constexpr (HZ >= 0 && (!GRAD || DEG >= 0)) {
        constexpr int DG = GRAD ? DEG : 0, NL = RB + 2 * DG;
        R v[NL + 2 * HZ];
#pragma unroll
        for (int k = 0; k < NL + 2 * HZ; k++) v[k] = m[k * ADJ_TX];
        // z pass: rows zr - deg .. zr + RB + deg of Lambda (GRAD) or the output rows
        R lz[NL];
#pragma unroll
        for (int i = 0; i < NL; i++) {
            R acc = R(0);
#pragma unroll
            for (int k = 0; k < NTZ; k++) acc += rz[k] * v[i + k];
            lz[i] = acc;
        }
        if constexpr (GRAD) {
#pragma unroll
            for (int j = 0; j < RB; j++) {
                R add = R(0);
#pragma unroll
                for (int p = 0; p <= DG; p++) {
                    R tj = R(0);
#pragma unroll
                    for (int k = -p; k <= p; k++) tj += (R)D.sj[p][8 + k] * lz[j + DG + k];
                    add += (R)D.psi_e[p] * tj;
                    gpart[p] += tj * pe1[j];
                }
                out[j] = add;
            }
        } else {
#pragma unroll
            for (int j = 0; j < RB; j++) out[j] = lz[j];
        }
    } else {
        // widths from the descriptor: the same sums read straight from LDS
        auto ztap = [&](int q) -> R {
            if constexpr (HZ >= 0) return rz[q];
            else return tz[q];
        };
#pragma unroll
        for (int j = 0; j < RB; j++) {
            R add = R(0);
            if constexpr (GRAD) {
#pragma unroll
                for (int p = 0; p < NJ; p++) {
                    if (p > deg) break;
                    R tj = R(0);
                    for (int k = -p; k <= p; k++) {
                        // Lambda at output row zr + j + k: mid rows zr + j + deg + k + [0, 2 hz]
                        const R *mm = m + (j + deg + k) * ADJ_TX;
                        R lam = R(0);
                        for (int q = 0; q <= 2 * hz; q++) lam += ztap(q) * mm[q * ADJ_TX];
                        tj += (R)D.sj[p][8 + k] * lam;
                    }
                    add += (R)D.psi_e[p] * tj;
                    gpart[p] += tj * pe1[j];
                }
            } else {
                const R *mm = m + j * ADJ_TX;
                for (int q = 0; q <= 2 * hz; q++) add += ztap(q) * mm[q * ADJ_TX];
            }
            out[j] = add;
        }
    }
    if (gx < nx) {
#pragma unroll
        for (int j = 0; j < RB; j++) {
            const int gz = z0 + zr + j;
            if (gz < nz) dst[gz * nx + gx] = pown[j] + out[j];
        }
    }
    if constexpr (GRAD) {
        // columns beyond the grid (gx >= nx) read clamped E1 and must not count
        if (gx >= nx)
#pragma unroll
            for (int j = 0; j < NJ; j++) gpart[j] = R(0);
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            if (DEG < 0 && j > deg) break;
            const double v = wave_sum((double)gpart[j]);
            if (lane == 0) red[j][wave] = v;
        }
        __syncthreads();
        if (threadIdx.x <= deg) {
            const int j = threadIdx.x;
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < NW; w++) v += red[j][w];
            if (v != 0.0) unsafeAtomicAdd(&D.grad[grad_copy() + j], v);
        }
    }
}

// blockIdx.y = component: x and y take the gradient path (z filter half-width
// HZE, Psi degree DEG), the others the combined stencil (half-width HZB).
template <class R, int TZ, int HZE, int HX, int DEG, int HZB>
__global__ void __launch_bounds__(256) k_adj_seen_2d(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work)
{
    if (blockIdx.y < 2) adj_seen_body<R, TZ, true, HZE, HX, DEG>(Dt, work, blockIdx.y);
    else adj_seen_body<R, TZ, false, HZB, HX, 0>(Dt, work, blockIdx.y);
}

// Fused transposed Yee update (2D): with h = dt/2 and Cb = Cf^T,
//   lE' = lE - h Cb lB;   lB' = lB + dt Cf lE';  lJ = -dt lE';   lE'' = lE' - h Cb lB'
// One window for the six input planes: cells [x0 - 2, x0 + TX + 1) x [z0 - 2, z0 + TZ + 1).
// CK: with the Cole-Karkkainen curl, the transposed Faraday curl averages each
// backward difference across its direction with (1/8, 3/4, 1/8); the window
// grows by two cells on the high side: lambda_E' on [-1, T+1], lambda_B'' on [-1, T].
// SPLIT blocks share one work item (a tile of SPLIT * TZ rows), TZ rows each:
// more blocks for the small grids the reverse sweep runs on.
template <class R, int TZ, bool CK = false, int SPLIT = 1>
__global__ void __launch_bounds__(256) k_adj_yee_2d(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work)
{
    constexpr int TX = PIC_YEE_TX;
    static_assert(TX == 64, "one lane per column");
    constexpr int WX = TX + (CK ? 5 : 3), WZ = TZ + (CK ? 5 : 3), WN = WX * WZ;
    // local ranges (local = global + 2): lambda_E' on [1, EH), lambda_B'' on [1, BH)
    constexpr int EHX = TX + (CK ? 4 : 3), EHZ = TZ + (CK ? 4 : 3);
    constexpr int BHX = TX + (CK ? 3 : 2), BHZ = TZ + (CK ? 3 : 2);
    __shared__ R sE[3][WN], sB[3][WN];
    const int item = blockIdx.x / SPLIT, part = blockIdx.x % SPLIT;
    const int inst = work[item].x, t = work[item].y;
    const InstDesc &D = Dt[inst];
    const int nx = D.n[0], nz = D.n[2];
    const int ntx = (nx + TX - 1) / TX;
    const int x0 = (t % ntx) * TX, z0 = (t / ntx) * (TZ * SPLIT) + part * TZ;
    const int lane = threadIdx.x & 63, wave = wave_id(), nwave = blockDim.x >> 6;
    // inputs: lambda_E, lambda_B as left in T1 by the reverse seen kernels
    const gp<const R> in[6] = {G<R>((const void *)D.T1[0]), G<R>((const void *)D.T1[1]), G<R>((const void *)D.T1[2]),
                               G<R>((const void *)D.T1[3]), G<R>((const void *)D.T1[4]), G<R>((const void *)D.T1[5])};
    gp<R> lE[3] = {G<R>(D.lE[0]), G<R>(D.lE[1]), G<R>(D.lE[2])};
    gp<R> lB[3] = {G<R>(D.lB[0]), G<R>(D.lB[1]), G<R>(D.lB[2])};
    gp<R> lJ[3] = {G<R>(D.lJ[0]), G<R>(D.lJ[1]), G<R>(D.lJ[2])};
    const bool hasb = lane < WX - TX;
    const int gxa = wrap_near(x0 - 2 + lane, nx);
    const int gxb = hasb ? wrap_near(x0 - 2 + TX + lane, nx) : gxa;
    constexpr int RW = (WZ + 3) / 4;
    for (int r0 = wave; r0 < WZ; r0 += RW * nwave) {
        R v[RW][2][6];
#pragma unroll
        for (int u = 0; u < RW; u++) {
            const int row = min(r0 + u * nwave, WZ - 1);
            const int base = wrap_near(z0 - 2 + row, nz) * nx;
#pragma unroll
            for (int hh = 0; hh < 2; hh++)
#pragma unroll
                for (int k = 0; k < 6; k++) v[u][hh][k] = in[k][base + (hh ? gxb : gxa)];
        }
#pragma unroll
        for (int u = 0; u < RW; u++) {
            const int row = r0 + u * nwave;
            if (row >= WZ) continue;
#pragma unroll
            for (int hh = 0; hh < 2; hh++) {
                if (hh == 1 && !hasb) continue;
                const int c = row * WX + (hh ? TX : 0) + lane;
#pragma unroll
                for (int k = 0; k < 3; k++) { sE[k][c] = v[u][hh][k]; sB[k][c] = v[u][hh][3 + k]; }
            }
        }
    }
    __syncthreads();
    const R idx = R(1) / (R)D.d[0], idz = R(1) / (R)D.d[2], dt = (R)D.dt, h = R(0.5) * dt;
    // transposed Faraday differences at window cell e: backward, CK-averaged across
    auto bdx = [&](const R *F, int e) {
        if constexpr (CK)
            return (R(0.75) * (F[e] - F[e - 1]) +
                    R(0.125) * ((F[e - WX] - F[e - WX - 1]) + (F[e + WX] - F[e + WX - 1]))) * idx;
        else
            return (F[e] - F[e - 1]) * idx;
    };
    auto bdz = [&](const R *F, int e) {
        if constexpr (CK)
            return (R(0.75) * (F[e] - F[e - WX]) +
                    R(0.125) * ((F[e - 1] - F[e - 1 - WX]) + (F[e + 1] - F[e + 1 - WX]))) * idz;
        else
            return (F[e] - F[e - WX]) * idz;
    };
    // The two halo phases cover a few more columns than the 64 lanes: their
    // (row, column) cells are dealt out to the block's threads in order.
    // lE' on local [1, EH) (cells -1 .. T, or T + 1 with CK): transposed Faraday of lB
    constexpr int C1 = EHX - 1, N1 = (EHZ - 1) * C1;
    for (int it = threadIdx.x; it < N1; it += blockDim.x) {
        const int e = (1 + it / C1) * WX + 1 + it % C1;
        const R cx = -bdz(sB[1], e);
        const R cy = bdz(sB[0], e) - bdx(sB[2], e);
        const R cz = bdx(sB[1], e);
        sE[0][e] -= h * cx;
        sE[1][e] -= h * cy;
        sE[2][e] -= h * cz;
    }
    __syncthreads();
    // lB' on local [1, BH) (cells -1 .. T - 1, or T with CK): forward differences of lE'
    constexpr int C2 = BHX - 1, N2 = (BHZ - 1) * C2;
    for (int it = threadIdx.x; it < N2; it += blockDim.x) {
        const int e = (1 + it / C2) * WX + 1 + it % C2, exp = e + 1, ezp = e + WX;
        const R fx = -(sE[1][ezp] - sE[1][e]) * idz;
        const R fy = (sE[0][ezp] - sE[0][e]) * idz - (sE[2][exp] - sE[2][e]) * idx;
        const R fz = (sE[1][exp] - sE[1][e]) * idx;
        sB[0][e] += dt * fx;
        sB[1][e] += dt * fy;
        sB[2][e] += dt * fz;
    }
    __syncthreads();
    const int gx = x0 + lane;
    if (gx >= nx) return;
    for (int lz = wave; lz < TZ; lz += nwave) {
        const int gz = z0 + lz;
        if (gz >= nz) break;
        const int e = (lz + 2) * WX + lane + 2;
        const R cx = -bdz(sB[1], e);
        const R cy = bdz(sB[0], e) - bdx(sB[2], e);
        const R cz = bdx(sB[1], e);
        const int g = gz * nx + gx;
        lJ[0][g] = -dt * sE[0][e]; lJ[1][g] = -dt * sE[1][e]; lJ[2][g] = -dt * sE[2][e];
        lE[0][g] = sE[0][e] - h * cx;
        lE[1][g] = sE[1][e] - h * cy;
        lE[2][g] = sE[2][e] - h * cz;
        lB[0][g] = sB[0][e]; lB[1][g] = sB[1][e]; lB[2][g] = sB[2][e];
        // lambda_Et, lambda_Bt were consumed by the reverse seen kernels: clear
        // them for the next reverse particle step
#pragma unroll
        for (int k = 0; k < 3; k++) { G<R>(D.lEt[k])[g] = R(0); G<R>(D.lBt[k])[g] = R(0); }
    }
}

inline int hip_ok(hipError_t e) { return e == hipSuccess ? 0 : -1; }

}  // namespace

#define DISPATCH_R(fp32, ...) \
    do { if (fp32) { typedef float R; __VA_ARGS__; } else { typedef double R; __VA_ARGS__; } } while (0)

size_t adjoint_smem_bytes(int dims, int fp32, const int wmax[3])
{
    const size_t wc = (size_t)wmax[0] * (dims == 3 ? wmax[1] : 1) * wmax[2];
    return adj_lf_offset(wc, fp32 ? 4 : 8) + 6 * wc * sizeof(double);
}

int launch_adj_seed(const LaunchCtx &c, const int2 *fwork, int nfwork, const int2 *cwork, int ncwork)
{
    DISPATCH_R(c.fp32, {
        if (nfwork > 0) k_adj_seed<R><<<dim3(nfwork), dim3(PIC_FIELD_CHUNK), 0, c.stream>>>(c.desc, fwork, c.par);
        if (ncwork > 0) k_adj_seed_particles<R><<<dim3(ncwork), dim3(PIC_PART_CHUNK), 0, c.stream>>>(c.desc, cwork);
    });
    return hip_ok(hipGetLastError());
}

// Reverse of one step.  `tape` addresses this step's E1, B2, particles and
// tile boxes; `live` the shared planes (identical for everything else).
size_t adj_seen_smem_bytes(int fp32)
{
    // worst case z halo: Psi degree + filter passes (GRAD) or the combined
    // stencil, both at most PIC_MAX_HZ; x halo PIC_MAX_HX
    const int wx = ADJ_TX + 2 * PIC_MAX_HX, wz = PIC_ADJ_TZ + 2 * PIC_MAX_HZ;
    return (size_t)(wx * wz + ADJ_TX * wz + 2 * PIC_MAX_HZ + 1 + 2 * PIC_MAX_HX + 1) * (fp32 ? 4 : 8);
}

int launch_adj_step(const LaunchCtx &live, const LaunchCtx &tape, const int2 *fwork, int nfwork, const int2 *swork,
                    int nswork, const int2 *awork, int nawork, const int2 *pwork, int npwork, int block,
                    const int wmax[3])
{
    // Et, Bt of this step: recorded in the tape slot in 2D, recomputed in 3D
    if (live.dims == 3 && launch_seen(tape, fwork, nfwork, swork, nswork)) return -1;
    const int wm[3] = {wmax[0], live.dims == 3 ? wmax[1] : 1, wmax[2]};
    const size_t smem = adjoint_smem_bytes(live.dims, live.fp32, wm);
    const dim3 gf(nfwork), g6(nfwork, 6), g2(nfwork, 2), bf(PIC_FIELD_CHUNK);
    hipStream_t st = live.stream;
#define AK(D_, L_)                                                                                             \
    do {                                                                                                       \
        if (live.gather == GATHER_UNIFORM)                                                                     \
            k_adj_particles<D_, L_, R, GATHER_UNIFORM><<<dim3(npwork), dim3(block), smem, st>>>(tape.desc, pwork, \
                                                                                              npwork, wm[0], wm[1], wm[2]); \
        else                                                                                                   \
            k_adj_particles<D_, L_, R, GATHER_GALERKIN><<<dim3(npwork), dim3(block), smem, st>>>(tape.desc, pwork, \
                                                                                               npwork, wm[0], wm[1], wm[2]); \
    } while (0)
    DISPATCH_R(live.fp32, {
        // 2D: the reverse Yee kernel of the previous reverse step (or the seed)
        // left lambda_Et, lambda_Bt zero
        if (live.dims == 3) k_zero_lseen<R><<<gf, bf, 0, st>>>(live.desc, fwork);
        if (npwork > 0) {
            if (live.dims == 2 && live.order == 1) AK(2, 1);
            else if (live.dims == 2 && live.order == 3) AK(2, 3);
            else if (live.dims == 3 && live.order == 1) AK(3, 1);
            else AK(3, 3);
        }
        if (live.dims == 2) {
            // fused LDS kernels on 64 x 8 tiles (the awork list)
            const size_t sm = adj_seen_smem_bytes(live.fp32);
            const dim3 g6a(nawork, 6);
            // the tape descriptors share every adjoint plane with the live ones
            if (live.hz == 8 && live.hx == 4 && live.psi_deg == 4 && live.hzf == 4)
                // correction of degree 4 with four filter passes: z filter 4, combined 8
                k_adj_seen_2d<R, PIC_ADJ_TZ, 4, 4, 4, 8><<<g6a, bf, sm, st>>>(tape.desc, awork);
            else
                k_adj_seen_2d<R, PIC_ADJ_TZ, -1, -1, -1, -1><<<g6a, bf, sm, st>>>(tape.desc, awork);
            // reverse Yee on half tiles (64 x 4 rows): twice the blocks
            if (live.ck) k_adj_yee_2d<R, PIC_ADJ_TZ / 2, true, 2><<<dim3(2 * nawork), bf, 0, st>>>(live.desc, awork);
            else k_adj_yee_2d<R, PIC_ADJ_TZ / 2, false, 2><<<dim3(2 * nawork), bf, 0, st>>>(live.desc, awork);
        } else {
            // lambda_E += M_E lambda_Et, lambda_B += M_B lambda_Bt
            k_pass<2, R><<<g6, bf, 0, st>>>(live.desc, fwork, PL_LSEEN, PL_T1, 0, 0);
            k_pass<0, R><<<g6, bf, 0, st>>>(live.desc, fwork, PL_T1, PL_T2, 0, 0);
            k_pass<1, R><<<g6, bf, 0, st>>>(live.desc, fwork, PL_T2, PL_LEB, 0, 1);
            // gradient: F lambda_Et_c (filter only), then <S^j ., E1_c>
            k_pass<2, R><<<g2, bf, 0, st>>>(live.desc, fwork, PL_LSEEN, PL_T1, 1, 0);
            k_pass<0, R><<<g2, bf, 0, st>>>(live.desc, fwork, PL_T1, PL_T2, 0, 0);
            k_pass<1, R><<<g2, bf, 0, st>>>(live.desc, fwork, PL_T2, PL_T1, 0, 0);
            k_adj_grad<R><<<g2, bf, 0, st>>>(tape.desc, fwork, PL_T1);
            // transposed Yee
            k_adj_yee_e<3, R><<<gf, bf, 0, st>>>(live.desc, fwork);
            k_adj_yee_b<3, R><<<gf, bf, 0, st>>>(live.desc, fwork);
            k_adj_yee_e<3, R><<<gf, bf, 0, st>>>(live.desc, fwork);
        }
    });
#undef AK
    return hip_ok(hipGetLastError());
}
