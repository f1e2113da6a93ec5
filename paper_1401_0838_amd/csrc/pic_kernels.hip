// HIP kernels (gfx950) of one FDTD-Esirkepov PIC step with the small-k_z
// correction stencils of Godfrey & Vay (arXiv:1401.0838).
//
//   yee        B half step, E full step, B half step (textbook Yee on the
//              staggered mesh, Sec. 2).  E, B and J alternate between two sets of
//              planes: a step reads set p and writes set p ^ 1 (and clears that
//              set's J for the deposit), so no plane is written while other
//              workgroups read it as halo.  2D: one LDS tile kernel; 3D: sweeps.
//   seen       combined z stencil (Psi(S_z) of Sec. 2 composed with the z filter
//              passes of Sec. 3 / Eq. 6), then x (then y): one LDS tile kernel
//              per component in 2D, separable passes in 3D
//   particles  one workgroup per particle tile: stage the seen fields of the
//              tile's bounding window (plus guard cells) in LDS, then per
//              particle Galerkin gather (Eq. 3 scheme), Boris push, move and
//              Esirkepov deposit into an LDS current window; flush the window
//              with global atomics
//   resort     counting sort of particles by tile when a tile's bounding box
//              has outgrown its LDS window
//   diag       float64 wavefront-shuffle reductions for energies, charge and
//              the Gauss-law residual
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <type_traits>

#include "pic_internal.h"
#include "pic_device.h"

namespace {

using namespace pic;

// Galerkin interpolation (Eq. 3 scheme) of one component with staggering (SX,
// SY, SZ): order l, lowered by one along half-staggered axes.
template <int SX, int SY, int SZ, int DIM, int L, class R, class Win>
__device__ __forceinline__ R interp(const Win &W, int comp, const int *lc, const R (*wi)[L + 1],
                                    const R (*wh)[L])
{
    constexpr int H = (L - 1) / 2;
    constexpr int NX = L + 1 - SX, NZ = L + 1 - SZ, NY = DIM == 3 ? L + 1 - SY : 1;
    // sums start from their first term (not from zero: an addition of zero is
    // an instruction the compiler may not drop)
    R s;
#pragma unroll
    for (int kz = 0; kz < NZ; kz++) {
        R wz;
        if constexpr (SZ) wz = wh[2][kz]; else wz = wi[2][kz];
#pragma unroll
        for (int ky = 0; ky < NY; ky++) {
            R wy = R(1);
            if constexpr (DIM == 3) {
                if constexpr (SY) wy = wh[1][ky]; else wy = wi[1][ky];
            }
            R row;
#pragma unroll
            for (int kx = 0; kx < NX; kx++) {
                R wx;
                if constexpr (SX) wx = wh[0][kx]; else wx = wi[0][kx];
                const R t = wx * W.f(comp, lc[0] - H + kx, DIM == 3 ? lc[1] - H + ky : 0, lc[2] - H + kz);
                row = kx == 0 ? t : row + t;
            }
            const R t = wy * wz * row;
            s = (kz == 0 && ky == 0) ? t : s + t;
        }
    }
    return s;
}

// Order-l interpolation of one component on every axis: the weights w[a][0..L]
// apply to the window cells b[a] .. b[a] + L.
template <int DIM, int L, class R, class Win>
__device__ __forceinline__ R interp_l(const Win &W, int comp, const int *b, const R *wx, const R *wy, const R *wz)
{
    constexpr int NY = DIM == 3 ? L + 1 : 1;
    R s;
#pragma unroll
    for (int kz = 0; kz <= L; kz++) {
#pragma unroll
        for (int ky = 0; ky < NY; ky++) {
            R row;
#pragma unroll
            for (int kx = 0; kx <= L; kx++) {
                const R t = wx[kx] * W.f(comp, b[0] + kx, DIM == 3 ? b[1] + ky : 0, b[2] + kz);
                row = kx == 0 ? t : row + t;
            }
            const R t = (DIM == 3 ? wy[ky] : R(1)) * wz[kz] * row;
            s = (kz == 0 && ky == 0) ? t : s + t;
        }
    }
    return s;
}

// Uniform interpolation (Eq. 4 scheme) of a component with staggering (SX, SY,
// SZ): order l from its own Yee location, i.e. along a half-staggered axis the
// weights wu of the coordinate shifted by half a cell, from window cell bu.
template <int SX, int SY, int SZ, int DIM, int L, class R, class Win>
__device__ __forceinline__ R interp_u(const Win &W, int comp, const int *bi, const int *bu, const R (*wi)[L + 1],
                                      const R (*wu)[L + 1])
{
    const int b[3] = {SX ? bu[0] : bi[0], SY ? bu[1] : bi[1], SZ ? bu[2] : bi[2]};
    return interp_l<DIM, L, R>(W, comp, b, SX ? wu[0] : wi[0], SY ? wu[1] : wi[1], SZ ? wu[2] : wi[2]);
}

// The six seen-field components at one particle with gather scheme IP.
template <int DIM, int L, int IP, class R, class Win>
__device__ __forceinline__ void gather6(const Win &W, const int *lc, const R *off, R *Ev, R *Bv)
{
    constexpr int H = (L - 1) / 2;
    R wi[3][L + 1];
    int bi[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        bi[a] = lc[a] - H;
        if (DIM == 2 && a == 1) continue;
        Shape<L, R>::integer(off[a], wi[a]);
    }
    // staggering: Ex(1,0,0) Ey(0,1,0) Ez(0,0,1) Bx(0,1,1) By(1,0,1) Bz(1,1,0)
    if constexpr (IP == GATHER_GALERKIN) {
        R wh[3][L];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (DIM == 2 && a == 1) continue;
            Shape<L, R>::half(off[a], wh[a]);
        }
        Ev[0] = interp<1, 0, 0, DIM, L, R>(W, 0, lc, wi, wh);
        Ev[1] = interp<0, 1, 0, DIM, L, R>(W, 1, lc, wi, wh);
        Ev[2] = interp<0, 0, 1, DIM, L, R>(W, 2, lc, wi, wh);
        Bv[0] = interp<0, 1, 1, DIM, L, R>(W, 3, lc, wi, wh);
        Bv[1] = interp<1, 0, 1, DIM, L, R>(W, 4, lc, wi, wh);
        Bv[2] = interp<1, 1, 0, DIM, L, R>(W, 5, lc, wi, wh);
    } else if constexpr (IP == GATHER_UNIFORM) {
        // half-staggered samples sit at cell + 1/2: the shifted coordinate's cell
        // is this one when off >= 1/2, else the one below
        R wu[3][L + 1];
        int bu[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            bu[a] = bi[a];
            if (DIM == 2 && a == 1) continue;
            const bool up = off[a] >= R(0.5);
            bu[a] -= up ? 0 : 1;
            Shape<L, R>::integer(up ? off[a] - R(0.5) : off[a] + R(0.5), wu[a]);
        }
        Ev[0] = interp_u<1, 0, 0, DIM, L, R>(W, 0, bi, bu, wi, wu);
        Ev[1] = interp_u<0, 1, 0, DIM, L, R>(W, 1, bi, bu, wi, wu);
        Ev[2] = interp_u<0, 0, 1, DIM, L, R>(W, 2, bi, bu, wi, wu);
        Bv[0] = interp_u<0, 1, 1, DIM, L, R>(W, 3, bi, bu, wi, wu);
        Bv[1] = interp_u<1, 0, 1, DIM, L, R>(W, 4, bi, bu, wi, wu);
        Bv[2] = interp_u<1, 1, 0, DIM, L, R>(W, 5, bi, bu, wi, wu);
    } else {
        // momentum-conserving (Eq. 5 scheme): the seen fields were averaged onto
        // the integer nodes, so every component shares one weight set
#pragma unroll
        for (int k = 0; k < 3; k++) {
            Ev[k] = interp_l<DIM, L, R>(W, k, bi, wi[0], wi[1], wi[2]);
            Bv[k] = interp_l<DIM, L, R>(W, 3 + k, bi, wi[0], wi[1], wi[2]);
        }
    }
}

// One particle: gather, Boris, move, Esirkepov deposit.
// lc: window-local cell; off: in-cell offsets; u: momenta (updated);
// dc / offn: cell step and new offsets (outputs).
template <int DIM, int L, class R, class JT, int IP, class Win>
__device__ __forceinline__ void push_particle(Win &W, const int *lc, const R *off, R *u, int *dc, R *offn,
                                              const R *dtd, R qdt2m, const R *cdep, R cy2d, int &err)
{
    constexpr int H = (L - 1) / 2;
    R Ev[3], Bv[3];
    gather6<DIM, L, IP, R>(W, lc, off, Ev, Bv);

    // Boris (textbook): half electric kick, magnetic rotation, half kick; then move
    R un[3];
    BorisTrace<R> bt;
    boris_push<R>(u, Ev, Bv, qdt2m, un, bt);
    const R ig = move_cells<DIM, R>(off, un, dtd, dc, offn, err);
    u[0] = un[0]; u[1] = un[1]; u[2] = un[2];

    // Esirkepov: shapes on the L+2 nodes starting at min(old, new) cell - H
    R S0[3][L + 2], DS[3][L + 2];
    int base[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (DIM == 2 && a == 1) { base[a] = 0; continue; }
        R w0[L + 1], w1[L + 1];
        Shape<L, R>::integer(off[a], w0);
        Shape<L, R>::integer(offn[a], w1);
        const int mn = dc[a] < 0 ? -1 : 0;
        const bool sh0 = mn < 0;          // old support starts one node in
        const bool sh1 = dc[a] > 0;       // new support starts one node in
        base[a] = lc[a] + mn - H;
#pragma unroll
        for (int i = 0; i < L + 2; i++) {
            // node i of the (L+2)-node stencil; supports are L+1 nodes, shifted by one
            // when the particle's cell is the upper of old / new
            const R lo0 = i >= 1 ? w0[i >= 1 ? i - 1 : 0] : R(0), hi0 = i < L + 1 ? w0[i < L + 1 ? i : L] : R(0);
            const R lo1 = i >= 1 ? w1[i >= 1 ? i - 1 : 0] : R(0), hi1 = i < L + 1 ? w1[i < L + 1 ? i : L] : R(0);
            const R a0 = sh0 ? lo0 : hi0;
            const R a1 = sh1 ? lo1 : hi1;
            S0[a][i] = a0;
            DS[a][i] = a1 - a0;
        }
    }
    JT *tag = nullptr;
    if constexpr (DIM == 2) {
        // A particle that stays in its cell along an axis has old and new shapes on
        // the first L + 1 of the L + 2 nodes, so everything it deposits on the last
        // node of that axis is zero, and so is the running sum of its shape change
        // up to node L (the changes sum to zero; the sum left at node L is rounding
        // only).  When no lane of the wave changed cell along the axis, the wave
        // skips those updates (whole LDS atomics, not just lanes).
        const bool lastx = __ballot(dc[0] != 0) != 0, lastz = __ballot(dc[2] != 0) != 0;
        // the running sums use the shape changes with the deposit constant
        // folded in (one multiply per node instead of one per update)
        R cx[L + 1], cz[L + 1];
#pragma unroll
        for (int i = 0; i < L + 1; i++) { cx[i] = cdep[0] * DS[0][i]; cz[i] = cdep[2] * DS[2][i]; }
        // J_x: running sum along x
#pragma unroll
        for (int k = 0; k < L + 2; k++) {
            if (k == L + 1 && !lastz) break;
            R tz = S0[2][k] + R(0.5) * DS[2][k];
            R acc;
#pragma unroll
            for (int i = 0; i < L + 1; i++) {
                if (i == L && !lastx) break;
                acc = i == 0 ? cx[i] * tz : acc + cx[i] * tz;
                // exactly zero (not a rounding residue) for a particle that kept its
                // x cell, so the result does not depend on which lanes share a wave
                const R v = (i == L && dc[0] == 0) ? R(0) : acc;
                W.add(0, base[0] + i, 0, base[2] + k, jcvt(v, tag));
            }
        }
        // J_z: running sum along z
#pragma unroll
        for (int i = 0; i < L + 2; i++) {
            if (i == L + 1 && !lastx) break;
            R tx = S0[0][i] + R(0.5) * DS[0][i];
            R acc;
#pragma unroll
            for (int k = 0; k < L + 1; k++) {
                if (k == L && !lastz) break;
                acc = k == 0 ? cz[k] * tx : acc + cz[k] * tx;
                const R v = (k == L && dc[2] == 0) ? R(0) : acc;
                W.add(2, base[0] + i, 0, base[2] + k, jcvt(v, tag));
            }
        }
        // J_y: out of plane, with v_y.  W_y = S0x (S0z/3 + S1z/6) + S1x (S0z/6 + S1z/3)
        // with S1 = S0 + dS is S0x (S0z + dSz/2) + dSx (S0z/2 + dSz/3): two
        // factors per z node, two operations per node
        const R cy = cy2d * u[1] * ig, cy2 = R(0.5) * cy, cy3 = R(1.0 / 3.0) * cy;
#pragma unroll
        for (int k = 0; k < L + 2; k++) {
            if (k == L + 1 && !lastz) break;
            const R pz = cy * S0[2][k] + cy2 * DS[2][k];
            const R qz = cy2 * S0[2][k] + cy3 * DS[2][k];
#pragma unroll
            for (int i = 0; i < L + 2; i++) {
                if (i == L + 1 && !lastx) break;
                const R wy = S0[0][i] * pz + DS[0][i] * qz;
                W.add(1, base[0] + i, 0, base[2] + k, jcvt(wy, tag));
            }
        }
    } else {
        // same skips as in 2D, per axis (see above)
        const bool last[3] = {__ballot(dc[0] != 0) != 0, __ballot(dc[1] != 0) != 0, __ballot(dc[2] != 0) != 0};
        // shape changes with the deposit constant folded in, for the running sums
        R cd[3][L + 1];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int i = 0; i < L + 1; i++) cd[a][i] = cdep[a] * DS[a][i];
        // J_x (outer loops stay rolled for cubic shapes to bound register use)
        constexpr int UNROLL_OUTER = L == 1 ? L + 2 : 1;
#pragma unroll UNROLL_OUTER
        for (int kz = 0; kz < L + 2; kz++) {
            if (kz == L + 1 && !last[2]) break;
            // the transverse weight S0y S0z + (dSy S0z + S0y dSz) / 2 + dSy dSz / 3,
            // grouped as S0y az + dSy bz with az, bz once per z node
            const R az = S0[2][kz] + R(0.5) * DS[2][kz], bz = R(0.5) * S0[2][kz] + R(1.0 / 3.0) * DS[2][kz];
#pragma unroll
            for (int ky = 0; ky < L + 2; ky++) {
                if (ky == L + 1 && !last[1]) break;
                const R tr = S0[1][ky] * az + DS[1][ky] * bz;
                R acc;
#pragma unroll
                for (int kx = 0; kx < L + 1; kx++) {
                    if (kx == L && !last[0]) break;
                    acc = kx == 0 ? cd[0][kx] * tr : acc + cd[0][kx] * tr;
                    const R v = (kx == L && dc[0] == 0) ? R(0) : acc;
                    W.add(0, base[0] + kx, base[1] + ky, base[2] + kz, jcvt(v, tag));
                }
            }
        }
        // J_y
#pragma unroll UNROLL_OUTER
        for (int kz = 0; kz < L + 2; kz++) {
            if (kz == L + 1 && !last[2]) break;
            const R az = S0[2][kz] + R(0.5) * DS[2][kz], bz = R(0.5) * S0[2][kz] + R(1.0 / 3.0) * DS[2][kz];
#pragma unroll
            for (int kx = 0; kx < L + 2; kx++) {
                if (kx == L + 1 && !last[0]) break;
                const R tr = S0[0][kx] * az + DS[0][kx] * bz;
                R acc;
#pragma unroll
                for (int ky = 0; ky < L + 1; ky++) {
                    if (ky == L && !last[1]) break;
                    acc = ky == 0 ? cd[1][ky] * tr : acc + cd[1][ky] * tr;
                    const R v = (ky == L && dc[1] == 0) ? R(0) : acc;
                    W.add(1, base[0] + kx, base[1] + ky, base[2] + kz, jcvt(v, tag));
                }
            }
        }
        // J_z
#pragma unroll UNROLL_OUTER
        for (int ky = 0; ky < L + 2; ky++) {
            if (ky == L + 1 && !last[1]) break;
            const R ay = S0[1][ky] + R(0.5) * DS[1][ky], by = R(0.5) * S0[1][ky] + R(1.0 / 3.0) * DS[1][ky];
#pragma unroll
            for (int kx = 0; kx < L + 2; kx++) {
                if (kx == L + 1 && !last[0]) break;
                const R tr = S0[0][kx] * ay + DS[0][kx] * by;
                R acc;
#pragma unroll
                for (int kz = 0; kz < L + 1; kz++) {
                    if (kz == L && !last[2]) break;
                    acc = kz == 0 ? cd[2][kz] * tr : acc + cd[2][kz] * tr;
                    const R v = (kz == L && dc[2] == 0) ? R(0) : acc;
                    W.add(2, base[0] + kx, base[1] + ky, base[2] + kz, jcvt(v, tag));
                }
            }
        }
    }
}

// ------------------------------------------------------------ particle kernel

// P > 0: LDS windows with compile-time pitches.  2D: row pitch P, plane P*P.
// 3D: P = PX * 10000 + PY * 100 + PZ (cells per row, rows per plane, planes).
// PF: load the next particle's state while the current one is processed.
// TP: also write the state each particle starts from, and each tile's box,
// to the tape slot named by the descriptor (reverse sweep recompute).
// MODE: how a tile whose particle box has outgrown the LDS window is stepped
// (fields read and current added straight in global memory).
//   PM_INLINE  in this kernel, on a branch of the particle loop;
//   PM_DEFER   not here: the tile goes on a list for a second launch, so the
//              global-memory code and its registers stay out of this kernel
//              (more waves per SIMD; pays off when tiles outnumber the slots);
//   PM_GLOBAL  that second launch: the listed tiles only.
enum { PM_INLINE = 0, PM_DEFER = 1, PM_GLOBAL = 2 };
template <int DIM, int L, class R, int P, bool PF, bool TP = false, int IP = GATHER_GALERKIN, int MODE = PM_INLINE>
__device__ __forceinline__ void particles_body(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                               int nwork, int wmx, int wmy, int wmz, int par,
                                               const int *__restrict__ dlist = nullptr)
{
    // LDS current sums: 64-bit fixed point in float mode (2D), 32-bit with a
    // per-tile quantum in 3D float (half the LDS traffic of the deposit's adds),
    // double in FP64
    typedef std::conditional_t<DIM == 3 && std::is_same<R, float>::value, int, typename JOf<R>::T> JT;
    typedef typename JGOf<R>::T JG;
    constexpr bool J32 = std::is_same<JT, int>::value;
    constexpr int JL = (L + 1) / 2;      // guard cells below the bounding box
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int sbox[6];
    const int tid = threadIdx.x, bs = blockDim.x;
    constexpr bool SLOW = MODE == PM_GLOBAL;
    // the deferred list is shared by all instances; its count was final when
    // the deferring launch ended (the second launch gets its address as an
    // argument: one dependent load fewer before the usual empty exit)
    const int *dfr = dlist ? dlist : Dt[0].defer;
    if constexpr (SLOW) {
        nwork = __hip_atomic_load(const_cast<int *>(dfr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // nothing deferred (the usual case): the list is already empty, so no
        // block needs to count itself done
        if (nwork == 0) return;
    }

    for (int item = blockIdx.x; item < nwork; item += gridDim.x) {
        // work == nullptr: one instance, slot -> tile in the host's XCD order
        int inst, tile;
        if constexpr (SLOW) {
            inst = dfr[2 + 2 * item];
            tile = dfr[3 + 2 * item];
        } else {
            inst = work ? work[item].x : 0;
        }
        const InstDesc &D = Dt[inst];
        if constexpr (!SLOW) tile = work ? work[item].y : xcd_tile(item, D.ntiles);
        // the tile's range is uniform: kept in scalar registers, so are the
        // per-pass array bases derived from it
        const int p0 = __builtin_amdgcn_readfirstlane(D.tstart[tile]);
        const int p1 = __builtin_amdgcn_readfirstlane(D.tstart[tile + 1]);
        if (p1 <= p0) continue;
        int lo[3], ext[3], o[3], wn[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = D.tbox[tile * 6 + a];
            ext[a] = D.tbox[tile * 6 + 3 + a];
            if (DIM == 2 && a == 1) { o[a] = 0; wn[a] = 1; continue; }
            o[a] = wrapi(lo[a] - JL, D.n[a]);
            wn[a] = ext[a] + L + 2;
        }
        if constexpr (TP) {
            if (tid < 6) D.rtbox[tile * 6 + tid] = tid < 3 ? lo[tid] : ext[tid - 3];
        }
        // PM_DEFER leaves a tile whose window does not fit to the PM_GLOBAL
        // launch, which takes only such tiles
        const bool fits = !SLOW && wn[0] <= wmx && wn[1] <= wmy && wn[2] <= wmz;
        if (!fits && MODE == PM_INLINE && tid == 0) {
            atomicAdd(&D.flags[FLAG_SLOW], 1);
            atomicExch(&D.flags[FLAG_RESORT], 1);
            atomicExch(D.any_resort, 1);
        }
        if (!fits && MODE == PM_DEFER) {
            if (tid == 0) {
                atomicAdd(&D.flags[FLAG_SLOW], 1);
                atomicExch(&D.flags[FLAG_RESORT], 1);
                atomicExch(D.any_resort, 1);
                const int k = atomicAdd(D.defer, 1);
                D.defer[2 + 2 * k] = inst;
                D.defer[3 + 2 * k] = tile;
            }
            continue;
        }
        // plane stride and row pitch of the LDS windows
        constexpr int PXc = DIM == 2 ? P : P / 10000, PYc = DIM == 2 ? 1 : (P / 100) % 100;
        constexpr int PZc = DIM == 2 ? P : P % 100;
        const int wc = P > 0 ? PXc * PYc * PZc : wn[0] * wn[1] * wn[2];
        const int pitch = P > 0 ? PXc : wn[0];
        // window cell c (x fastest over wn) -> its LDS slot.  The quotients are
        // taken with a float reciprocal, (c + 1/2) / w rounded down, which is
        // exact for c below 2^22 (windows hold a few thousand cells) and costs a
        // few instructions where an integer division costs a few tens
        // (the reciprocals are uniform: kept in scalar registers across the loop)
        const float rw0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(1.0f / (float)wn[0])));
        const float rw1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(1.0f / (float)wn[1])));
        auto lslot = [&](int c) {
            if constexpr (P > 0) {
                const int r = (int)(((float)c + 0.5f) * rw0);
                const int x = c - r * wn[0];
                if constexpr (DIM == 2) {
                    return r * PXc + x;
                } else {
                    const int z = (int)(((float)r + 0.5f) * rw1);
                    return ((z * PYc + (r - z * wn[1])) * PXc) + x;
                }
            } else {
                return c;
            }
        };
        JT *sJ = reinterpret_cast<JT *>(smem);
        R *sF = reinterpret_cast<R *>(smem + (size_t)3 * wmx * wmy * wmz * sizeof(JT));

        if (tid < 3) { sbox[tid] = INT_MAX; sbox[3 + tid] = INT_MIN; }
        if (fits) {
            gp<const R> src[6] = {G<R>((const void *)D.Et[0]), G<R>((const void *)D.Et[1]),
                                  G<R>((const void *)D.Et[2]), G<R>((const void *)D.Bt[0]),
                                  G<R>((const void *)D.Bt[1]), G<R>((const void *)D.Bt[2])};
            const int nwin = wn[0] * wn[1] * wn[2];
            for (int c = tid; c < nwin; c += bs) {
                const int g = window_cell(c, wn, o, D.n);
                const int l = lslot(c);
#pragma unroll
                for (int k = 0; k < 6; k++) sF[k * wc + l] = src[k][g];
#pragma unroll
                for (int k = 0; k < 3; k++) sJ[k * wc + l] = JT(0);
            }
        }
        __syncthreads();

        // 32-bit sums count units of jq 2^kq.  Along axis a a contribution is
        // |cdep_a| = |q w| d_a / (c dt dV) times a running sum of shape changes,
        // which is at most the particle's move in cells (|v| dt / d_a < c dt / d_a)
        // times the slope bound of the partial sums of the spline (the peak of the
        // spline one order lower: 1 linear, 3/4 cubic), times a transverse weight
        // (at most the spline's peak squared: 1, 4/9).  So it is below
        // |q w| / dV = |rho_c| for linear and |rho_c| / 3 for cubic splines.  kq is
        // the least that keeps the tile's particles, all adding to one cell, below
        // 2^30 (cubic, 512 particles, c dt / d = 0.5: kq = 5).  A tile stepped in
        // global memory adds each contribution to HBM on its own: kq = 0
        int kq = 0;
        if constexpr (J32) if (fits) {
            const double cmax = (L == 3 ? 1.0 / 3.0 : 1.0) * fabs(D.rho_c) / D.jq;
            const double np_t = (double)(p1 - p0);
            while (kq < 28 && np_t * cmax > ldexp(1.0, 30 + kq)) kq++;
        }
        const R cq = J32 ? (R)ldexpf(1.0f, -kq) : R(1);
        const R dtd[3] = {(R)D.dtd[0], (R)D.dtd[1], (R)D.dtd[2]};
        const R cdep[3] = {(R)D.cdep[0] * cq, (R)D.cdep[1] * cq, (R)D.cdep[2] * cq};
        const R qdt2m = (R)D.qdt2m, cy2d = (R)D.cy2d;
        gp<R> poff[3] = {G<R>(D.poff[0]), G<R>(D.poff[1]), G<R>(D.poff[2])};
        gp<R> pu[3] = {G<R>(D.pu[0]), G<R>(D.pu[1]), G<R>(D.pu[2])};
        gp<unsigned> pidx = G<unsigned>(D.pidx);
        int bmin[3] = {INT_MAX, INT_MAX, INT_MAX}, bmax[3] = {INT_MIN, INT_MIN, INT_MIN};
        // grid extents in registers: the loop's stores could alias the
        // descriptor, so reads of it inside the loop would be repeated (and
        // wait on the scalar cache, and with it on LDS) every pass
        const int nn[3] = {D.n[0], D.n[1], D.n[2]};
        int err = 0;

        LdsWin<R, JT> lw{sF, sJ, pitch, pitch * wn[1], wc};
        LdsWinP<R, JT, (P > 0 ? PXc : 1), (P > 0 ? PYc : 1), (P > 0 ? PZc : 1)> lwp{sF, sJ};
        GlbWin<R, JT> gw;
        gw.ovf = false;
        if (SLOW || (MODE == PM_INLINE && !fits)) {
            for (int k = 0; k < 3; k++) {
                gw.F[k] = G<R>((const void *)D.Et[k]);
                gw.F[3 + k] = G<R>((const void *)D.Bt[k]);
                gw.J[k] = G<JG>(D.J[par][k]);
                gw.o[k] = o[k];
                gw.n[k] = D.n[k];
            }
            gw.shift = D.jshift - kq;
        }

        // The particle state is streamed: read once and written once per step.
        // When the batch's state is larger than the last-level cache (D.nts), its
        // loads and stores are non-temporal and leave the caches to what is
        // reused, the tile windows of the seen fields and the current lines the
        // flush adds to (64-instance batch of 31 M particles: step 0.470 ->
        // 0.433 ms); a state that fits stays cached from one step to the next
        // (512 x 512 x 16 ppc: particle launch 48 us, 57 us non-temporal).  The
        // loop is compiled once for each (NTS).
        // With PF, software pipelining: the next particle's state is loaded
        // while the current one is processed (twice the bytes in flight per wave)
        auto particle_loop = [&](auto nts_tag) {
        constexpr bool NTS = decltype(nts_tag)::value;
        unsigned nidx = 0;
        R noff[3] = {R(0), R(0), R(0)}, nu[3] = {R(0), R(0), R(0)};
        if (PF && p0 + tid < p1) {
            const unsigned b4 = (unsigned)(p0 + tid) * 4u, bR = (unsigned)(p0 + tid) * (unsigned)sizeof(R);
            nidx = sload<NTS>(lane_ptr(pidx, b4));
#pragma unroll
            for (int a = 0; a < 3; a++) {
                if (!(DIM == 2 && a == 1)) noff[a] = sload<NTS>(lane_ptr(poff[a], bR));
                nu[a] = sload<NTS>(lane_ptr(pu[a], bR));
            }
        }
        for (int pb = p0; pb < p1; pb += bs) {
            const int p = pb + tid;
            if (p >= p1) continue;   // last pass only; the loop exit stays uniform
            // per-lane byte offsets (32-bit, zero-extended) from the uniform array
            // bases: the loads and stores take the scalar-base + vector-offset form
            const unsigned b4 = (unsigned)p * 4u, bR = (unsigned)p * (unsigned)sizeof(R);
            if (!PF) {
                nidx = sload<NTS>(lane_ptr(pidx, b4));
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    if (!(DIM == 2 && a == 1)) noff[a] = sload<NTS>(lane_ptr(poff[a], bR));
                    nu[a] = sload<NTS>(lane_ptr(pu[a], bR));
                }
            }
            int c[3];
            unpack_cell<DIM>(nidx, c);
            int lc[3];
            R off[3], u[3], offn[3];
            int dc[3];
            if constexpr (TP) {
                sstore<NTS>(nidx, &G<unsigned>((void *)D.rpidx)[p]);
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    if (!(DIM == 2 && a == 1)) sstore<NTS>(noff[a], &G<R>(D.roff[a])[p]);
                    sstore<NTS>(nu[a], &G<R>(D.ru[a])[p]);
                }
            }
#pragma unroll
            for (int a = 0; a < 3; a++) {
                u[a] = nu[a];
                if (DIM == 2 && a == 1) { lc[a] = 0; off[a] = R(0); continue; }
                int rel = c[a] - lo[a];
                rel += rel < 0 ? nn[a] : 0;
                lc[a] = rel + JL;
                off[a] = noff[a];
            }
            if (PF && p + bs < p1) {
                const unsigned q4 = (unsigned)(p + bs) * 4u, qR = (unsigned)(p + bs) * (unsigned)sizeof(R);
                nidx = sload<NTS>(lane_ptr(pidx, q4));
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    if (!(DIM == 2 && a == 1)) noff[a] = sload<NTS>(lane_ptr(poff[a], qR));
                    nu[a] = sload<NTS>(lane_ptr(pu[a], qR));
                }
            }
            if (!SLOW && (MODE == PM_DEFER || fits)) {
                if constexpr (P > 0) push_particle<DIM, L, R, JT, IP>(lwp, lc, off, u, dc, offn, dtd, qdt2m, cdep, cy2d, err);
                else push_particle<DIM, L, R, JT, IP>(lw, lc, off, u, dc, offn, dtd, qdt2m, cdep, cy2d, err);
            } else if constexpr (MODE != PM_DEFER)
                push_particle<DIM, L, R, JT, IP>(gw, lc, off, u, dc, offn, dtd, qdt2m, cdep, cy2d, err);
            // the store offsets are taken from here as plain 32-bit values (an
            // empty asm the compiler cannot look through), so the stores too get
            // the scalar-base + vector-offset form rather than 64-bit addresses
            // formed before the branches above
            unsigned s4 = b4, sR = bR;
            asm volatile("" : "+v"(s4), "+v"(sR));
            int nc[3];
#pragma unroll
            for (int a = 0; a < 3; a++) {
                nc[a] = c[a];
                if (DIM == 2 && a == 1) continue;
                nc[a] = wrapu(c[a] + dc[a], nn[a]);
                sstore<NTS>(offn[a], lane_ptr(poff[a], sR));
                const int l1 = lc[a] + dc[a];
                bmin[a] = min(bmin[a], l1);
                bmax[a] = max(bmax[a], l1);
            }
#pragma unroll
            for (int a = 0; a < 3; a++) sstore<NTS>(u[a], lane_ptr(pu[a], sR));
            sstore<NTS>(pack_cell<DIM>(nc[0], nc[1], nc[2]), lane_ptr(pidx, s4));
        }
        };
        if (D.nts) particle_loop(std::true_type{});
        else particle_loop(std::false_type{});
        if (err) atomicExch(&D.flags[FLAG_PERR], 1);
        if (gw.ovf) atomicExch(&D.flags[FLAG_JRANGE], 1);
        // bounding box of the moved particles (window-local coordinates)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            int mn = wave_min_i(bmin[a]), mx = wave_max_i(bmax[a]);
            if ((tid & 63) == 0) { atomicMin(&sbox[a], mn); atomicMax(&sbox[3 + a], mx); }
        }
        __syncthreads();
        if (fits) {
            // the window's sums go to HBM (rounded to its coarser quantum in float mode)
            gp<JG> gJ[3] = {G<JG>(D.J[par][0]), G<JG>(D.J[par][1]), G<JG>(D.J[par][2])};
            const int nwin = wn[0] * wn[1] * wn[2];
            if constexpr (sizeof(JG) == 4) {
                // Adds that return nothing (a returning add would make every
                // thread wait for it).  Range check in two parts: a rounded window
                // sum must stay below BND in magnitude (else it is dropped and flagged),
                // and the Yee update, which reads every current word, flags a word
                // outside +-2^30.  At most nine windows (27 in 3D) cover a node, so
                // a word that wrapped past 32 bits lands outside +-2^30.
                // LDS quantum jq 2^kq -> HBM quantum jq 2^jshift (exact when kq >= jshift)
                const int js = D.jshift - kq;
                const long long half = js > 0 ? (1LL << (js - 1)) : 0;
                constexpr long long BND = DIM == 2 ? (1LL << 28) : (1LL << 26);
                bool ovf = false;
                for (int c = tid; c < nwin; c += bs) {
                    const int g = window_cell(c, wn, o, D.n);
                    const int l = lslot(c);
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const long long sv = sJ[k * wc + l];
                        const long long r = js >= 0 ? (sv + half) >> js : sv * (1LL << -js);
                        const bool big = r >= BND || r <= -BND;
                        ovf |= big;
                        if (r != 0 && !big) gatomic_add(gJ[k] + g, (int)r);
                    }
                }
                if (ovf) atomicExch(&D.flags[FLAG_JRANGE], 1);
            } else {
                for (int c = tid; c < nwin; c += bs) {
                    const int g = window_cell(c, wn, o, D.n);
                    const int l = lslot(c);
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        JT v = sJ[k * wc + l];
                        if (v != JT(0)) gatomic_add(gJ[k] + g, v);
                    }
                }
            }
        }
        if (tid == 0) {
            bool regrow = false;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                if (DIM == 2 && a == 1) continue;
                int e = sbox[3 + a] - sbox[a] + 1;
                int l = (o[a] + sbox[a]) % D.n[a];
                l += l < 0 ? D.n[a] : 0;
                if (e >= D.n[a]) { e = D.n[a]; l = 0; }
                D.tbox[tile * 6 + a] = l;
                D.tbox[tile * 6 + 3 + a] = e;
                if (e > D.tile[a] + PIC_TILE_SLACK) regrow = true;
            }
            if (regrow) { atomicExch(&D.flags[FLAG_RESORT], 1); atomicExch(D.any_resort, 1); }
        }
        __syncthreads();
    }
    if constexpr (SLOW) {
        // the last block to finish empties the list for the next step's LDS pass
        // (every block read the count before it counted itself done)
        if (tid == 0) {
            __threadfence();
            int *dw = const_cast<int *>(dfr);
            if (atomicAdd(dw + 1, 1) == (int)gridDim.x - 1) {
                atomicExch(dw, 0);
                atomicExch(dw + 1, 0);
            }
        }
    }
}

template <int DIM, int L, class R, int P, bool PF = false, bool TP = false, int IP = GATHER_GALERKIN,
          int MODE = PM_INLINE>
__global__ void __launch_bounds__(512) k_particles(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                   int nwork, int wmx, int wmy, int wmz, int par)
{
    particles_body<DIM, L, R, P, PF, TP, IP, MODE>(Dt, work, nwork, wmx, wmy, wmz, par);
}

// the tiles a PM_DEFER launch left, in global memory (launched right after it)
template <int DIM, int L, class R, bool TP = false, int IP = GATHER_GALERKIN>
__global__ void __launch_bounds__(256) k_particles_deferred(const InstDesc *__restrict__ Dt, int par,
                                                            const int *__restrict__ dlist)
{
    particles_body<DIM, L, R, 0, false, TP, IP, PM_GLOBAL>(Dt, nullptr, 0, 0, 0, 0, par, dlist);
}

// same body compiled for four waves per SIMD (at most 128 VGPRs); TP: also
// record the tape slot of the reverse sweep
template <int DIM, int L, class R, int P, bool PF = false, bool TP = false>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_particles_w4(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work, int nwork, int wmx, int wmy, int wmz,
               int par)
{
    particles_body<DIM, L, R, P, PF, TP>(Dt, work, nwork, wmx, wmy, wmz, par);
}

// ------------------------------------------------------------- Yee sweeps

template <class R>
__device__ __forceinline__ void cell_ijk(const InstDesc &D, int cell, int &i, int &j, int &k)
{
    i = cell % D.n[0];
    int r = cell / D.n[0];
    j = r % D.n[1];
    k = r / D.n[1];
}

// B[pbo] = B[pbi] - (dt/2) curl E[pe] with forward differences
template <int DIM, class R>
__global__ void __launch_bounds__(256) k_yee_b(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work, int pe,
                                               int pbi, int pbo)
{
    const int inst = work[blockIdx.x].x;
    const InstDesc &D = Dt[inst];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    if (cell >= D.ncell) return;
    int i, j, k;
    cell_ijk<R>(D, cell, i, j, k);
    const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
    const int ip = (i + 1 == nx ? 0 : i + 1) + (j + (k * ny)) * nx;
    const int kp = i + (j + (k + 1 == nz ? 0 : k + 1) * ny) * nx;
    const R *Ex = (const R *)D.E[pe][0], *Ey = (const R *)D.E[pe][1], *Ez = (const R *)D.E[pe][2];
    const R *Bix = (const R *)D.B[pbi][0], *Biy = (const R *)D.B[pbi][1], *Biz = (const R *)D.B[pbi][2];
    R *Bx = (R *)D.B[pbo][0], *By = (R *)D.B[pbo][1], *Bz = (R *)D.B[pbo][2];
    const R idx = R(1) / (R)D.d[0], idz = R(1) / (R)D.d[2];
    const R h = R(0.5) * (R)D.dt;
    const R ex = Ex[cell], ey = Ey[cell], ez = Ez[cell];
    R dyEz = R(0), dyEx = R(0);
    if constexpr (DIM == 3) {
        const int jp = i + ((j + 1 == ny ? 0 : j + 1) + k * ny) * nx;
        const R idy = R(1) / (R)D.d[1];
        dyEz = (Ez[jp] - ez) * idy;
        dyEx = (Ex[jp] - ex) * idy;
    }
    const R dzEy = (Ey[kp] - ey) * idz, dzEx = (Ex[kp] - ex) * idz;
    const R dxEz = (Ez[ip] - ez) * idx, dxEy = (Ey[ip] - ey) * idx;
    Bx[cell] = Bix[cell] - h * (dyEz - dzEy);
    By[cell] = Biy[cell] - h * (dzEx - dxEz);
    Bz[cell] = Biz[cell] - h * (dxEy - dyEx);
}

// E[po] = E[pi] + dt (curl B[po] - J[pi] - J_bg) with backward differences;
// clears J[po] for the coming deposit
template <int DIM, class R>
__global__ void __launch_bounds__(256) k_yee_e(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work, int pi,
                                               int po)
{
    typedef typename JGOf<R>::T JG;
    const int inst = work[blockIdx.x].x;
    const InstDesc &D = Dt[inst];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    if (cell >= D.ncell) return;
    int i, j, k;
    cell_ijk<R>(D, cell, i, j, k);
    const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
    const int im = (i == 0 ? nx - 1 : i - 1) + (j + k * ny) * nx;
    const int km = i + (j + (k == 0 ? nz - 1 : k - 1) * ny) * nx;
    const R *Bx = (const R *)D.B[po][0], *By = (const R *)D.B[po][1], *Bz = (const R *)D.B[po][2];
    const R *Eix = (const R *)D.E[pi][0], *Eiy = (const R *)D.E[pi][1], *Eiz = (const R *)D.E[pi][2];
    R *Ex = (R *)D.E[po][0], *Ey = (R *)D.E[po][1], *Ez = (R *)D.E[po][2];
    const JG *J0 = (const JG *)D.J[pi][0], *J1 = (const JG *)D.J[pi][1], *J2 = (const JG *)D.J[pi][2];
    const R idx = R(1) / (R)D.d[0], idz = R(1) / (R)D.d[2];
    const R dt = (R)D.dt;
    const R bx = Bx[cell], by = By[cell], bz = Bz[cell];
    R dyBz = R(0), dyBx = R(0);
    if constexpr (DIM == 3) {
        const int jm = i + ((j == 0 ? ny - 1 : j - 1) + k * ny) * nx;
        const R idy = R(1) / (R)D.d[1];
        dyBz = (bz - Bz[jm]) * idy;
        dyBx = (bx - Bx[jm]) * idy;
    }
    const R dzBy = (by - By[km]) * idz, dzBx = (bx - Bx[km]) * idz;
    const R dxBz = (bz - Bz[im]) * idx, dxBy = (by - By[im]) * idx;
    const R jx = (R)(jreal(J0[cell], D.jqg) + D.jbg[0]);
    const R jy = (R)(jreal(J1[cell], D.jqg) + D.jbg[1]);
    const R jz = (R)(jreal(J2[cell], D.jqg) + D.jbg[2]);
    if (jrange_bad(J0[cell]) | jrange_bad(J1[cell]) | jrange_bad(J2[cell])) atomicExch(&D.flags[FLAG_JRANGE], 1);
    Ex[cell] = Eix[cell] + dt * (dyBz - dzBy - jx);
    Ey[cell] = Eiy[cell] + dt * (dzBx - dxBz - jy);
    Ez[cell] = Eiz[cell] + dt * (dxBy - dyBx - jz);
#pragma unroll
    for (int c = 0; c < 3; c++) ((JG *)D.J[po][c])[cell] = JG(0);
}

// Fused 2D Yee update: B half step, E step (J read and cleared), B half step
// for a (YEE_TX x TZ) tile in one pass.  LDS windows, in global coordinates
// relative to the tile origin (x0, z0):
//   E^{n-1} on [-1, T+1], B^{n-1} on [-1, T]; J on [0, T] in registers
// B^{n-1/2} is formed on [-1, T], E^n on [0, T], B^n and the stores on [0, T).
// CK: the Cole-Karkkainen curl in Faraday's law (2D, square cells): each
// forward difference of E is the (1/8, 3/4, 1/8) mean of that difference on
// its line and on the two neighbouring lines across it.  The window grows by
// two cells on the low side: E^{n-1} on [-3, T+1], B^{n-1/2} formed on
// [-2, T], E^n on [-1, T].
#define YEE_TX PIC_YEE_TX

template <class R, int TZ, bool CK = false>
__global__ void __launch_bounds__(256) k_yee_2d(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                int nwork, int par)
{
    typedef typename JGOf<R>::T JT;
    constexpr int TX = YEE_TX;
    static_assert(TX == 64, "one lane per column");
    // one window for all nine planes: cells [x0 - LO, x0 + TX + 2) x [z0 - LO, z0 + TZ + 2)
    constexpr int LO = CK ? 3 : 1;
    constexpr int WX = TX + LO + 2, WZ = TZ + LO + 2, WN = WX * WZ;
    // local ranges: B^{n-1/2} on [ELO - 1, EH), E^n on [ELO, EH), the tile on [LO, T + LO)
    constexpr int ELO = CK ? LO - 1 : LO;
    constexpr int EHZ = TZ + LO + 1, EHX = TX + LO + 1;
    // Staging: wave w stages rows w, w + 4, ... of the window's first 64 columns
    // (lane = column; one round: four waves), and the block's first NH threads
    // stage the NHX columns past them, one (row, column) cell each.  J enters
    // only the E step, at the cell itself, so it stays in the staging threads'
    // registers and the same threads form E^n on the cells they staged: no LDS
    // for J.  A wave keeps at most 9 (RW + 1) loads in flight per item, within
    // what its load counter tracks, so the waits below are exact.
    constexpr int RW = (WZ + 3) / 4;   // rows per wave with four waves
    static_assert(RW * 4 >= WZ, "one staging round");
    constexpr int NHX = WX - TX, NH = NHX * WZ;
    static_assert(NH <= 256, "one halo cell per thread");
    // 64 spare words per plane after the window: a lane with no cell to stage
    // stores into its own spare word, so the staging stores have no branches (a
    // branch there makes the compiler wait for every outstanding load,
    // including the next item's)
    __shared__ R sE[3][WN + 64], sB[3][WN + 64];
    const int lane = threadIdx.x & 63, wave = wave_id(), nwave = blockDim.x >> 6;
    const int tid = threadIdx.x;
    const bool hth = tid < NH;                 // this thread stages a halo cell
    const int hrow = hth ? tid / NHX : 0, hcol = TX + (hth ? tid % NHX : 0);
    // One block per item (tile).  Threads share data through LDS only, so the
    // barriers are LDS-only (no wait for outstanding global memory operations).
    // work == nullptr: one instance, item b is tile b in the host's XCD order
    // (saves a dependent load)
    auto tile_of = [&](int item, int &inst, int &t) {
        inst = work ? work[item].x : 0;
        t = work ? work[item].y : xcd_tile(item, nwork);
    };
    R ve[RW][3], vb[RW][3], he[3], hb[3];
    // E, B of an item's window into ve, vb (columns 0..63) and he, hb (halo cell)
    auto load_eb = [&](int item) {
        int inst, t;
        tile_of(item, inst, t);
        const InstDesc &D = Dt[inst];
        const int nx = D.n[0], nz = D.n[2];
        const PerMod wx(nx), wz(nz);
        const int ntx = (nx + TX - 1) / TX;
        const int x0 = (t % ntx) * TX + (nx % TX == 0 ? LO : 0), z0 = (t / ntx) * TZ;
        const gp<const R> E[3] = {G<R>((const void *)D.E[par][0]), G<R>((const void *)D.E[par][1]),
                                  G<R>((const void *)D.E[par][2])};
        const gp<const R> B[3] = {G<R>((const void *)D.B[par][0]), G<R>((const void *)D.B[par][1]),
                                  G<R>((const void *)D.B[par][2])};
        // branch-free addresses (a branch between the loads and their use costs
        // exact waits); the row of a wave is uniform, so its wrap is scalar
        const int gxa = wx(x0 - LO + lane);
#pragma unroll
        for (int u = 0; u < RW; u++) {
            const int zr = __builtin_amdgcn_readfirstlane(wz(z0 - LO + min(wave + u * nwave, WZ - 1)));
            const int g = zr * nx + gxa;
#pragma unroll
            for (int k = 0; k < 3; k++) { ve[u][k] = E[k][g]; vb[u][k] = B[k][g]; }
        }
        const int gh = wz(z0 - LO + hrow) * nx + wx(x0 - LO + hcol);
#pragma unroll
        for (int k = 0; k < 3; k++) { he[k] = E[k][gh]; hb[k] = B[k][gh]; }
    };
    const int item = blockIdx.x;
    load_eb(item);
    {
        int inst, t;
        tile_of(item, inst, t);
        const InstDesc &D = Dt[inst];
        const int nx = D.n[0], nz = D.n[2];
        const PerMod wx(nx), wz(nz);
        const int ntx = (nx + TX - 1) / TX;
        const int x0 = (t % ntx) * TX + (nx % TX == 0 ? LO : 0), z0 = (t / ntx) * TZ;
        const gp<const JT> J[3] = {G<JT>((const void *)D.J[par][0]), G<JT>((const void *)D.J[par][1]),
                                   G<JT>((const void *)D.J[par][2])};
        // E, B and J are read with halos that neighbouring tiles own, so the new
        // fields go to the other set of planes (E then B), and that set's J is cleared
        const int po = par ^ 1;
        gp<R> O[6] = {G<R>(D.E[po][0]), G<R>(D.E[po][1]), G<R>(D.E[po][2]),
                      G<R>(D.B[po][0]), G<R>(D.B[po][1]), G<R>(D.B[po][2])};
        const double jq = D.jqg, jb[3] = {D.jbg[0], D.jbg[1], D.jbg[2]};
#pragma unroll
        for (int u = 0; u < RW; u++) {
            const int row = wave + u * nwave;
            const int c = row < WZ ? row * WX + lane : WN + lane;
#pragma unroll
            for (int k = 0; k < 3; k++) { sE[k][c] = ve[u][k]; sB[k][c] = vb[u][k]; }
        }
        {
            const int c = hth ? hrow * WX + hcol : WN + lane;
#pragma unroll
            for (int k = 0; k < 3; k++) { sE[k][c] = he[k]; sB[k][c] = hb[k]; }
        }
        // J of every staged cell, loaded without a branch (a window cell is always
        // a valid address; only the cells where E^n is formed use it) after the
        // LDS stores, so the wait for the staged E, B does not include these;
        // they are used after the B half step
        JT vj[RW][3], hj[3];
        bool jbad = false;
        {
            const int gxa = wx(x0 - LO + lane);
#pragma unroll
            for (int u = 0; u < RW; u++) {
                const int zr = __builtin_amdgcn_readfirstlane(wz(z0 - LO + min(wave + u * nwave, WZ - 1)));
                const int g = zr * nx + gxa;
#pragma unroll
                for (int k = 0; k < 3; k++) vj[u][k] = J[k][g];
            }
            const int gh = wz(z0 - LO + hrow) * nx + wx(x0 - LO + hcol);
#pragma unroll
            for (int k = 0; k < 3; k++) hj[k] = J[k][gh];
        }
        lds_barrier();
        const R idx = R(1) / (R)D.d[0], idz = R(1) / (R)D.d[2], dt = (R)D.dt, h = R(0.5) * dt;
        // Faraday's forward differences at window cell e: Yee, or averaged across
        // the difference's direction with (1/8, 3/4, 1/8)
        auto fdx = [&](const R *F, int e) {
            if constexpr (CK)
                return (R(0.75) * (F[e + 1] - F[e]) +
                        R(0.125) * ((F[e + 1 - WX] - F[e - WX]) + (F[e + 1 + WX] - F[e + WX]))) * idx;
            else
                return (F[e + 1] - F[e]) * idx;
        };
        auto fdz = [&](const R *F, int e) {
            if constexpr (CK)
                return (R(0.75) * (F[e + WX] - F[e]) +
                        R(0.125) * ((F[e - 1 + WX] - F[e - 1]) + (F[e + 1 + WX] - F[e + 1]))) * idz;
            else
                return (F[e + WX] - F[e]) * idz;
        };
        // The first halo phase covers a few more columns than the 64 lanes; its
        // (row, column) cells are dealt out to the block's threads in order, so no
        // wave runs a second pass for those few columns.
        // B^{n-1/2} on local rows and columns [ELO - 1, EH): forward differences of E
        constexpr int C1 = EHX - ELO + 1, N1 = (EHZ - ELO + 1) * C1;
        for (int it = threadIdx.x; it < N1; it += blockDim.x) {
            const int e = (ELO - 1 + it / C1) * WX + ELO - 1 + it % C1;
            const R dzEy = fdz(sE[1], e), dzEx = fdz(sE[0], e);
            const R dxEz = fdx(sE[2], e), dxEy = fdx(sE[1], e);
            sB[0][e] -= h * (-dzEy);
            sB[1][e] -= h * (dzEx - dxEz);
            sB[2][e] -= h * dxEy;
        }
        lds_barrier();
        // E^n on local [ELO, EH): backward differences of B^{n-1/2}, by the threads
        // that staged each cell (their J is in registers)
        auto e_step = [&](int e, const JT *j) {
            const int exm = e - 1, ezm = e - WX;
            const R dzBy = (sB[1][e] - sB[1][ezm]) * idz, dzBx = (sB[0][e] - sB[0][ezm]) * idz;
            const R dxBz = (sB[2][e] - sB[2][exm]) * idx, dxBy = (sB[1][e] - sB[1][exm]) * idx;
            const R j0 = (R)(jreal(j[0], jq) + jb[0]);
            const R j1 = (R)(jreal(j[1], jq) + jb[1]);
            const R j2 = (R)(jreal(j[2], jq) + jb[2]);
            sE[0][e] += dt * (-dzBy - j0);
            sE[1][e] += dt * (dzBx - dxBz - j1);
            sE[2][e] += dt * (dxBy - j2);
            jbad |= jrange_bad(j[0]) | jrange_bad(j[1]) | jrange_bad(j[2]);
        };
#pragma unroll
        for (int u = 0; u < RW; u++) {
            const int row = wave + u * nwave;
            if (row >= ELO && row < EHZ && lane >= ELO) e_step(row * WX + lane, vj[u]);
        }
        if (hth && hrow >= ELO && hrow < EHZ && hcol < EHX) e_step(hrow * WX + hcol, hj);
        // a plain global store (every writer writes 1): an atomic that returns a
        // value, or a flat store, makes the wave wait for all its loads, the next
        // item's included
        if (jbad) G<int>((void *)D.flags)[FLAG_JRANGE] = 1;
        lds_barrier();
        // B^n on the tile and the stores (rows unrolled: a loop here would make
        // the compiler wait for every outstanding load before it).  On grids
        // whose width is a multiple of 64 the tiles start LO cells past a 64-cell
        // boundary, so each staged row begins on a 256-byte boundary (three
        // 128-byte lines a row rather than four), and the last tile's outputs
        // wrap onto the first LO columns
        const int gxs = x0 + lane;
        const int gx = gxs >= nx && nx % TX == 0 ? gxs - nx : gxs;
        if (gx < nx) {
#pragma unroll
            for (int r = 0; r < (TZ + 3) / 4; r++) {
                const int lz = wave + r * 4;
                const int gz = z0 + lz;
                if (lz >= TZ || gz >= nz) continue;
                const int e = (lz + LO) * WX + lane + LO;
                const R dzEy = fdz(sE[1], e), dzEx = fdz(sE[0], e);
                const R dxEz = fdx(sE[2], e), dxEy = fdx(sE[1], e);
                const int g = gz * nx + gx;
                const R b0 = sB[0][e] - h * (-dzEy), b1 = sB[1][e] - h * (dzEx - dxEz), b2 = sB[2][e] - h * dxEy;
                O[3][g] = b0; O[4][g] = b1; O[5][g] = b2;
                O[0][g] = sE[0][e]; O[1][g] = sE[1][e]; O[2][g] = sE[2][e];
#pragma unroll
                for (int k = 0; k < 3; k++) G<JT>(D.J[po][k])[g] = JT(0);
                if (D.rE[0]) {
                    // recording a tape slot: E^n, B^n of this step
                    G<R>(D.rE[0])[g] = sE[0][e]; G<R>(D.rE[1])[g] = sE[1][e]; G<R>(D.rE[2])[g] = sE[2][e];
                    G<R>(D.rB[0])[g] = b0; G<R>(D.rB[1])[g] = b1; G<R>(D.rB[2])[g] = b2;
                }
            }
        }
    }
}

// ------------------------------------------------------ seen-field passes
// Taps of component comp (Ex Ey Ez Bx By Bz) along z, x and y.  With the
// momentum-conserving gather, the axes along which a component is
// half-staggered (z: Ez Bx By; x: Ex By Bz; y: Ey Bx Bz) take the taps composed
// with the node average.
__device__ __forceinline__ const double *ztaps(const InstDesc &D, int comp)
{
    return (D.nodal && comp >= 2 && comp <= 4) ? D.tzn : D.tz[comp < 2 ? 0 : 1];
}
__device__ __forceinline__ const double *xtaps(const InstDesc &D, int comp)
{
    return (D.nodal && (comp == 0 || comp >= 4)) ? D.txn : D.tx;
}
__device__ __forceinline__ const double *ytaps(const InstDesc &D, int comp)
{
    return (D.nodal && (comp & 1)) ? D.tyn : D.ty;
}

// axis 2: combined z taps (Psi_E o filter for Ex, Ey; Psi_B o filter for Ez, Bx,
// By, Bz); axis 0 / 1: filter taps along x / y.  blockIdx.y selects the component.
template <int AXIS, class R, int HW>
__global__ void __launch_bounds__(256) k_seen_pass(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                   int src_sel, int dst_sel, int par)
{
    // HW >= 0: the pass's half-width at compile time (taps unrolled, all loads
    // of a cell in flight at once); -1: read it from the descriptor
    const int inst = work[blockIdx.x].x;
    const InstDesc &D = Dt[inst];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    const int comp = blockIdx.y;
    if (cell >= D.ncell) return;
    const R *src;
    if (src_sel == 0) src = comp < 3 ? (const R *)D.E[par][comp] : (const R *)D.B[par][comp - 3];
    else if (src_sel == 1) src = (const R *)D.T1[comp];
    else src = (const R *)D.T2[comp];
    R *dst;
    if (dst_sel == 1) dst = (R *)D.T1[comp];
    else if (dst_sel == 2) dst = (R *)D.T2[comp];
    else dst = comp < 3 ? (R *)D.Et[comp] : (R *)D.Bt[comp - 3];
    int i, j, k;
    cell_ijk<R>(D, cell, i, j, k);
    const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
    const double *tap = AXIS == 2 ? ztaps(D, comp) : (AXIS == 0 ? xtaps(D, comp) : ytaps(D, comp));
    const int h = HW >= 0 ? HW : (AXIS == 2 ? D.hz : (AXIS == 0 ? D.hx : D.hy));
    // index along the axis, its extent and the stride between neighbours
    const int q = AXIS == 2 ? k : (AXIS == 0 ? i : j);
    const int nq = AXIS == 2 ? nz : (AXIS == 0 ? nx : ny);
    const int stride = AXIS == 2 ? nx * ny : (AXIS == 0 ? 1 : nx);
    const int base = cell - q * stride;
    const gp<const R> s = G<R>((const void *)src);
    R acc = R(0);
    if constexpr (HW >= 0) {
#pragma unroll
        for (int t = -HW; t <= HW; t++) acc += (R)tap[t + HW] * s[base + wrap_near(q + t, nq) * stride];
    } else {
        for (int t = -h; t <= h; t++) acc += (R)tap[t + h] * s[base + wrap_near(q + t, nq) * stride];
    }
    G<R>(dst)[cell] = acc;
}

// One pass of the 3D seen-field stencils along a strided axis (AXIS 2: z,
// 1: y), HW taps either side: each thread walks one column of the grid (lanes
// on consecutive x, so every load of a wave is one contiguous row), keeps the
// RUN + 2 HW values of its run of RUN output cells in registers and writes the
// RUN outputs.  The taps are converted to R once per thread and every input
// value is loaded once per run instead of once per tap.  blockIdx.y =
// component, blockIdx.z = instance (from inst0).
template <int AXIS, class R, int HW, int RUN>
__global__ void __launch_bounds__(256) k_seen_col(const InstDesc *__restrict__ Dt, int inst0, int src_sel,
                                                  int dst_sel, int par)
{
    const InstDesc &D = Dt[inst0 + blockIdx.z];
    const int comp = blockIdx.y;
    const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
    const int nq = AXIS == 2 ? nz : ny;              // cells along the pass
    const int ncol = AXIS == 2 ? nx * ny : nx * nz;  // columns
    const int nseg = (nq + RUN - 1) / RUN;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ncol * nseg) return;
    const int seg = g / ncol, col = g - seg * ncol;
    const int i = col % nx, o = col / nx;            // o: y index (z pass) or z index (y pass)
    const int stride = AXIS == 2 ? nx * ny : nx;
    const int base = AXIS == 2 ? i + o * nx : i + o * nx * ny;
    const R *src;
    if (src_sel == 0) src = comp < 3 ? (const R *)D.E[par][comp] : (const R *)D.B[par][comp - 3];
    else if (src_sel == 1) src = (const R *)D.T1[comp];
    else src = (const R *)D.T2[comp];
    R *dst;
    if (dst_sel == 1) dst = (R *)D.T1[comp];
    else if (dst_sel == 2) dst = (R *)D.T2[comp];
    else dst = comp < 3 ? (R *)D.Et[comp] : (R *)D.Bt[comp - 3];
    const double *tap = AXIS == 2 ? ztaps(D, comp) : ytaps(D, comp);
    R tp[2 * HW + 1];
#pragma unroll
    for (int t = 0; t <= 2 * HW; t++) tp[t] = (R)tap[t];
    const gp<const R> sp = G<R>((const void *)src);
    const gp<R> dp = G<R>((void *)dst);
    const int q0 = seg * RUN;
    // the run's inputs q0 - HW .. q0 + RUN + HW - 1, periodic along the axis
    int q = ((q0 - HW) % nq + nq) % nq;
    R w[RUN + 2 * HW];
#pragma unroll
    for (int t = 0; t < RUN + 2 * HW; t++) {
        w[t] = sp[base + q * stride];
        q = q + 1 == nq ? 0 : q + 1;
    }
#pragma unroll
    for (int r = 0; r < RUN; r++) {
        if (q0 + r >= nq) break;
        R acc = R(0);
#pragma unroll
        for (int t = 0; t <= 2 * HW; t++) acc += tp[t] * w[r + t];
        dp[base + (q0 + r) * stride] = acc;
    }
}

// 3D x-direction pass (compile-time half-width): blockIdx.z = instance,
// blockIdx.y = component; a workgroup takes PIC_SEEN_XSEG 64-cell row
// segments per wave.  Rows whose length is a multiple of 64: each wave loads
// all its segments, with their row-wrapped ends, into LDS before it waits for
// any (2 PIC_SEEN_XSEG loads in flight a lane), and every output then reads
// its taps at fixed offsets.  Other rows: one cell per thread, a wrapped index
// and a load per tap.  Both add the same products in the same order.
template <class R, int HW>
__global__ void __launch_bounds__(256) k_seen_x(const InstDesc *__restrict__ Dt, int inst0, int src_sel, int dst_sel,
                                                int par)
{
    constexpr int K = PIC_SEEN_XSEG, SW = 64 + 2 * HW;
    __shared__ R st[4][K][SW + 1];
    const InstDesc &D = Dt[inst0 + blockIdx.z];
    const int comp = blockIdx.y;
    const int nx = D.n[0], ncell = D.ncell;
    const int cb = (int)blockIdx.x * (256 * K);
    if (cb >= ncell) return;   // uniform over the workgroup
    const gp<const R> s = G<R>(src_sel == 0 ? (comp < 3 ? D.E[par][comp] : D.B[par][comp - 3])
                                            : (src_sel == 1 ? D.T1[comp] : D.T2[comp]));
    const gp<R> dst = G<R>(dst_sel == 1 ? D.T1[comp]
                                        : (dst_sel == 2 ? D.T2[comp] : (comp < 3 ? D.Et[comp] : D.Bt[comp - 3])));
    const double *tap = xtaps(D, comp);
    R tp[2 * HW + 1];
#pragma unroll
    for (int t = 0; t <= 2 * HW; t++) tp[t] = (R)tap[t];
    const PerMod wx(nx);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (nx % 64 == 0) {
        // segment k of wave w: cells [sg, sg + 64), sg = cb + 64 (4 k + w);
        // ncell is a multiple of 64, so a segment is whole or absent (an absent
        // one loads the block's first segment again and stores nothing)
        R va[K], vb[K];
        const int hl = lane < 2 * HW ? lane : 0;
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int sg0 = cb + 64 * (4 * k + w);
            const int sg = sg0 < ncell ? sg0 : cb;
            const int i0 = wx(sg), rb = sg - i0;
            va[k] = s[rb + wx(i0 - HW + lane)];
            vb[k] = s[rb + wx(i0 - HW + 64 + hl)];
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            st[w][k][lane] = va[k];
            // lanes past the halo store into the spare word
            st[w][k][lane < 2 * HW ? 64 + lane : SW] = vb[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int sg = cb + 64 * (4 * k + w);
            R acc = R(0);
#pragma unroll
            for (int t = 0; t <= 2 * HW; t++) acc += tp[t] * st[w][k][lane + t];
            if (sg < ncell) dst[sg + lane] = acc;
        }
    } else {
#pragma unroll 1
        for (int k = 0; k < K; k++) {
            const int cell = cb + 256 * k + (int)threadIdx.x;
            if (cell >= ncell) break;
            const int i = wx(cell), base = cell - i;
            R acc = R(0);
#pragma unroll
            for (int t = -HW; t <= HW; t++) acc += tp[t + HW] * s[base + wrap_near(i + t, nx)];
            dst[cell] = acc;
        }
    }
}

// 2D fields as seen by the particles in one kernel: one component's (64 x SEEN_TZ)
// output tile is staged in LDS with its stencil halo (waves own rows, lanes own
// columns, so addresses are affine in the lane); the x filter stencil then runs
// on every staged row for the 64 output columns, four neighbouring columns per
// thread with their shared inputs read once; last, the combined z stencil
// (Psi o z filter) walks down each column, SEEN_TZ / 4 consecutive output rows
// per wave, the rows they share read once.  The two stencils act on different
// axes of a periodic grid, so they commute: x then z is the same operator as
// z then x.  blockIdx.y = component, work = (inst, tile); four waves per block.
// HZ, HX >= 0 fix the stencil half-widths at compile time (taps in registers,
// loops unrolled); -1 reads them from the descriptor.
#define SEEN_TX PIC_SEEN_TX
template <class R, int SEEN_TZ, int HZ, int HX>
__global__ void __launch_bounds__(256) k_seen_2d(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                 int par)
{
    static_assert(SEEN_TX == 64, "one lane per column");
    static_assert(SEEN_TZ % 4 == 0, "the four waves split the output rows");
    extern __shared__ __align__(16) unsigned char smem[];
    // work == nullptr: one instance, block b is tile b in the host's XCD order
    // (saves a dependent load)
    const int inst = work ? work[blockIdx.x].x : 0;
    const int t = work ? work[blockIdx.x].y : xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int comp = blockIdx.y;
    const InstDesc &D = Dt[inst];
    const int nx = D.n[0], nz = D.n[2];
    const int ntx = (nx + SEEN_TX - 1) / SEEN_TX;
    const int x0 = (t % ntx) * SEEN_TX, z0 = (t / ntx) * SEEN_TZ;
    const int hz = HZ >= 0 ? HZ : D.hz, hx = HX >= 0 ? HX : D.hx;
    const int wx = SEEN_TX + 2 * hx, wz = SEEN_TZ + 2 * hz;
    const int lane = threadIdx.x & 63, wave = wave_id(), nwave = blockDim.x >> 6;
    R *win = reinterpret_cast<R *>(smem);   // wz x wx: the staged window
    R *mid = win + wx * wz;                 // wz x 64: after the x stencil
    R *tz = mid + SEEN_TX * wz;
    R *tx = tz + 2 * PIC_MAX_HZ + 1;
    const double *tzs = ztaps(D, comp), *txs = xtaps(D, comp);
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
        for (int k = 0; k < NTX; k++) rx[k] = (R)txs[k];
    } else {
        for (int i = threadIdx.x; i <= 2 * hx; i += blockDim.x) tx[i] = (R)txs[i];
    }
    const void *sp = comp < 3 ? D.E[par][comp] : D.B[par][comp - 3];
    const gp<const R> src = G<R>(sp);
    // staging: column a = lane, column b = 64 + lane for the right halo (lane < 2 hx)
    const bool hasb = lane < 2 * hx;
    const int gxa = wrap_near(x0 - hx + lane, nx);
    const int gxb = hasb ? wrap_near(x0 - hx + SEEN_TX + lane, nx) : gxa;
    // rows per wave and pass: with compile-time widths, the whole window in one
    // pass of the four waves (every load of a wave in flight before its first
    // wait); rows past the window land in the x-filtered area, which is written
    // only after the barrier below
    constexpr bool FIXED = HZ >= 0 && SEEN_TZ >= 32;
    constexpr int U = FIXED ? (SEEN_TZ + 2 * (HZ > 0 ? HZ : 0) + 3) / 4 : 8;
    const PerMod wzm(nz);
    for (int r0 = wave; r0 < wz; r0 += U * nwave) {
        R va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int row = min(r0 + u * nwave, wz - 1);
            const int base = wzm(z0 - hz + row) * nx;
            va[u] = src[base + gxa];
            vb[u] = src[base + gxb];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int row = r0 + u * nwave;
            if (FIXED || row < wz) {
                win[row * wx + lane] = va[u];
                if (hasb) win[row * wx + SEEN_TX + lane] = vb[u];
            }
        }
    }
    __syncthreads();
    // x stencil: item (row r, output columns [4 q, 4 q + 4)) of wz x 16 items
    constexpr int XQ = 4, NQ = SEEN_TX / XQ;
    for (int it = threadIdx.x; it < wz * NQ; it += blockDim.x) {
        const int r = it / NQ, c0 = (it % NQ) * XQ;
        const R *w = win + r * wx + c0;
        R *o = mid + r * SEEN_TX + c0;
        if constexpr (HX >= 0) {
            R v[XQ + 2 * HX];
#pragma unroll
            for (int k = 0; k < XQ + 2 * HX; k++) v[k] = w[k];
#pragma unroll
            for (int q = 0; q < XQ; q++) {
                R acc = rx[0] * v[q];
#pragma unroll
                for (int k = 1; k < NTX; k++) acc += rx[k] * v[q + k];
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
    // z stencil: wave -> output rows [RB wave, RB wave + RB), lane -> column
    constexpr int RB = SEEN_TZ / 4;
    gp<R> dst = G<R>(comp < 3 ? D.Et[comp] : D.Bt[comp - 3]);
    const int gx = x0 + lane, zr = wave * RB;
    if (gx >= nx) return;
    const R *m = mid + zr * SEEN_TX + lane;
    if constexpr (HZ >= 0) {
        R v[RB + 2 * HZ];
#pragma unroll
        for (int k = 0; k < RB + 2 * HZ; k++) v[k] = m[k * SEEN_TX];
#pragma unroll
        for (int j = 0; j < RB; j++) {
            const int gz = z0 + zr + j;
            R acc = rz[0] * v[j];
#pragma unroll
            for (int k = 1; k < NTZ; k++) acc += rz[k] * v[j + k];
            if (gz < nz) dst[gz * nx + gx] = acc;
        }
    } else {
        for (int j = 0; j < RB; j++) {
            const int gz = z0 + zr + j;
            if (gz >= nz) break;
            R acc = R(0);
            for (int k = 0; k <= 2 * hz; k++) acc += tz[k] * m[(j + k) * SEEN_TX];
            dst[gz * nx + gx] = acc;
        }
    }
}

// The same operator streamed along z (float, compile-time widths): one block
// takes one component's PIC_SEEN_SW-column strip over SEG rows and walks down
// it in chunks of SEEN_CZ rows.  Each chunk's new rows (with the x halo) are
// staged in LDS and filtered along x into a ring of SEEN_CZ + 2 HZ rows, which
// keeps the z halo the next chunk needs, so a row enters from HBM once per
// segment (the 2 HZ halo rows once per SEG rows, not once per 32-row tile, and
// the 2 HX halo columns once per 128 columns).  The next chunk's rows are
// loaded into registers while the current one is filtered, and the barriers
// wait for LDS only.  Eight waves: four over the rows of each 64-column half,
// lanes on columns.
#define SEEN_CZ 32
template <class R, int SEG, int HZ, int HX>
__global__ void __launch_bounds__(512) k_seen_2d_stream(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                        int par)
{
    constexpr int TW = PIC_SEEN_SW;
    static_assert(TW == 128 && SEG % SEEN_CZ == 0, "two 64-column halves, whole chunks");
    constexpr int CZ = SEEN_CZ, NW = 4, RW = CZ / NW, NCH = SEG / CZ;
    constexpr int RING = CZ + 2 * HZ, WX = TW + 2 * HX;
    constexpr int R0 = (RING + NW - 1) / NW;          // rows per wave of the first chunk
    constexpr int NTZ = 2 * HZ + 1, NTX = 2 * HX + 1, XQ = 4, NQ = TW / XQ;
    __shared__ R raw[RING * WX];                      // rows staged by this chunk
    __shared__ R mid[RING * TW];                      // x-filtered rows, ring by window row
    const int inst = work ? work[blockIdx.x].x : 0;
    const int t = work ? work[blockIdx.x].y : xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int comp = blockIdx.y;
    const InstDesc &D = Dt[inst];
    const int nx = D.n[0], nz = D.n[2];
    const int ntx = (nx + TW - 1) / TW;
    // grids whose width is a multiple of 64: strips start HX cells past a
    // 64-cell boundary, so that every staged row begins on a 256-byte boundary;
    // the last strip's outputs wrap onto the first HX columns (and, where the
    // width is an odd multiple of 64, its columns past those repeat ones another
    // strip stores: they are not stored)
    const int sh = nx % 64 == 0 ? HX : 0;
    const int x0 = (t % ntx) * TW + sh, z0 = (t / ntx) * SEG;
    const int nch = (min(SEG, nz - z0) + CZ - 1) / CZ;  // chunks of this segment (uniform)
    const double *tzs = ztaps(D, comp), *txs = xtaps(D, comp);
    R rz[NTZ], rx[NTX];
#pragma unroll
    for (int k = 0; k < NTZ; k++) rz[k] = (R)tzs[k];
#pragma unroll
    for (int k = 0; k < NTX; k++) rx[k] = (R)txs[k];
    const gp<const R> src = G<R>(comp < 3 ? D.E[par][comp] : D.B[par][comp - 3]);
    gp<R> dst = G<R>(comp < 3 ? D.Et[comp] : D.Bt[comp - 3]);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int half = wave >> 2, wr = wave & 3, col = 64 * half + lane;
    const bool hasb = half == 1 && lane < 2 * HX;     // the right halo columns TW + lane
    const PerMod wx(nx), wz(nz);
    const int gxa = wx(x0 - HX + col);
    const int gxb = hasb ? wx(x0 - HX + TW + lane) : gxa;
    // window row w is grid row z0 - HZ + w; the first chunk stages rows
    // [0, RING), chunk c >= 1 rows [c CZ + 2 HZ, (c + 1) CZ + 2 HZ)
    auto grow = [&](int w) { return wz(z0 - HZ + w) * nx; };
    {
        R va[R0], vb[R0];
#pragma unroll
        for (int u = 0; u < R0; u++) {
            const int base = grow(min(wr + u * NW, RING - 1));
            va[u] = src[base + gxa];
            vb[u] = src[base + gxb];
        }
#pragma unroll
        for (int u = 0; u < R0; u++) {
            const int r = wr + u * NW;
            if (r < RING) {
                raw[r * WX + col] = va[u];
                if (hasb) raw[r * WX + TW + lane] = vb[u];
            }
        }
    }
    R pa[RW], pb[RW];
#pragma unroll
    for (int c = 0; c < NCH; c++) {
        if (c >= nch) break;
        if (c > 0) {
            // this chunk's rows, loaded during the previous one
#pragma unroll
            for (int u = 0; u < RW; u++) {
                const int r = wr + u * NW;
                raw[r * WX + col] = pa[u];
                if (hasb) raw[r * WX + TW + lane] = pb[u];
            }
        }
        if (c + 1 < nch) {
#pragma unroll
            for (int u = 0; u < RW; u++) {
                const int base = grow((c + 1) * CZ + 2 * HZ + wr + u * NW);
                pa[u] = src[base + gxa];
                pb[u] = src[base + gxb];
            }
        }
        lds_barrier();
        // x stencil on the staged rows: item (row, 4 output columns)
        const int nr = c == 0 ? RING : CZ, w0 = c == 0 ? 0 : c * CZ + 2 * HZ;
        for (int it = threadIdx.x; it < nr * NQ; it += 512) {
            const int r = it / NQ, c0 = (it % NQ) * XQ;
            const R *w = raw + r * WX + c0;
            R v[XQ + 2 * HX];
#pragma unroll
            for (int k = 0; k < XQ + 2 * HX; k++) v[k] = w[k];
            R *o = mid + ((w0 + r) % RING) * TW + c0;
#pragma unroll
            for (int q = 0; q < XQ; q++) {
                R acc = rx[0] * v[q];
#pragma unroll
                for (int k = 1; k < NTX; k++) acc += rx[k] * v[q + k];
                o[q] = acc;
            }
        }
        lds_barrier();
        // z stencil: output rows c CZ + wr RW + [0, RW) take window rows
        // c CZ + wr RW + [0, RW + 2 HZ)
        const int s0 = (c * CZ + wr * RW) % RING;
        R v[RW + 2 * HZ];
#pragma unroll
        for (int k = 0; k < RW + 2 * HZ; k++) {
            const int s = s0 + k < RING ? s0 + k : s0 + k - RING;
            v[k] = mid[s * TW + col];
        }
        const int gxs = x0 + col;
        const bool xok = sh ? gxs < nx + sh : gxs < nx;
        const int gx = gxs >= nx ? gxs - nx : gxs;
#pragma unroll
        for (int j = 0; j < RW; j++) {
            const int gz = z0 + c * CZ + wr * RW + j;
            R acc = rz[0] * v[j];
#pragma unroll
            for (int k = 1; k < NTZ; k++) acc += rz[k] * v[j + k];
            if (xok && gz < nz) dst[gz * nx + gx] = acc;
        }
    }
}

// ------------------------------------------- exact ratio: Psi_B^{-1} along z
// The variant that multiplies the transverse E by the full Psi_E / Psi_B
// applies Psi_B(S_z)^{-1} after the seen pass (Sec. 2: the denominator
// inverted by tri-diagonal solves).  With Psi_B(s) = b prod_q (s - r_q) over
// its real roots (outside [0, 1]), each factor S_z - r_q is the periodic
// tri-diagonal (-1/4, 1/2 - r_q, -1/4) = -(1 / (4 l_q)) (1 - l_q E^-1)(1 - l_q E),
// l_q + 1/l_q = 2 - 4 r_q, |l_q| < 1: a causal then an anti-causal first-order
// recursion, the constants gathered in rscale.  One wave solves one z column
// (PIC_RATIO_TC columns per workgroup): its 64 lanes own contiguous segments of
// ceil(nz / 64) rows, loaded straight into registers (all loads of a lane in
// flight at once; the neighbouring columns of the same cache lines belong to
// the sibling waves).  Each lane runs the recursion over its segment from a
// zero state, a wave scan of the segments' affine maps s -> A s + e gives
// every segment its exact periodic incoming state, and the lane adds that
// state's decaying contribution.
template <class R>
__global__ void __launch_bounds__(256) k_psi_inv_z(const InstDesc *__restrict__ Dt, int inst0)
{
    constexpr int MAXL = PIC_RATIO_MAXNZ / 64;
    const int inst = inst0 + blockIdx.y, comp = blockIdx.z;
    const InstDesc &D = Dt[inst];
    const int ncol = D.n[0] * D.n[1], nz = D.n[2];
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int col = blockIdx.x * PIC_RATIO_TC + wave;
    if (col >= ncol) return;
    const int Ls = (nz + 63) / 64;
    const int len = max(0, min(Ls, nz - lane * Ls));
    const gp<R> F = G<R>(D.Et[comp]) + col;
    const size_t base = (size_t)lane * Ls * ncol;
    R v[MAXL];
#pragma unroll
    for (int i = 0; i < MAXL; i++) v[i] = i < len ? F[base + (size_t)i * ncol] : R(0);
    for (int q = 0; q < D.nroot; q++) {
        const R l = (R)D.lam[q];
        // causal: w[k] = v[k] + l w[k-1]
        R st = R(0), A = R(1);
#pragma unroll
        for (int i = 0; i < MAXL; i++)
            if (i < len) { st = v[i] + l * st; v[i] = st; A *= l; }
        // prefix composition over lanes 0..63 (F_j = f_j o F_{j-1})
        R P = A, Q = st;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const R Pp = __shfl_up(P, d), Qp = __shfl_up(Q, d);
            if (lane >= d) { Q = P * Qp + Q; P = P * Pp; }
        }
        // periodic: the state entering lane 0 is the one leaving lane 63
        const R C0 = __shfl(Q, 63) / (R(1) - __shfl(P, 63));
        const R Pm = __shfl_up(P, 1), Qm = __shfl_up(Q, 1);
        R C = lane == 0 ? C0 : Pm * C0 + Qm;
#pragma unroll
        for (int i = 0; i < MAXL; i++)
            if (i < len) { C *= l; v[i] += C; }
        // anti-causal: y[k] = w[k] + l y[k+1]
        st = R(0); A = R(1);
#pragma unroll
        for (int i = MAXL - 1; i >= 0; i--)
            if (i < len) { st = v[i] + l * st; v[i] = st; A *= l; }
        // suffix composition over lanes 63..0 (G_j = f_j o G_{j+1})
        P = A; Q = st;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const R Pn = __shfl_down(P, d), Qn = __shfl_down(Q, d);
            if (lane + d < 64) { Q = P * Qn + Q; P = P * Pn; }
        }
        // periodic: the state entering lane 63 is the one leaving lane 0
        const R C63 = __shfl(Q, 0) / (R(1) - __shfl(P, 0));
        const R Pn1 = __shfl_down(P, 1), Qn1 = __shfl_down(Q, 1);
        C = lane == 63 ? C63 : Pn1 * C63 + Qn1;
#pragma unroll
        for (int i = MAXL - 1; i >= 0; i--)
            if (i < len) { C *= l; v[i] += C; }
    }
    const R sc = (R)D.rscale;
#pragma unroll
    for (int i = 0; i < MAXL; i++)
        if (i < len) F[base + (size_t)i * ncol] = sc * v[i];
}

// ------------------------------------------------------------------ resort

template <int DIM> __device__ __forceinline__ int tile_of(const InstDesc &D, unsigned idx)
{
    int c[3];
    unpack_cell<DIM>(idx, c);
    return (c[2] / D.tile[2] * D.nt[1] + c[1] / D.tile[1]) * D.nt[0] + c[0] / D.tile[0];
}

// The re-sort kernels run every few steps and mostly find nothing to do: each
// wave first reads the shared pending word and leaves if it is clear.  They
// walk the particle chunks with a block-strided loop over a small grid.
#define RESORT_GRID 512

template <int DIM>
__global__ void __launch_bounds__(256) k_resort_count(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                      int nwork, const int *__restrict__ any)
{
    if (!*any) return;
    for (int it = blockIdx.x; it < nwork; it += gridDim.x) {
        const InstDesc &D = Dt[work[it].x];
        if (!D.flags[FLAG_RESORT]) continue;
        const long long p = (long long)work[it].y * PIC_PART_CHUNK + threadIdx.x;
        if (p >= D.np) continue;
        const int t = tile_of<DIM>(D, (unsigned)D.pidx[p]);
        D.stile[p] = t;
        D.srank[p] = atomicAdd(&D.tcount[t], 1);
    }
}

// one 1024-thread block per instance: exclusive scan of the tile counts
__global__ void __launch_bounds__(1024) k_resort_scan(const InstDesc *__restrict__ Dt, int inst0,
                                                      const int *__restrict__ any)
{
    if (!*any) return;
    const InstDesc &D = Dt[inst0 + blockIdx.x];
    if (!D.flags[FLAG_RESORT]) return;
    __shared__ int part[1024];
    const int n = D.ntiles, tid = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int b = tid * per, e = min(n, b + per);
    int s = 0;
    for (int t = b; t < e; t++) s += D.tcount[t];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = tid == 0 ? 0 : part[tid - 1];
    for (int t = b; t < e; t++) {
        D.tstart[t] = run;
        run += D.tcount[t];
        D.tcount[t] = 0;
    }
    if (tid == 1023) D.tstart[n] = part[1023];
}

template <int DIM, class R>
__global__ void __launch_bounds__(256) k_resort_scatter(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                        int nwork, const int *__restrict__ any)
{
    if (!*any) return;
    for (int it = blockIdx.x; it < nwork; it += gridDim.x) {
        const InstDesc &D = Dt[work[it].x];
        if (!D.flags[FLAG_RESORT]) continue;
        const long long p = (long long)work[it].y * PIC_PART_CHUNK + threadIdx.x;
        if (p >= D.np) continue;
        const int q = D.tstart[D.stile[p]] + D.srank[p];
        D.sidx[q] = D.pidx[p];
        D.spid[q] = D.ppid[p];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (!(DIM == 2 && a == 1)) ((R *)D.soff[a])[q] = ((const R *)D.poff[a])[p];
            ((R *)D.su[a])[q] = ((const R *)D.pu[a])[p];
        }
    }
}

template <int DIM, class R>
__global__ void __launch_bounds__(256) k_resort_copy(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                     int nwork, const int *__restrict__ any)
{
    if (!*any) return;
    for (int it = blockIdx.x; it < nwork; it += gridDim.x) {
        const InstDesc &D = Dt[work[it].x];
        if (!D.flags[FLAG_RESORT]) continue;
        const long long p = (long long)work[it].y * PIC_PART_CHUNK + threadIdx.x;
        if (p >= D.np) continue;
        D.pidx[p] = D.sidx[p];
        D.ppid[p] = D.spid[p];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (!(DIM == 2 && a == 1)) ((R *)D.poff[a])[p] = ((const R *)D.soff[a])[p];
            ((R *)D.pu[a])[p] = ((const R *)D.su[a])[p];
        }
    }
}

// per instance: reset every tile's bounding box to the tile itself and clear the flag
__global__ void __launch_bounds__(256) k_resort_done(const InstDesc *__restrict__ Dt, int inst0, int force,
                                                     int *__restrict__ any, int clear_any)
{
    const InstDesc &D = Dt[inst0 + blockIdx.x];
    // no block of this kernel reads the shared word, so block 0 may clear it
    if (clear_any && blockIdx.x == 0 && threadIdx.x == 0) *any = 0;
    if (!force && !D.flags[FLAG_RESORT]) return;
    for (int t = threadIdx.x; t < D.ntiles; t += blockDim.x) {
        const int tx = t % D.nt[0], r = t / D.nt[0];
        const int ty = r % D.nt[1], tz = r / D.nt[1];
        const int tc[3] = {tx, ty, tz};
        for (int a = 0; a < 3; a++) {
            const int lo = tc[a] * D.tile[a];
            D.tbox[t * 6 + a] = lo;
            D.tbox[t * 6 + 3 + a] = min(D.tile[a], D.n[a] - lo);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        D.flags[FLAG_RESORT] = 0;
        if (!force) D.flags[FLAG_NRESORT] += 1;
    }
}

// ------------------------------------------------------------- diagnostics

template <class R> __device__ __forceinline__ bool finite_r(R v) { return isfinite(v); }

__device__ __forceinline__ void block_sum_to(double v, double *dst)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && v != 0.0) unsafeAtomicAdd(dst, v);
}

#define ENERGY_ITEMS 16

// 1/2 sum E_c^2 dV and 1/2 sum B_c^2 dV; a block covers ENERGY_ITEMS field
// chunks (all of one instance or split where instances change)
template <class R>
__global__ void __launch_bounds__(256) k_energy(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work,
                                                int nwork, double *out, int out_stride, const int *pos, int cap,
                                                int par)
{
    const int it0 = blockIdx.x * ENERGY_ITEMS, it1 = min(nwork, it0 + ENERGY_ITEMS);
    int inst = work[it0].x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    double bad = 0.0;
    for (int it = it0; it <= it1; it++) {
        const bool flush = it == it1 || work[it].x != inst;
        if (flush) {
            // wave-uniform: every lane sees the same item sequence
            const InstDesc &D = Dt[inst];
            double *dst = pos ? out + ((size_t)(*pos % cap) * out_stride + inst) * 6 : D.diag;
            const double h = 0.5 * D.dV;
            for (int c = 0; c < 6; c++) { block_sum_to(h * v[c], dst + c); v[c] = 0.0; }
            if (!pos) block_sum_to(bad, D.diag + DG_NONFIN);
            bad = 0.0;
            if (it == it1) break;
            inst = work[it].x;
        }
        const InstDesc &D = Dt[inst];
        const int cell = work[it].y * PIC_FIELD_CHUNK + threadIdx.x;
        if (cell < D.ncell) {
            for (int c = 0; c < 3; c++) {
                const double e = (double)G<R>((const void *)D.E[par][c])[cell];
                const double b = (double)G<R>((const void *)D.B[par][c])[cell];
                v[c] += e * e;
                v[3 + c] += b * b;
                if (!isfinite(e) || !isfinite(b)) bad = 1.0;
            }
        }
    }
}

// charge density (order-L shape on integer nodes) of the current particles,
// plus kinetic energy and non-finite momenta
// block-wide sum / maximum into one global word (one atomic per block); red is
// an LDS scratch of one double per wave
__device__ __forceinline__ void block_atomic_sum(double v, double *dst, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) t += red[i];
        if (t != 0.0) unsafeAtomicAdd(dst, t);
    }
    __syncthreads();
}
__device__ __forceinline__ void block_atomic_max(double v, double *dst, double *red)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) t = fmax(t, red[i]);
        atomic_max_pos(dst, t);
    }
    __syncthreads();
}

// Charge density (order-L B-spline on the nodes) and kinetic energy, one particle
// tile per work item: the tile's nodes are accumulated in an LDS window (double
// atomics) and flushed once, as the particle kernel does for J.
template <int DIM, int L, class R>
__global__ void __launch_bounds__(256) k_rho(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work, int nwork,
                                             int wmx, int wmy, int wmz, int to_rho0, int with_kin)
{
    constexpr int JL = (L + 1) / 2, H = (L - 1) / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    double *srho = reinterpret_cast<double *>(smem);
    __shared__ double red[8];
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int item = blockIdx.x; item < nwork; item += gridDim.x) {
        const int inst = work[item].x, tile = work[item].y;
        const InstDesc &D = Dt[inst];
        const int p0 = D.tstart[tile], p1 = D.tstart[tile + 1];
        if (p1 <= p0) continue;
        int lo[3], o[3], wn[3];
        for (int a = 0; a < 3; a++) {
            lo[a] = D.tbox[tile * 6 + a];
            const int ext = D.tbox[tile * 6 + 3 + a];
            if (DIM == 2 && a == 1) { o[a] = 0; wn[a] = 1; continue; }
            o[a] = wrapi(lo[a] - JL, D.n[a]);
            wn[a] = ext + L + 2;
        }
        const int nn[3] = {D.n[0], D.n[1], D.n[2]};
        const bool fits = wn[0] <= wmx && wn[1] <= wmy && wn[2] <= wmz;
        const int wc = wn[0] * wn[1] * wn[2];
        if (fits)
            for (int c = tid; c < wc; c += bs) srho[c] = 0.0;
        __syncthreads();
        double *rho = to_rho0 ? D.rho0 : D.rho;
        const double rc = D.rho_c;
        double kin = 0.0, bad = 0.0;
        for (int p = p0 + tid; p < p1; p += bs) {
            int c[3];
            unpack_cell<DIM>((unsigned)D.pidx[p], c);
            double w[3][L + 1];
            int lc[3] = {0, 0, 0};
            for (int a = 0; a < 3; a++) {
                if (DIM == 2 && a == 1) { w[a][0] = 1.0; continue; }
                Shape<L, double>::integer((double)((const R *)D.poff[a])[p], w[a]);
                int rel = c[a] - lo[a];
                rel += rel < 0 ? nn[a] : 0;
                lc[a] = rel + JL - H;
            }
            const int NY = DIM == 3 ? L + 1 : 1;
            for (int kz = 0; kz < L + 1; kz++)
                for (int ky = 0; ky < NY; ky++)
                    for (int kx = 0; kx < L + 1; kx++) {
                        const double v = rc * w[0][kx] * (DIM == 3 ? w[1][ky] : 1.0) * w[2][kz];
                        const int x = lc[0] + kx, y = DIM == 3 ? lc[1] + ky : 0, z = lc[2] + kz;
                        if (fits) {
                            unsafeAtomicAdd(&srho[(z * wn[1] + y) * wn[0] + x], v);
                        } else {
                            const int gx = (o[0] + x) % nn[0], gy = (o[1] + y) % nn[1], gz = (o[2] + z) % nn[2];
                            unsafeAtomicAdd(&rho[(gz * nn[1] + gy) * nn[0] + gx], v);
                        }
                    }
            if (with_kin) {
                const double u0 = ((const R *)D.pu[0])[p], u1 = ((const R *)D.pu[1])[p], u2 = ((const R *)D.pu[2])[p];
                const double uu = u0 * u0 + u1 * u1 + u2 * u2;
                if (!isfinite(uu)) bad = 1.0;
                else kin += D.w * D.m * uu / (sqrt(1.0 + uu) + 1.0);   // gamma - 1 without cancellation
            }
        }
        __syncthreads();
        if (fits)
            for (int c = tid; c < wc; c += bs) {
                const double v = srho[c];
                if (v != 0.0) unsafeAtomicAdd(&rho[window_cell(c, wn, o, nn)], v);
            }
        if (with_kin) {
            block_atomic_sum(kin, D.diag + DG_WKIN, red);
            block_atomic_sum(bad, D.diag + DG_NONFIN, red);
        }
        __syncthreads();
    }
}

// Gauss residual after a step: div E^n - dt div J^{n+1/2} - (rho^{n+1} - rho^0)
#define GAUSS_ITEMS 16
template <int DIM, class R>
__global__ void __launch_bounds__(256) k_gauss(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work, int nwork,
                                               int par)
{
    typedef typename JGOf<R>::T JT;
    __shared__ double red[8];
    const int it0 = blockIdx.x * GAUSS_ITEMS, it1 = min(nwork, it0 + GAUSS_ITEMS);
    double g2 = 0.0, gmax = 0.0, chg = 0.0, rmax = 0.0;
    for (int it = it0; it < it1; it++) {
        const InstDesc &D = Dt[work[it].x];
        const int cell = work[it].y * PIC_FIELD_CHUNK + threadIdx.x;
        if (cell < D.ncell) {
            int i, j, k;
            cell_ijk<R>(D, cell, i, j, k);
            const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
            const int im = (i == 0 ? nx - 1 : i - 1) + (j + k * ny) * nx;
            const int km = i + (j + (k == 0 ? nz - 1 : k - 1) * ny) * nx;
            const R *E0 = (const R *)D.E[par][0], *E1 = (const R *)D.E[par][1], *E2 = (const R *)D.E[par][2];
            const JT *J0 = (const JT *)D.J[par][0], *J1 = (const JT *)D.J[par][1], *J2 = (const JT *)D.J[par][2];
            double divE = ((double)E0[cell] - (double)E0[im]) / D.d[0] + ((double)E2[cell] - (double)E2[km]) / D.d[2];
            double divJ = (jreal(J0[cell], D.jqg) - jreal(J0[im], D.jqg)) / D.d[0] +
                          (jreal(J2[cell], D.jqg) - jreal(J2[km], D.jqg)) / D.d[2];
            if (DIM == 3) {
                const int jm = i + ((j == 0 ? ny - 1 : j - 1) + k * ny) * nx;
                divE += ((double)E1[cell] - (double)E1[jm]) / D.d[1];
                divJ += (jreal(J1[cell], D.jqg) - jreal(J1[jm], D.jqg)) / D.d[1];
            }
            const double rho = D.rho[cell];
            const double res = divE - D.dt * divJ - (rho - D.rho0[cell]);
            g2 += res * res;
            gmax = fmax(gmax, fabs(res));
            chg += rho * D.dV;
            rmax = fmax(rmax, fabs(rho));
        }
        // flush at the block's last item or where the next item is another instance
        if (it + 1 == it1 || work[it + 1].x != work[it].x) {
            block_atomic_sum(g2, D.diag + DG_G2, red);
            block_atomic_sum(chg, D.diag + DG_CHARGE, red);
            block_atomic_max(gmax, D.diag + DG_GMAX, red);
            block_atomic_max(rmax, D.diag + DG_RHOMAX, red);
            g2 = gmax = chg = rmax = 0.0;
        }
    }
}

__global__ void k_zero_rho_diag(const InstDesc *__restrict__ Dt, const int2 *__restrict__ work, int rho0)
{
    const InstDesc &D = Dt[work[blockIdx.x].x];
    const int cell = work[blockIdx.x].y * PIC_FIELD_CHUNK + threadIdx.x;
    if (cell < D.ncell) (rho0 ? D.rho0 : D.rho)[cell] = 0.0;
    if (work[blockIdx.x].y == 0 && threadIdx.x < DG_COUNT && !rho0) D.diag[threadIdx.x] = 0.0;
}

__global__ void k_trace_tick(int *pos, double *trace, int n_inst, int cap)
{
    // advance the trace row and clear the next one
    const int next = (*pos + 1) % cap;
    for (int t = threadIdx.x; t < n_inst * 6; t += blockDim.x) trace[(size_t)next * n_inst * 6 + t] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) *pos += 1;
}


inline int hip_ok(hipError_t e) { return e == hipSuccess ? 0 : -1; }

}  // namespace

// ================================================================ launchers

#define DISPATCH_R(fp32, ...) \
    do { if (fp32) { typedef float R; __VA_ARGS__; } else { typedef double R; __VA_ARGS__; } } while (0)

template <class R, bool CK> void launch_yee_2d_s(const LaunchCtx &c, const int2 *ywork, int nywork)
{
    const dim3 g(nywork), b(PIC_FIELD_CHUNK);
    if (c.single) ywork = nullptr;
    if (c.yee_tz == 4) k_yee_2d<R, 4, CK><<<g, b, 0, c.stream>>>(c.desc, ywork, nywork, c.par);
    else if constexpr (sizeof(R) == 4) {
        if (c.yee_tz == 16) k_yee_2d<R, 16, CK><<<g, b, 0, c.stream>>>(c.desc, ywork, nywork, c.par);
        else k_yee_2d<R, 8, CK><<<g, b, 0, c.stream>>>(c.desc, ywork, nywork, c.par);
    } else {
        // 16 rows of doubles exceed the LDS
        k_yee_2d<R, 8, CK><<<g, b, 0, c.stream>>>(c.desc, ywork, nywork, c.par);
    }
}

template <class R> void launch_yee_2d(const LaunchCtx &c, const int2 *ywork, int nywork)
{
    if (c.ck) launch_yee_2d_s<R, true>(c, ywork, nywork);
    else launch_yee_2d_s<R, false>(c, ywork, nywork);
}

int launch_yee(const LaunchCtx &c, const int2 *fwork, int nwork, const int2 *ywork, int nywork)
{
    if (nwork <= 0) return 0;
    dim3 g(nwork), b(PIC_FIELD_CHUNK);
    DISPATCH_R(c.fp32, {
        if (c.dims == 2) {
            launch_yee_2d<R>(c, ywork, nywork);
        } else {
            const int p = c.par, q = c.par ^ 1;
            k_yee_b<3, R><<<g, b, 0, c.stream>>>(c.desc, fwork, p, p, q);
            k_yee_e<3, R><<<g, b, 0, c.stream>>>(c.desc, fwork, p, q);
            k_yee_b<3, R><<<g, b, 0, c.stream>>>(c.desc, fwork, q, q, q);
        }
    });
    return hip_ok(hipGetLastError());
}

size_t seen_smem_bytes(int fp32, int tz, int hz, int hx)
{
    const int wx = SEEN_TX + 2 * hx, wz = tz + 2 * hz;
    return (size_t)(wx * wz + SEEN_TX * wz + 2 * PIC_MAX_HZ + 1 + 2 * PIC_MAX_HX + 1) * (fp32 ? 4 : 8);
}

template <class R, int TZ>
void launch_seen_2d_tz(const LaunchCtx &c, const int2 *swork, int nswork)
{
    // instances with different stencils (c.hz < 0) size the window for the widest
    const size_t sm = seen_smem_bytes(c.fp32, TZ, c.hz < 0 ? PIC_MAX_HZ : c.hz, c.hx < 0 ? PIC_MAX_HX : c.hx);
    const dim3 g(nswork, 6), b(PIC_FIELD_CHUNK);
    if (c.single) swork = nullptr;
    // half-widths: correction of degree 4 with four filter passes (8, 4);
    // filter alone (4, 4); correction alone (4, 0); neither (0, 0); the first
    // with the node average of the momentum-conserving gather (9, 5)
    if (c.hz == 8 && c.hx == 4) k_seen_2d<R, TZ, 8, 4><<<g, b, sm, c.stream>>>(c.desc, swork, c.par);
    else if (c.hz == 9 && c.hx == 5) k_seen_2d<R, TZ, 9, 5><<<g, b, sm, c.stream>>>(c.desc, swork, c.par);
    else if (c.hz == 4 && c.hx == 4) k_seen_2d<R, TZ, 4, 4><<<g, b, sm, c.stream>>>(c.desc, swork, c.par);
    else if (c.hz == 4 && c.hx == 0) k_seen_2d<R, TZ, 4, 0><<<g, b, sm, c.stream>>>(c.desc, swork, c.par);
    else if (c.hz == 0 && c.hx == 0) k_seen_2d<R, TZ, 0, 0><<<g, b, sm, c.stream>>>(c.desc, swork, c.par);
    else k_seen_2d<R, TZ, -1, -1><<<g, b, sm, c.stream>>>(c.desc, swork, c.par);
}

// returns nonzero for a tile height the work list cannot serve
template <class R>
int launch_seen_2d(const LaunchCtx &c, const int2 *swork, int nswork)
{
    if constexpr (sizeof(R) == 4) {
        // 128-row segments streamed in 32-row chunks (the usual stencil widths)
        if (c.seen_tz == 128 && ((c.hz == 8 && c.hx == 4) || (c.hz == 9 && c.hx == 5))) {
            const dim3 g(nswork, 6), b(512);
            const int2 *w = c.single ? nullptr : swork;
            if (c.hz == 8) k_seen_2d_stream<R, 128, 8, 4><<<g, b, 0, c.stream>>>(c.desc, w, c.par);
            else k_seen_2d_stream<R, 128, 9, 5><<<g, b, 0, c.stream>>>(c.desc, w, c.par);
            return 0;
        }
    }
    // the host sets a tile height of 128 only with the streamed pass's widths
    // (its work list holds PIC_SEEN_SW-wide strips)
    if (c.seen_tz == 128) return 1;
    if (c.seen_tz == 8) launch_seen_2d_tz<R, 8>(c, swork, nswork);
    else if (c.seen_tz == 16) launch_seen_2d_tz<R, 16>(c, swork, nswork);
    else if constexpr (sizeof(R) == 4) {
        // 64 rows of doubles with the widest stencils exceed 64 KB of LDS
        if (c.seen_tz == 64) launch_seen_2d_tz<R, 64>(c, swork, nswork);
        else launch_seen_2d_tz<R, 32>(c, swork, nswork);
    } else launch_seen_2d_tz<R, 32>(c, swork, nswork);
    return 0;
}

int launch_seen(const LaunchCtx &c, const int2 *fwork, int nwork, const int2 *swork, int nswork)
{
    if (nwork <= 0) return 0;
    dim3 g(nwork, 6), b(PIC_FIELD_CHUNK);
    DISPATCH_R(c.fp32, {
        if (c.dims == 2) {
            if (launch_seen_2d<R>(c, swork, nswork)) return 1;
        } else {
            // usual widths: correction of degree 4 with four filter passes (z 8, x and y 4),
            // one more with the node average of the momentum-conserving gather
            // z and y: column passes; x (contiguous): one cell per thread
            const dim3 gz(c.col_blocks[0], 6, c.ninst), gy(c.col_blocks[1], 6, c.ninst);
            const dim3 gx(c.x_blocks, 6, c.ninst);
            if (c.hz == 8 && c.hx == 4) {
                k_seen_col<2, R, 8, PIC_COL_RUN><<<gz, b, 0, c.stream>>>(c.desc, c.inst0, 0, 1, c.par);
                k_seen_x<R, 4><<<gx, b, 0, c.stream>>>(c.desc, c.inst0, 1, 2, c.par);
                k_seen_col<1, R, 4, PIC_COL_RUN><<<gy, b, 0, c.stream>>>(c.desc, c.inst0, 2, 0, c.par);
            } else if (c.hz == 9 && c.hx == 5) {
                k_seen_col<2, R, 9, PIC_COL_RUN><<<gz, b, 0, c.stream>>>(c.desc, c.inst0, 0, 1, c.par);
                k_seen_x<R, 5><<<gx, b, 0, c.stream>>>(c.desc, c.inst0, 1, 2, c.par);
                k_seen_col<1, R, 5, PIC_COL_RUN><<<gy, b, 0, c.stream>>>(c.desc, c.inst0, 2, 0, c.par);
            } else {
                k_seen_pass<2, R, -1><<<g, b, 0, c.stream>>>(c.desc, fwork, 0, 1, c.par);
                k_seen_pass<0, R, -1><<<g, b, 0, c.stream>>>(c.desc, fwork, 1, 2, c.par);
                k_seen_pass<1, R, -1><<<g, b, 0, c.stream>>>(c.desc, fwork, 2, 0, c.par);
            }
        }
        if (c.ratio && c.rtiles > 0) {
            // the exact-ratio variant: the transverse E then get Psi_B(S_z)^{-1}
            k_psi_inv_z<R><<<dim3(c.rtiles, c.ninst, 2), dim3(64 * PIC_RATIO_TC), 0, c.stream>>>(c.desc, c.inst0);
        }
    });
    return hip_ok(hipGetLastError());
}

size_t particle_smem_bytes(int dims, int fp32, const int wmax[3])
{
    const size_t wc = (size_t)wmax[0] * (dims == 3 ? wmax[1] : 1) * wmax[2];
    const size_t r = fp32 ? 4 : 8;
    const size_t jb = (dims == 3 && fp32) ? 4 : 8;   // LDS current sums (see particles_body)
    return wc * (3 * jb + 6 * r);
}

// the deferred-tile pass for the gather scheme in use
template <class R, int D, int L, bool TP> void launch_deferred(const LaunchCtx &c, dim3 g)
{
    const int *dl = c.defer;
    if (c.gather == GATHER_UNIFORM) k_particles_deferred<D, L, R, TP, GATHER_UNIFORM><<<g, 256, 0, c.stream>>>(c.desc, c.par, dl);
    else if constexpr (!TP) {
        if (c.gather == GATHER_NODAL) k_particles_deferred<D, L, R, false, GATHER_NODAL><<<g, 256, 0, c.stream>>>(c.desc, c.par, dl);
        else k_particles_deferred<D, L, R, false, GATHER_GALERKIN><<<g, 256, 0, c.stream>>>(c.desc, c.par, dl);
    } else k_particles_deferred<D, L, R, true, GATHER_GALERKIN><<<g, 256, 0, c.stream>>>(c.desc, c.par, dl);
}

// one launch of the particle kernel in mode M (3D is always launched deferring)
template <int M>
void launch_particles_m(const LaunchCtx &c, const int2 *pwork, int nwork, dim3 g, dim3 b, size_t smem, const int *wm)
{
    const int2 *w = c.single ? nullptr : pwork;
#define PK(D_, L_, P_) k_particles<D_, L_, R, P_, false, false, GATHER_GALERKIN, M><<<g, b, smem, c.stream>>>(c.desc, w, nwork, wm[0], wm[1], wm[2], c.par)
#define PK24(K_, PF_) K_<2, 1, float, 24, PF_><<<g, b, smem, c.stream>>>(c.desc, w, nwork, wm[0], wm[1], wm[2], c.par)
#define PKR(L_, P_) k_particles<2, L_, R, P_, false, true, GATHER_GALERKIN, M><<<g, b, smem, c.stream>>>(c.desc, w, nwork, wm[0], wm[1], wm[2], c.par)
#define PKS(D_, L_, P_, IP_) k_particles<D_, L_, R, P_, false, false, IP_, M><<<g, b, smem, c.stream>>>(c.desc, w, nwork, wm[0], wm[1], wm[2], c.par)
#define PKRU(L_, P_) k_particles<2, L_, R, P_, false, true, GATHER_UNIFORM, M><<<g, b, smem, c.stream>>>(c.desc, w, nwork, wm[0], wm[1], wm[2], c.par)
#define PK_SCHEME(IP_)                                                              \
    do {                                                                            \
        if (c.dims == 2 && c.order == 1) {                                          \
            if (wm[0] == 24 && wm[2] == 24) PKS(2, 1, 24, IP_);                     \
            else if (wm[0] == 32 && wm[2] == 32) PKS(2, 1, 32, IP_);                \
            else PKS(2, 1, 0, IP_);                                                 \
        } else if (c.dims == 2) {                                                   \
            if (wm[0] == 32 && wm[2] == 32) PKS(2, 3, 32, IP_);                     \
            else PKS(2, 3, 0, IP_);                                                 \
        } else if constexpr (M == PM_DEFER) {                                       \
            if (c.order == 1) PKS(3, 1, 0, IP_);                                    \
            else if (wm[0] == 15 && wm[1] == 9 && wm[2] == 11) PKS(3, 3, 150911, IP_); \
            else PKS(3, 3, 0, IP_);                                                 \
        }                                                                           \
    } while (0)
    DISPATCH_R(c.fp32, {
        if (c.gather == GATHER_UNIFORM && c.record && c.dims == 2) {
            // recording a tape slot (2D reverse sweep) with the Uniform gather
            if (c.order == 1) {
                if (wm[0] == 24 && wm[2] == 24) PKRU(1, 24);
                else if (wm[0] == 32 && wm[2] == 32) PKRU(1, 32);
                else PKRU(1, 0);
            } else {
                if (wm[0] == 32 && wm[2] == 32) PKRU(3, 32);
                else PKRU(3, 0);
            }
        } else if (c.gather == GATHER_UNIFORM) {
            PK_SCHEME(GATHER_UNIFORM);
        } else if (c.gather == GATHER_NODAL) {
            PK_SCHEME(GATHER_NODAL);
        } else if (c.record && c.dims == 2) {
            // recording a tape slot (2D reverse sweep)
            if (c.order == 1) {
                if (wm[0] == 24 && wm[2] == 24 && M == PM_INLINE && c.fp32 && c.waves4)
                    k_particles_w4<2, 1, float, 24, false, true><<<g, b, smem, c.stream>>>(c.desc, w, nwork, wm[0],
                                                                                            wm[1], wm[2], c.par);
                else if (wm[0] == 24 && wm[2] == 24) PKR(1, 24);
                else if (wm[0] == 32 && wm[2] == 32) PKR(1, 32);
                else PKR(1, 0);
            } else {
                if (wm[0] == 32 && wm[2] == 32) PKR(3, 32);
                else PKR(3, 0);
            }
        } else if (c.dims == 2 && c.order == 1) {
            if (wm[0] == 24 && wm[2] == 24) {
                // the tuning variants exist in the inline mode only
                if (M == PM_INLINE && c.fp32 && c.waves4 && c.prefetch) PK24(k_particles_w4, true);
                else if (M == PM_INLINE && c.fp32 && c.waves4) PK24(k_particles_w4, false);
                else if (M == PM_INLINE && c.fp32 && c.prefetch) PK24(k_particles, true);
                else PK(2, 1, 24);
            } else if (wm[0] == 32 && wm[2] == 32) PK(2, 1, 32);
            else PK(2, 1, 0);
        } else if (c.dims == 2 && c.order == 3) {
            if (wm[0] == 32 && wm[2] == 32) PK(2, 3, 32);
            else PK(2, 3, 0);
        } else if constexpr (M == PM_DEFER) {
            if (c.order == 1) PK(3, 1, 0);
            else if (wm[0] == 15 && wm[1] == 9 && wm[2] == 11) PK(3, 3, 150911);
            else PK(3, 3, 0);
        }
    });
#undef PK
#undef PK24
#undef PKR
#undef PKS
#undef PKRU
#undef PK_SCHEME
}

int launch_particles(const LaunchCtx &c, const int2 *pwork, int nwork, int grid, int block, const int wmax[3])
{
    if (nwork <= 0) return 0;
    const int wy = c.dims == 3 ? wmax[1] : 1;
    const int wm[3] = {wmax[0], wy, wmax[2]};
    const size_t smem = particle_smem_bytes(c.dims, c.fp32, wm);
    const dim3 g(grid > 0 ? grid : nwork), b(block);
    // Keeping the global-memory path out of the kernel lowers its registers (2D
    // linear FP32 72 against 126 VGPRs, 3D cubic 167 against 256 with spills)
    // and lets more waves share a SIMD, at the cost of a second launch per
    // step.  The extra waves pay only when tiles queue for slots; with at most
    // four tiles per compute unit the one-launch form is faster.
    const bool defer = c.dims == 3 || (c.defer_mode < 0 ? nwork > 4 * c.cus : c.defer_mode == 1);
    if (!defer) {
        launch_particles_m<PM_INLINE>(c, pwork, nwork, g, b, smem, wm);
        return hip_ok(hipGetLastError());
    }
    launch_particles_m<PM_DEFER>(c, pwork, nwork, g, b, smem, wm);
    // tiles whose window did not fit were left in the deferred list; when there
    // are none every block of this pass leaves after one read
    const dim3 gd(nwork < 128 ? nwork : 128);
    DISPATCH_R(c.fp32, {
        const bool rec = c.record && c.dims == 2;
        if (c.dims == 2 && c.order == 1) {
            if (rec) launch_deferred<R, 2, 1, true>(c, gd);
            else launch_deferred<R, 2, 1, false>(c, gd);
        } else if (c.dims == 2) {
            if (rec) launch_deferred<R, 2, 3, true>(c, gd);
            else launch_deferred<R, 2, 3, false>(c, gd);
        } else if (c.order == 1) launch_deferred<R, 3, 1, false>(c, gd);
        else launch_deferred<R, 3, 3, false>(c, gd);
    });
    return hip_ok(hipGetLastError());
}

int launch_resort(const LaunchCtx &c, const int2 *cwork, int ncwork, int inst0, int n_inst, int clear_any)
{
    if (ncwork <= 0) return 0;
    const int *any = c.any_resort;
    int *anyw = const_cast<int *>(any);
    dim3 g(ncwork < RESORT_GRID ? ncwork : RESORT_GRID), b(PIC_PART_CHUNK);
    if (c.dims == 2) k_resort_count<2><<<g, b, 0, c.stream>>>(c.desc, cwork, ncwork, any);
    else k_resort_count<3><<<g, b, 0, c.stream>>>(c.desc, cwork, ncwork, any);
    k_resort_scan<<<dim3(n_inst), dim3(1024), 0, c.stream>>>(c.desc, inst0, any);
    DISPATCH_R(c.fp32, {
        if (c.dims == 2) {
            k_resort_scatter<2, R><<<g, b, 0, c.stream>>>(c.desc, cwork, ncwork, any);
            k_resort_copy<2, R><<<g, b, 0, c.stream>>>(c.desc, cwork, ncwork, any);
        } else {
            k_resort_scatter<3, R><<<g, b, 0, c.stream>>>(c.desc, cwork, ncwork, any);
            k_resort_copy<3, R><<<g, b, 0, c.stream>>>(c.desc, cwork, ncwork, any);
        }
    });
    k_resort_done<<<dim3(n_inst), dim3(256), 0, c.stream>>>(c.desc, inst0, 0, anyw, clear_any);
    return hip_ok(hipGetLastError());
}


// Several device-to-device copies in one launch (checkpoint saves and
// restores): 16-byte words, then each range's 4-byte tail.
__global__ void __launch_bounds__(256) k_copy_list(CopyList L)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (int k = 0; k < L.n; k++) {
        const long long n16 = L.bytes[k] / 16;
        const uint4 *s = (const uint4 *)L.src[k];
        uint4 *d = (uint4 *)L.dst[k];
        for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n16; i += stride) d[i] = s[i];
        const long long t4 = (L.bytes[k] - n16 * 16) / 4;
        if (blockIdx.x == 0 && threadIdx.x < t4)
            ((int *)L.dst[k])[n16 * 4 + threadIdx.x] = ((const int *)L.src[k])[n16 * 4 + threadIdx.x];
    }
}

int launch_copy_list(hipStream_t st, const CopyList &L)
{
    if (L.n <= 0) return 0;
    k_copy_list<<<dim3(1024), dim3(256), 0, st>>>(L);
    return hip_ok(hipGetLastError());
}

int launch_rho(const LaunchCtx &c, const int2 *pwork, int npwork, const int2 *fwork, int nfwork, const int wmax[3],
               int to_rho0)
{
    if (nfwork > 0)
        k_zero_rho_diag<<<dim3(nfwork), dim3(PIC_FIELD_CHUNK), 0, c.stream>>>(c.desc, fwork, to_rho0);
    if (npwork > 0) {
        const int wm[3] = {wmax[0], c.dims == 3 ? wmax[1] : 1, wmax[2]};
        const size_t sm = (size_t)wm[0] * wm[1] * wm[2] * sizeof(double);
        dim3 g(npwork), b(256);
#define RK(D_, L_) k_rho<D_, L_, R><<<g, b, sm, c.stream>>>(c.desc, pwork, npwork, wm[0], wm[1], wm[2], to_rho0, to_rho0 ? 0 : 1)
        DISPATCH_R(c.fp32, {
            if (c.dims == 2 && c.order == 1) RK(2, 1);
            else if (c.dims == 2 && c.order == 3) RK(2, 3);
            else if (c.dims == 3 && c.order == 1) RK(3, 1);
            else RK(3, 3);
        });
#undef RK
    }
    return hip_ok(hipGetLastError());
}

int launch_diag(const LaunchCtx &c, const int2 *fwork, int nfwork, const int2 *pwork, int npwork, const int wmax[3])
{
    // zero rho and the accumulators, deposit rho (+ kinetic energy), then the grid reductions
    if (launch_rho(c, pwork, npwork, fwork, nfwork, wmax, 0)) return -1;
    if (nfwork <= 0) return 0;
    dim3 b(PIC_FIELD_CHUNK);
    DISPATCH_R(c.fp32, {
        k_energy<R><<<dim3((nfwork + ENERGY_ITEMS - 1) / ENERGY_ITEMS), b, 0, c.stream>>>(c.desc, fwork, nfwork,
                                                                                      nullptr, 0, nullptr, 1, c.par);
        const dim3 gg((nfwork + GAUSS_ITEMS - 1) / GAUSS_ITEMS);
        if (c.dims == 2) k_gauss<2, R><<<gg, b, 0, c.stream>>>(c.desc, fwork, nfwork, c.par);
        else k_gauss<3, R><<<gg, b, 0, c.stream>>>(c.desc, fwork, nfwork, c.par);
    });
    return hip_ok(hipGetLastError());
}

int launch_trace_rows(const LaunchCtx &c, const int2 *fwork, int nfwork, int *pos, double *trace, int n_inst,
                      int cap)
{
    if (nfwork <= 0 || cap <= 0) return 0;
    DISPATCH_R(c.fp32, {
        k_energy<R><<<dim3((nfwork + ENERGY_ITEMS - 1) / ENERGY_ITEMS), dim3(PIC_FIELD_CHUNK), 0, c.stream>>>(
            c.desc, fwork, nfwork, trace, n_inst, pos, cap, c.par);
    });
    k_trace_tick<<<dim3(1), dim3(256), 0, c.stream>>>(pos, trace, n_inst, cap);
    return hip_ok(hipGetLastError());
}

int launch_fill_bbox(const LaunchCtx &c, int inst0, int n_inst)
{
    k_resort_done<<<dim3(n_inst), dim3(256), 0, c.stream>>>(c.desc, inst0, 1, const_cast<int *>(c.any_resort), 0);
    return hip_ok(hipGetLastError());
}
