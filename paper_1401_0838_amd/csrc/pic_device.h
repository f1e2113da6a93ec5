// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include <climits>

#include "pic_internal.h"

namespace pic {

// ------------------------------------------------------------------ helpers

// current accumulator in LDS (JOf) and current planes in HBM (JGOf): in float
// mode a tile sums its particles' contributions in 64-bit fixed point and adds
// the sums, rounded to a coarser 32-bit fixed point, to HBM; integer sums do
// not depend on the order of the adds, so float runs are bitwise reproducible
template <class R> struct JOf;
template <> struct JOf<float> { typedef long long T; };   // 64-bit fixed point
template <> struct JOf<double> { typedef double T; };
template <class R> struct JGOf;
template <> struct JGOf<float> { typedef int T; };        // 32-bit fixed point
template <> struct JGOf<double> { typedef double T; };

__device__ __forceinline__ int wrapi(int i, int n)
{
    // i in (-n, 2n)
    return i < 0 ? i + n : (i >= n ? i - n : i);
}
// the same for i in (-n, 2n) through two unsigned minima: for i < 0, i + n is
// the smaller as unsigned; for i >= n, i - n is (four instructions, no compares)
__device__ __forceinline__ int wrapu(int i, int n)
{
    const unsigned a = min((unsigned)i, (unsigned)(i + n));
    return (int)min(a, a - (unsigned)n);
}

// loads and stores of data read or written once per step: non-temporal when NT
template <bool NT, class P> __device__ __forceinline__ auto sload(P p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return std::remove_cv_t<std::remove_reference_t<decltype(*p)>>(*p);
}
template <bool NT, class T, class P> __device__ __forceinline__ void sstore(T v, P p)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__device__ __forceinline__ void jadd(long long *p, long long v)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
}
__device__ __forceinline__ void jadd(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void jadd(int *p, int v) { atomicAdd(p, v); }

// contribution -> accumulator type (already scaled by 1/quantum in float mode)
// truncation toward zero (one instruction); the bias is below one quantum
__device__ __forceinline__ long long jcvt(float v, long long *) { return (long long)(int)v; }
// 32-bit sums (3D float) use a coarser quantum: rounded to nearest, unbiased
__device__ __forceinline__ int jcvt(float v, int *) { return __float2int_rn(v); }
__device__ __forceinline__ double jcvt(double v, double *) { return v; }

__device__ __forceinline__ double jreal(long long v, double q) { return (double)v * q; }
__device__ __forceinline__ double jreal(int v, double q) { return (double)v * q; }
__device__ __forceinline__ double jreal(double v, double) { return v; }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// atomic max of a non-negative double through its bit pattern
__device__ __forceinline__ void atomic_max_pos(double *p, double v)
{
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

// ----------------------------------------------------------- shape factors
// Weights of the centred B-spline of order O for a point a fraction d in
// [0,1) past its cell's lower node.
//   integer nodes (order L): node c - (L-1)/2 + j, j in [0, L+1)
//   half nodes (order L-1):  node c - (L-1)/2 + j + 1/2, j in [0, L)

template <int L, class R> struct Shape;

template <class R> struct Shape<1, R> {
    static __device__ __forceinline__ void integer(R d, R *w) { w[0] = R(1) - d; w[1] = d; }
    static __device__ __forceinline__ void half(R, R *w) { w[0] = R(1); }
};

template <class R> struct Shape<3, R> {
    static __device__ __forceinline__ void integer(R d, R *w)
    {
        R e = R(1) - d;
        w[0] = e * e * e * R(1.0 / 6.0);
        w[1] = R(2.0 / 3.0) - d * d + R(0.5) * d * d * d;
        w[2] = R(2.0 / 3.0) - e * e + R(0.5) * e * e * e;
        w[3] = d * d * d * R(1.0 / 6.0);
    }
    static __device__ __forceinline__ void half(R d, R *w)
    {
        R e = R(1) - d, h = d - R(0.5);
        w[0] = R(0.5) * e * e;
        w[1] = R(0.75) - h * h;
        w[2] = R(0.5) * d * d;
    }
};

// Workgroup barrier for LDS traffic only: waits for the wave's own LDS
// operations (lgkmcnt 0, vmcnt and expcnt left at their maxima) and meets the
// other waves at s_barrier.  Unlike __syncthreads() it does not wait for
// outstanding global loads, so loads issued for a later tile stay in flight
// across it; only for kernels whose threads share data through LDS alone.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
}

// Index of the calling wave in its block.  threadIdx.x >> 6 is the same on
// every lane of a wave, but the compiler does not know it; read from the first
// lane it is a scalar, and the row and address arithmetic that depends only on
// it runs on the scalar unit instead of the vector ALUs.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// -------------------------------------------------------- global pointers
// Pointers read from the descriptor are generic; casting them to the global
// address space makes the compiler emit global (not flat) loads, stores and
// atomics, so LDS and HBM waits are tracked separately.
template <class T> using gp = __attribute__((address_space(1))) T *;
template <class T> __device__ __forceinline__ gp<T> G(void *p) { return (gp<T>)p; }
template <class T> __device__ __forceinline__ gp<const T> G(const void *p) { return (gp<const T>)p; }
// base plus a 32-bit byte offset (zero-extended): with a uniform base the
// compiler addresses it as scalar base + vector offset
template <class T> __device__ __forceinline__ gp<T> lane_ptr(gp<T> base, unsigned byte_off)
{
    return (gp<T>)((__attribute__((address_space(1))) char *)base + byte_off);
}
template <class T> __device__ __forceinline__ gp<const T> lane_ptr(gp<const T> base, unsigned byte_off)
{
    return (gp<const T>)((const __attribute__((address_space(1))) char *)base + byte_off);
}

__device__ __forceinline__ void gatomic_add(gp<long long> p, long long v)
{
    __hip_atomic_fetch_add((gp<unsigned long long>)p, (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gatomic_add(gp<int> p, int v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gatomic_add(gp<double> p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gatomic_add(gp<float> p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Add a fixed-point current sum v (LDS quantum) to an HBM current word whose
// quantum is 2^s coarser: v is rounded to the nearest HBM quantum (ties up).
// Returns true when the sum or the word's new value leaves the 32-bit range
// (the add is then skipped or wraps, and the caller flags the instance).
__device__ __forceinline__ bool jflush(gp<int> p, long long v, int s)
{
    // s < 0: the HBM quantum is the finer one (exact)
    const long long r = s >= 0 ? (v + (s > 0 ? (1LL << (s - 1)) : 0)) >> s : v * (1LL << -s);
    if (r == 0) return false;
    if (r > INT_MAX || r < INT_MIN) return true;
    const int old = __hip_atomic_fetch_add(p, (int)r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long nw = (long long)old + r;
    return nw > INT_MAX || nw < INT_MIN;
}
__device__ __forceinline__ bool jflush(gp<double> p, double v, int)
{
    gatomic_add(p, v);
    return false;
}

// a float-mode current word outside +-2^30: the sum it holds may have wrapped
__device__ __forceinline__ bool jrange_bad(int v) { return (unsigned)v + (1u << 30) >= (1u << 31); }
__device__ __forceinline__ bool jrange_bad(double) { return false; }

// ------------------------------------------------------------ LDS staging
// For c in [0, n) and k < K:  dst[k * dpitch + dix(c)] = cv(k, src[k][addr(c)]).
// U iterations of the block-strided loop are unrolled and all their loads are
// issued before the first LDS store, so each thread keeps K * U global loads
// in flight (a plain loop waits for every load before the next).
template <int U, int K, class TS, class TD, class Addr, class Dix, class Cv>
__device__ __forceinline__ void stage(TD *dst, int dpitch, const gp<const TS> *src, int n, Addr addr, Dix dix, Cv cv)
{
    const int bs = blockDim.x;
    for (int c0 = threadIdx.x; c0 < n; c0 += U * bs) {
        int g[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int c = c0 + u * bs;
            g[u] = c < n ? addr(c) : 0;      // index 0 is always a valid address
        }
        TS v[U][K];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int k = 0; k < K; k++) v[u][k] = src[k][g[u]];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int c = c0 + u * bs;
            if (c < n) {
                const int d = dix(c);
#pragma unroll
                for (int k = 0; k < K; k++) dst[k * dpitch + d] = cv(k, v[u][k]);
            }
        }
    }
}

struct IdentityIx {
    __device__ __forceinline__ int operator()(int c) const { return c; }
};
struct PlainCv {
    template <class T> __device__ __forceinline__ T operator()(int, T v) const { return v; }
};

// periodic index by a remainder: no branch, for any g > -n * 2^20
__device__ __forceinline__ int pmod(int g, int n)
{
    const int r = (g + (n << 20)) % n;
    return r;
}

// periodic index g mod n by a multiply with a reciprocal taken once (a block's
// row and column wraps: a remainder costs a few tens of instructions, this five):
// with x = g + 16 n and m = floor((2^32 - 1) / n), the high word of x m is the
// quotient or one below it, so one conditional subtract finishes the
// remainder.  Exact for g in [-16 n, 2^31 - 16 n), n >= 1.
struct PerMod {
    unsigned n, m, off;
    __device__ __forceinline__ explicit PerMod(int n_)
        : n((unsigned)n_), m(0xFFFFFFFFu / (unsigned)n_), off(16u * (unsigned)n_) {}
    __device__ __forceinline__ int operator()(int g) const
    {
        const unsigned x = (unsigned)g + off;
        const unsigned r = x - __umulhi(x, m) * n;
        return (int)(r >= n ? r - n : r);
    }
};

// periodic index for g in [-n, 2n) (one compare each way), else a modulo
__device__ __forceinline__ int wrap_near(int g, int n)
{
    g += g < 0 ? n : 0;
    g -= g >= n ? n : 0;
    return (g < 0 || g >= n) ? ((g % n) + n) % n : g;
}

// reciprocal and reciprocal square root: hardware approximations (1 ulp) in
// float, exact division in double
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// ----------------------------------------------------- packed cell index
// 2D: x | z << 16 ;  3D: x | y << 11 | z << 21  (unsigned 32-bit)
template <int DIM> __host__ __device__ __forceinline__ unsigned pack_cell(int x, int y, int z)
{
    return DIM == 2 ? ((unsigned)x | ((unsigned)z << 16)) : ((unsigned)x | ((unsigned)y << 11) | ((unsigned)z << 21));
}
template <int DIM> __host__ __device__ __forceinline__ void unpack_cell(unsigned v, int *c)
{
    if (DIM == 2) { c[0] = (int)(v & 0xffffu); c[1] = 0; c[2] = (int)(v >> 16); }
    else { c[0] = (int)(v & 0x7ffu); c[1] = (int)((v >> 11) & 0x3ffu); c[2] = (int)(v >> 21); }
}

// ------------------------------------------------- Boris push and move
// Shared by the forward kernel and the adjoint's recomputation so both take
// bit-identical cell steps.
// x clamped into [-1, 2): the largest value below 2 is the upper bound
__device__ __forceinline__ float clamp_step(float x) { return __builtin_amdgcn_fmed3f(x, -1.0f, 0x1.fffffep0f); }
__device__ __forceinline__ double clamp_step(double x) { return fmin(fmax(x, -1.0), 0x1.fffffffffffffp0); }

template <class R> struct BorisTrace {
    R um[3], t[3], sv[3], up[3];
    R igm, f;
};

template <class R>
__device__ __forceinline__ void boris_push(const R *u, const R *E, const R *B, R qdt2m, R *un, BorisTrace<R> &b)
{
#pragma unroll
    for (int a = 0; a < 3; a++) b.um[a] = u[a] + qdt2m * E[a];
    b.igm = rsq(R(1) + b.um[0] * b.um[0] + b.um[1] * b.um[1] + b.um[2] * b.um[2]);
#pragma unroll
    for (int a = 0; a < 3; a++) b.t[a] = qdt2m * B[a] * b.igm;
    b.f = R(2) * rcp(R(1) + b.t[0] * b.t[0] + b.t[1] * b.t[1] + b.t[2] * b.t[2]);
#pragma unroll
    for (int a = 0; a < 3; a++) b.sv[a] = b.f * b.t[a];
    b.up[0] = b.um[0] + (b.um[1] * b.t[2] - b.um[2] * b.t[1]);
    b.up[1] = b.um[1] + (b.um[2] * b.t[0] - b.um[0] * b.t[2]);
    b.up[2] = b.um[2] + (b.um[0] * b.t[1] - b.um[1] * b.t[0]);
    un[0] = b.um[0] + (b.up[1] * b.sv[2] - b.up[2] * b.sv[1]) + qdt2m * E[0];
    un[1] = b.um[1] + (b.up[2] * b.sv[0] - b.up[0] * b.sv[2]) + qdt2m * E[1];
    un[2] = b.um[2] + (b.up[0] * b.sv[1] - b.up[1] * b.sv[0]) + qdt2m * E[2];
}

// new offsets and cell steps (cell units); returns 1/gamma of un
template <int DIM, class R>
__device__ __forceinline__ R move_cells(const R *off, const R *un, const R *dtd, int *dc, R *offn, int &err)
{
    const R ig = rsq(R(1) + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (DIM == 2 && a == 1) { dc[a] = 0; offn[a] = R(0); continue; }
        const R x = off[a] + dtd[a] * un[a] * ig;
        // More than one cell per step (c dt above the cell size) is an error:
        // flagged, and the position clamped into [-1, 2) to keep the state in
        // range (a NaN position is flagged the same way).
        const R x1 = clamp_step(x);
        err |= x1 != x;
        const R fl = floor(x1);
        int c = (int)fl;
        R on = x1 - fl;
        // x1 in [-1, 0): x1 + 1 may round up to 1
        if (on >= R(1)) { on -= R(1); c += 1; }
        dc[a] = c;
        offn[a] = on;
    }
    return ig;
}

// global cell of window cell c (window dims wn, origin o, grid n); the
// window may exceed the grid on tiny grids, hence the second wrap
__device__ __forceinline__ int window_cell(int c, const int *wn, const int *o, const int *n)
{
    const int wxy = wn[0] * wn[1];
    int z = (int)(((float)c + 0.5f) * (1.0f / (float)wxy));
    int r = c - z * wxy;
    int y = (int)(((float)r + 0.5f) * (1.0f / (float)wn[0]));
    int x = r - y * wn[0];
    int gx = o[0] + x, gy = o[1] + y, gz = o[2] + z;
    gx = gx >= n[0] ? gx - n[0] : gx;
    gy = gy >= n[1] ? gy - n[1] : gy;
    gz = gz >= n[2] ? gz - n[2] : gz;
    if (gx >= n[0] || gy >= n[1] || gz >= n[2]) { gx %= n[0]; gy %= n[1]; gz %= n[2]; }
    return (gz * n[1] + gy) * n[0] + gx;
}

// ------------------------------------------------------------ accessors
// Field / current access by window-local node coordinates.

template <class R, class JT> struct LdsWin {
    const R *F;   // 6 planes of wc values: Ex Ey Ez Bx By Bz (seen)
    JT *J;        // 3 planes
    int wx, wxy, wc;
    __device__ __forceinline__ int at(int x, int y, int z) const { return z * wxy + y * wx + x; }
    __device__ __forceinline__ R f(int comp, int x, int y, int z) const { return F[comp * wc + at(x, y, z)]; }
    __device__ __forceinline__ void add(int comp, int x, int y, int z, JT v) { jadd(&J[comp * wc + at(x, y, z)], v); }
};

// LDS window with compile-time pitches (PX cells per row, PY rows per plane,
// PZ planes; 2D: PY = 1): every node a particle touches is at a constant
// offset from one base address
template <class R, class JT, int PX, int PY, int PZ> struct LdsWinP {
    const R *F;
    JT *J;
    static constexpr int wc = PX * PY * PZ;
    __device__ __forceinline__ int at(int x, int y, int z) const { return (z * PY + y) * PX + x; }
    __device__ __forceinline__ R f(int comp, int x, int y, int z) const { return F[comp * wc + at(x, y, z)]; }
    __device__ __forceinline__ void add(int comp, int x, int y, int z, JT v) { jadd(&J[comp * wc + at(x, y, z)], v); }
};

// fields and current straight in global memory (a tile whose particles
// outgrew the LDS window): each contribution goes to the HBM current on its own
template <class R, class JT> struct GlbWin {
    typedef typename JGOf<R>::T JG;
    gp<const R> F[6];
    gp<JG> J[3];
    int o[3], n[3];
    int shift;          // LDS -> HBM quantum shift (float mode)
    bool ovf;           // some add left the 32-bit range
    __device__ __forceinline__ int at(int x, int y, int z) const
    {
        int gx = (o[0] + x) % n[0], gy = (o[1] + y) % n[1], gz = (o[2] + z) % n[2];
        return (gz * n[1] + gy) * n[0] + gx;
    }
    __device__ __forceinline__ R f(int comp, int x, int y, int z) const { return F[comp][at(x, y, z)]; }
    __device__ __forceinline__ void add(int comp, int x, int y, int z, JT v)
    {
        if (jflush(J[comp] + at(x, y, z), v, shift)) ovf = true;
    }
};


}  // namespace pic
