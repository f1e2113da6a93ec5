// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include "pic_internal.h"

namespace pic {

// ------------------------------------------------------------------ helpers

template <class R> struct JOf;
template <> struct JOf<float> { typedef long long T; };   // 64-bit fixed point
template <> struct JOf<double> { typedef double T; };

__device__ __forceinline__ int wrapi(int i, int n)
{
    // i in (-n, 2n)
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

__device__ __forceinline__ void jadd(long long *p, long long v)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
}
__device__ __forceinline__ void jadd(double *p, double v) { unsafeAtomicAdd(p, v); }

// contribution -> accumulator type (already scaled by 1/quantum in float mode)
__device__ __forceinline__ long long jcvt(float v, long long *) { return (long long)__float2int_rn(v); }
__device__ __forceinline__ double jcvt(double v, double *) { return v; }

__device__ __forceinline__ double jreal(long long v, double q) { return (double)v * q; }
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

template <class R, class JT> struct GlbWin {
    const R *F[6];
    JT *J[3];
    int o[3], n[3];
    __device__ __forceinline__ int at(int x, int y, int z) const
    {
        int gx = (o[0] + x) % n[0], gy = (o[1] + y) % n[1], gz = (o[2] + z) % n[2];
        return (gz * n[1] + gy) * n[0] + gx;
    }
    __device__ __forceinline__ R f(int comp, int x, int y, int z) const { return F[comp][at(x, y, z)]; }
    __device__ __forceinline__ void add(int comp, int x, int y, int z, JT v) { jadd(&J[comp][at(x, y, z)], v); }
};


}  // namespace pic
