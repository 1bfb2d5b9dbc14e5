// Device code of the feature pass shared by the per-call kernels (features.hip) and the batched
// persistent kernel (batch.hip).  See features.hip for the design notes.
#pragma once

#include <math.h>

#include "common.hpp"

namespace dvr {

constexpr int NT = 256;  // lanes per workgroup of the feature kernels

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ------------------------------------------------------------------------------------------------
// eigenvalues of a symmetric 3x3 matrix: closed-form trigonometric solution (Smith 1961) of the
// characteristic cubic of B = (A - m I) / p, m = tr A / 3, p^2 = tr((A - m I)^2) / 6.
template <typename T>
__device__ __forceinline__ void eig_trig(T a00, T a11, T a22, T a01, T a02, T a12, T &lmin, T &lmid, T &lmax)
{
    // constant divisors as products with their reciprocals (a few ulps, no division sequences)
    const T m = (a00 + a11 + a22) * T(1.0 / 3.0);
    const T b00 = a00 - m, b11 = a11 - m, b22 = a22 - m;
    const T p2 = (b00 * b00 + b11 * b11 + b22 * b22 + T(2) * (a01 * a01 + a02 * a02 + a12 * a12)) * T(1.0 / 6.0);
    if (!(p2 > T(0))) {
        lmin = lmid = lmax = m;
        return;
    }
    const T p = sqrt(p2);
    const T ip = T(1) / p;
    const T c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip, c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
    T q = T(0.5) * (c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02));
    q = q < T(-1) ? T(-1) : (q > T(1) ? T(1) : q);
    const T phi = acos(q) * T(1.0 / 3.0);
    // cos(phi + 2 pi / 3) = -cos(phi) / 2 - sin(phi) sqrt(3) / 2: one sincos instead of two cosines
    T sp, cp;
    if constexpr (sizeof(T) == 4) sincosf(phi, &sp, &cp);
    else sincos(phi, &sp, &cp);
    lmax = m + T(2) * p * cp;
    lmin = m - p * (cp + T(1.7320508075688772935) * sp);
    lmid = (a00 + a11 + a22) - lmax - lmin;
}

// Eigenvalues in FP32; re-solved in FP64 when the smallest gap is below tau * max|lambda|
// (the closed form loses accuracy as two roots merge).  Returned sorted by (|l|, l) ascending.
__device__ __forceinline__ void eig_sorted(const float A[6], float tau, float &l1, float &l2, float &l3)
{
    float lo, mi, hi;
    eig_trig<float>(A[0], A[1], A[2], A[3], A[4], A[5], lo, mi, hi);
    const float gap = fminf(hi - mi, mi - lo);
    const float scl = fmaxf(fabsf(hi), fabsf(lo));
    if (gap < tau * scl) {
        double dlo, dmi, dhi;
        eig_trig<double>(A[0], A[1], A[2], A[3], A[4], A[5], dlo, dmi, dhi);
        lo = (float)dlo;
        mi = (float)dmi;
        hi = (float)dhi;
    }
    // order by magnitude, the negative one first on an exact tie
    float a = lo, b = mi, c = hi, t;
#define DVR_KEY_LESS(u, v) (fabsf(u) < fabsf(v) || (fabsf(u) == fabsf(v) && (u) < (v)))
    if (DVR_KEY_LESS(b, a)) { t = a; a = b; b = t; }
    if (DVR_KEY_LESS(c, b)) { t = b; b = c; c = t; }
    if (DVR_KEY_LESS(b, a)) { t = a; a = b; b = t; }
#undef DVR_KEY_LESS
    l1 = a;
    l2 = b;
    l3 = c;
}

// Frangi bright-tube vesselness of magnitude-sorted eigenvalues.
__device__ __forceinline__ float frangi(float l1, float l2, float l3, float inv2a2, float inv2b2, float inv2c2)
{
    if (l2 >= 0.f || l3 >= 0.f) return 0.f;
    // quotients through the hardware reciprocal (1 ulp) instead of IEEE division sequences
    const float Ra2 = (l2 * l2) * __builtin_amdgcn_rcpf(l3 * l3);
    const float Rb2 = (l1 * l1) * __builtin_amdgcn_rcpf(fabsf(l2 * l3));
    const float S2 = l1 * l1 + l2 * l2 + l3 * l3;
    return (-expm1f(-Ra2 * inv2a2)) * expf(-Rb2 * inv2b2) * (-expm1f(-S2 * inv2c2));
}

// ------------------------------------------------------------------------------------------------
// One-dimensional filters on a strided line of values v(m), m = -R..R (callers pass accessors).
// cls: 0 interior, 1 first voxel of the axis, 2 last voxel of the axis.
struct Line3 {
    float g, d1, d2;
};

template <typename AT, typename F>
__device__ __forceinline__ Line3 filt3(const AT &t, int cls, F &&v)
{
    Line3 o;
    const int R = t.R;
    const float c0 = v(0);
    float g = t.G[0] * c0;
    if (cls == 0) {
        float d1 = 0.f, d2 = t.D2[0] * c0;
        for (int m = 1; m <= R; ++m) {
            const float a = v(m), b = v(-m);
            g = fmaf(t.G[m], a + b, g);
            d2 = fmaf(t.D2[m], a + b, d2);
            d1 = fmaf(t.D1[m], a - b, d1);
        }
        o.d1 = d1;
        o.d2 = d2;
    } else {
        float d1 = 0.f, d2 = 0.f;
        for (int m = 1; m <= R; ++m) g = fmaf(t.G[m], v(m) + v(-m), g);
        if (cls == 1) {
            for (int m = -R; m <= R; ++m) {
                const float x = v(m);
                d1 = fmaf(t.E1[m + R], x, d1);
                d2 = fmaf(t.E2[m + R], x, d2);
            }
        } else {
            for (int m = -R; m <= R; ++m) {
                const float x = v(m);
                d1 = fmaf(t.E1[m + 1 + R], x, d1);
                d2 = fmaf(-t.E2[m + 1 + R], x, d2);
            }
        }
        o.d1 = d1;
        o.d2 = d2;
    }
    o.g = g;
    return o;
}

template <typename AT, typename F>
__device__ __forceinline__ float filtG(const AT &t, F &&v)
{
    float g = t.G[0] * v(0);
    for (int m = 1; m <= t.R; ++m) g = fmaf(t.G[m], v(m) + v(-m), g);
    return g;
}

template <typename AT, typename F>
__device__ __forceinline__ float filtD1(const AT &t, int cls, F &&v)
{
    const int R = t.R;
    float d = 0.f;
    if (cls == 0) {
        for (int m = 1; m <= R; ++m) d = fmaf(t.D1[m], v(m) - v(-m), d);
    } else if (cls == 1) {
        for (int m = -R; m <= R; ++m) d = fmaf(t.E1[m + R], v(m), d);
    } else {
        for (int m = -R; m <= R; ++m) d = fmaf(t.E1[m + 1 + R], v(m), d);
    }
    return d;
}

template <typename AT, typename F>
__device__ __forceinline__ Line3 filtGD1(const AT &t, int cls, F &&v)
{
    Line3 o;
    o.g = filtG(t, v);
    o.d1 = filtD1(t, cls, v);
    o.d2 = 0.f;
    return o;
}

template <typename AT, typename F>
__device__ __forceinline__ float filtD2(const AT &t, int cls, F &&v)
{
    const int R = t.R;
    float d = t.D2[0] * v(0);
    if (cls == 0) {
        for (int m = 1; m <= R; ++m) d = fmaf(t.D2[m], v(m) + v(-m), d);
    } else if (cls == 1) {
        d = 0.f;
        for (int m = -R; m <= R; ++m) d = fmaf(t.E2[m + R], v(m), d);
    } else {
        d = 0.f;
        for (int m = -R; m <= R; ++m) d = fmaf(-t.E2[m + 1 + R], v(m), d);
    }
    return d;
}



__device__ __forceinline__ void atomic_max_pos(float *addr, float v)
{
    // non-negative floats order like their bit patterns; skip the atomic when it cannot win
    if (v > __hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(reinterpret_cast<unsigned int *>(addr), __float_as_uint(v));
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

template <int OUT_DT>
__device__ __forceinline__ void st(void *p, uint32_t idx, float v)
{
    if constexpr (OUT_DT == DVR_F32) reinterpret_cast<float *>(p)[idx] = v;
    else reinterpret_cast<__half *>(p)[idx] = __float2half_rn(v);
}

template <int OUT_DT>
__device__ __forceinline__ float ldo(const void *p, uint32_t idx)
{
    if constexpr (OUT_DT == DVR_F32) return reinterpret_cast<const float *>(p)[idx];
    else return __half2float(reinterpret_cast<const __half *>(p)[idx]);
}

struct XYArgs {
    const float *ws;
    const void *vol;
    void *grad, *kappa, *ves;
    float *gmax;
    float *fro;  // device scalar: max |sigma^2 H|_F (c <= 0 rule), or null
    int nx, ny, nz;
    float inv2h[3];
    float c_host;       // > 0: the Frangi c; otherwise c = fro/2 read from the device
    float inv2a2, inv2b2;
    float tau;
    int first, fro_pass;
};

// z filters of one voxel: (Gz, D1z, D2z) of I at in-plane index e of slice z.
template <int DT, typename AT>
__device__ __forceinline__ void zpass_voxel(const void *__restrict__ vol, float *__restrict__ ws, int nx, int ny,
                                            int nz, const AT &tz, uint32_t e, int z)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t N = plane * (uint32_t)nz;
    Buf b = make_buf(vol, N * ElemSize<DT>::v);
    auto v = [&](int m) -> float {
        const int zz = clampi(z + m, 0, nz - 1);
        return ldv<DT>(b, (uint32_t)zz * plane + e);
    };
    const int cls = (z == 0) ? 1 : (z == nz - 1 ? 2 : 0);
    const Line3 o = filt3(tz, cls, v);
    const uint32_t i = (uint32_t)z * plane + e;
    ws[i] = o.g;
    ws[N + i] = o.d1;
    ws[2u * N + i] = o.d2;
}

// Per-voxel epilogue: from the Hessian H of the smoothed volume (Hxx, Hyy, Hzz, Hxy, Hxz, Hyz) and,
// on the first scale, the intensities In = (I, I[x+1], I[x-1], I[y+1], I[y-1], I[z+1], I[z-1])
// (clamped neighbours): the gradient (Eq. 2), k (Eq. 3), the eigenvalues of sigma^2 H and V.
// Updates vmax with this voxel's |g| (first scale) or |sigma^2 H|_F (Frangi-c pass).
template <int OUT_DT, int LAYOUT>
__device__ __forceinline__ void voxel_out(const XYArgs &a, float sigma2, const float H[6], const float In[7], uint32_t v,
                                          uint32_t N, float &vmax)
{
    if constexpr (LAYOUT == kHessianOut) {
        // the adjoint's recomputation: H itself, [6][N] FP32 in a.grad
        float *Ho = reinterpret_cast<float *>(a.grad);
#pragma unroll
        for (int e = 0; e < 6; ++e) Ho[(size_t)e * N + v] = H[e];
        return;
    }
    float A[6];
    for (int e = 0; e < 6; ++e) A[e] = sigma2 * H[e];
    if (a.fro_pass) {
        const float f2 = A[0] * A[0] + A[1] * A[1] + A[2] * A[2] + 2.f * (A[3] * A[3] + A[4] * A[4] + A[5] * A[5]);
        vmax = fmaxf(vmax, sqrtf(f2));
        return;
    }
    float gx_ = 0.f, gy_ = 0.f, gz_ = 0.f, kap = 0.f;
    const float Ival = In[0];
    if (a.first) {
        gx_ = (In[1] - In[2]) * a.inv2h[0];
        gy_ = (In[3] - In[4]) * a.inv2h[1];
        gz_ = (In[5] - In[6]) * a.inv2h[2];
        vmax = fmaxf(vmax, sqrtf(gx_ * gx_ + gy_ * gy_ + gz_ * gz_));
        const float gm = fmaxf(fabsf(gx_), fmaxf(fabsf(gy_), fabsf(gz_)));
        if (gm > 0.f) {
            const float ig = __builtin_amdgcn_rcpf(gm);
            const float u0 = gx_ * ig, u1 = gy_ * ig, u2 = gz_ * ig;
            const float num = H[0] * u0 * u0 + H[1] * u1 * u1 + H[2] * u2 * u2 +
                              2.f * (H[3] * u0 * u1 + H[4] * u0 * u2 + H[5] * u1 * u2);
            kap = num * __builtin_amdgcn_rcpf(u0 * u0 + u1 * u1 + u2 * u2);  // the sum is >= 1
        }
    }
    float l1, l2, l3;
    eig_sorted(A, a.tau, l1, l2, l3);
    float c = a.c_host;
    if (!(c > 0.f)) {
        c = 0.5f * __hip_atomic_load(a.fro, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!(c > 0.f)) c = 1.f;
    }
    float V = frangi(l1, l2, l3, a.inv2a2, a.inv2b2, 0.5f * __builtin_amdgcn_rcpf(c * c));
    if constexpr (LAYOUT == DVR_PLANAR) {
        if (!a.first) V = fmaxf(V, ldo<OUT_DT>(a.ves, v));
        else {
            st<OUT_DT>(a.grad, v, gx_);
            st<OUT_DT>(a.grad, N + v, gy_);
            st<OUT_DT>(a.grad, 2u * N + v, gz_);
            st<OUT_DT>(a.kappa, v, kap);
        }
        st<OUT_DT>(a.ves, v, V);
    } else if constexpr (LAYOUT == DVR_SPLIT) {
        if (!a.first) V = fmaxf(V, ldo<OUT_DT>(a.ves, v));
        else if constexpr (OUT_DT == DVR_F32) {
            reinterpret_cast<float4 *>(a.grad)[v] = make_float4(gx_, gy_, gz_, kap);
        } else {
            union { __half h[4]; uint2 u; } rec;
            rec.h[0] = __float2half_rn(gx_);
            rec.h[1] = __float2half_rn(gy_);
            rec.h[2] = __float2half_rn(gz_);
            rec.h[3] = __float2half_rn(kap);
            reinterpret_cast<uint2 *>(a.grad)[v] = rec.u;
        }
        st<OUT_DT>(a.ves, v, V);
    } else {
        if (!a.first) {
            V = fmaxf(V, ldo<OUT_DT>(a.grad, 8u * v + 5u));
            st<OUT_DT>(a.grad, 8u * v + 5u, V);
        } else if constexpr (OUT_DT == DVR_F32) {
            float4 *r = reinterpret_cast<float4 *>(a.grad) + 2u * v;
            r[0] = make_float4(Ival, gx_, gy_, gz_);
            r[1] = make_float4(kap, V, 0.f, 0.f);
        } else {
            union { __half h[8]; uint4 u; } rec;
            rec.h[0] = __float2half_rn(Ival);
            rec.h[1] = __float2half_rn(gx_);
            rec.h[2] = __float2half_rn(gy_);
            rec.h[3] = __float2half_rn(gz_);
            rec.h[4] = __float2half_rn(kap);
            rec.h[5] = __float2half_rn(V);
            rec.h[6] = __float2half_rn(0.f);
            rec.h[7] = __float2half_rn(0.f);
            reinterpret_cast<uint4 *>(a.grad)[v] = rec.u;
        }
    }
}

// y and x filters of one TX x TY tile of slice z from the staged z-filtered fields, then the
// per-voxel epilogue.  Returns this lane's contribution to |g|_max (first scale) or to
// max |sigma^2 H|_F (Frangi-c pass); the caller reduces it.  lds holds
// (3 (TY + 2 Ry) + 6 TY) (TX + 2 Rx) floats.  The taps may live in any address space (kernel
// arguments, or a device table read through the constant address space by the batched kernel).
template <int DT, int OUT_DT, int LAYOUT, int TX, int TY, typename ST>
__device__ __forceinline__ float xy_tile(const XYArgs &a, const ST &taps, int x0, int y0, int z, float *lds)
{
    const auto &tx = taps.ax[0];
    const auto &ty = taps.ax[1];
    const int Rx = tx.R, Ry = ty.R;
    const int W = TX + 2 * Rx, HH = TY + 2 * Ry;
    float *F = lds;                   // [3][HH][W]
    float *Fy = lds + 3 * HH * W;     // [6][TY][W]
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t N = plane * (uint32_t)nz;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    __syncthreads();  // the LDS of a previous tile may still be read by other waves
    // stage the z-filtered fields of the tile and its halo (clamped coordinates)
    for (int row = wv; row < 3 * HH; row += NT / 64) {
        const int f = row / HH, yy = row - f * HH;
        const int gy = clampi(y0 - Ry + yy, 0, ny - 1);
        const float *src = a.ws + (size_t)f * N + (size_t)z * plane + (size_t)gy * nx;
        for (int xx = lane; xx < W; xx += 64) F[row * W + xx] = src[clampi(x0 - Rx + xx, 0, nx - 1)];
    }
    __syncthreads();

    // y filters: rows of the tile, all W columns
    for (int yy = wv; yy < TY; yy += NT / 64) {
        const int gy = y0 + yy;
        const int cls = (gy == 0) ? 1 : (gy == ny - 1 ? 2 : 0);
        for (int xx = lane; xx < W; xx += 64) {
            auto f0 = [&](int m) { return F[(0 * HH + yy + Ry + m) * W + xx]; };
            auto f1 = [&](int m) { return F[(1 * HH + yy + Ry + m) * W + xx]; };
            auto f2 = [&](int m) { return F[(2 * HH + yy + Ry + m) * W + xx]; };
            const Line3 r0 = filt3(ty, cls, f0);     // Gy Gz, D1y Gz, D2y Gz
            const Line3 r1 = filtGD1(ty, cls, f1);   // Gy D1z, D1y D1z
            const float r2 = filtG(ty, f2);          // Gy D2z
            const int o = yy * W + xx;
            Fy[0 * TY * W + o] = r0.g;
            Fy[1 * TY * W + o] = r0.d1;
            Fy[2 * TY * W + o] = r0.d2;
            Fy[3 * TY * W + o] = r1.g;
            Fy[4 * TY * W + o] = r1.d1;
            Fy[5 * TY * W + o] = r2;
        }
    }
    __syncthreads();

    float vmax = 0.f;
    for (int p = threadIdx.x; p < TX * TY; p += NT) {
        const int yy = p / TX, xx = p - yy * TX;
        const int gx = x0 + xx, gy = y0 + yy;
        const bool live = gx < nx && gy < ny;
        const int cls = (gx == 0) ? 1 : (gx == nx - 1 ? 2 : 0);
        auto fy = [&](int k) { return [=](int m) { return Fy[k * TY * W + yy * W + xx + Rx + m]; }; };
        float H[6];
        H[0] = filtD2(tx, cls, fy(0));   // Hxx = D2x Gy Gz
        H[3] = filtD1(tx, cls, fy(1));   // Hxy = D1x D1y Gz
        H[1] = filtG(tx, fy(2));         // Hyy = Gx D2y Gz
        H[4] = filtD1(tx, cls, fy(3));   // Hxz = D1x Gy D1z
        H[5] = filtG(tx, fy(4));         // Hyz = Gx D1y D1z
        H[2] = filtG(tx, fy(5));         // Hzz = Gx Gy D2z
        if (!live) continue;
        const uint32_t v = (uint32_t)z * plane + (uint32_t)gy * nx + gx;
        float In[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (a.first) {
            Buf b = make_buf(a.vol, N * ElemSize<DT>::v);
            const uint32_t row = (uint32_t)z * plane + (uint32_t)gy * nx;
            In[0] = ldv<DT>(b, v);
            In[1] = ldv<DT>(b, row + clampi(gx + 1, 0, nx - 1));
            In[2] = ldv<DT>(b, row + clampi(gx - 1, 0, nx - 1));
            In[3] = ldv<DT>(b, (uint32_t)z * plane + (uint32_t)clampi(gy + 1, 0, ny - 1) * nx + gx);
            In[4] = ldv<DT>(b, (uint32_t)z * plane + (uint32_t)clampi(gy - 1, 0, ny - 1) * nx + gx);
            In[5] = ldv<DT>(b, (uint32_t)clampi(z + 1, 0, nz - 1) * plane + (uint32_t)gy * nx + gx);
            In[6] = ldv<DT>(b, (uint32_t)clampi(z - 1, 0, nz - 1) * plane + (uint32_t)gy * nx + gx);
        }
        voxel_out<OUT_DT, LAYOUT>(a, taps.sigma2, H, In, v, N, vmax);
    }
    return vmax;
}

// ------------------------------------------------------------------------------------------------
// Fixed-radius filters: the same sums as filt3 / filtG / filtD1 / filtD2 with the stencil radius R a
// compile-time constant, so the loops unroll and the taps are read at constant offsets.  The
// smoothing tap G[R] is exactly zero (R = r + 1), so its term is left out.
template <int R, typename F>
__device__ __forceinline__ float rG(const AxisTaps &t, F &&v)
{
    float g = t.G[0] * v(0);
#pragma unroll
    for (int m = 1; m < R; ++m) g = fmaf(t.G[m], v(m) + v(-m), g);
    return g;
}

template <int R, typename F>
__device__ __forceinline__ float rD1(const AxisTaps &t, int cls, F &&v)
{
    float d = 0.f;
    if (cls == 0) {
#pragma unroll
        for (int m = 1; m <= R; ++m) d = fmaf(t.D1[m], v(m) - v(-m), d);
    } else if (cls == 1) {
#pragma unroll
        for (int m = -R; m <= R; ++m) d = fmaf(t.E1[m + R], v(m), d);
    } else {
#pragma unroll
        for (int m = -R; m <= R; ++m) d = fmaf(t.E1[m + 1 + R], v(m), d);
    }
    return d;
}

template <int R, typename F>
__device__ __forceinline__ float rD2(const AxisTaps &t, int cls, F &&v)
{
    float d;
    if (cls == 0) {
        d = t.D2[0] * v(0);
#pragma unroll
        for (int m = 1; m <= R; ++m) d = fmaf(t.D2[m], v(m) + v(-m), d);
    } else if (cls == 1) {
        d = 0.f;
#pragma unroll
        for (int m = -R; m <= R; ++m) d = fmaf(t.E2[m + R], v(m), d);
    } else {
        d = 0.f;
#pragma unroll
        for (int m = -R; m <= R; ++m) d = fmaf(-t.E2[m + 1 + R], v(m), d);
    }
    return d;
}

template <int R, typename F>
__device__ __forceinline__ Line3 r3(const AxisTaps &t, int cls, F &&v)
{
    Line3 o;
    if (cls == 0) {
        const float c0 = v(0);
        float g = t.G[0] * c0, d1 = 0.f, d2 = t.D2[0] * c0;
#pragma unroll
        for (int m = 1; m <= R; ++m) {
            const float a = v(m), b = v(-m);
            if (m < R) g = fmaf(t.G[m], a + b, g);
            d2 = fmaf(t.D2[m], a + b, d2);
            d1 = fmaf(t.D1[m], a - b, d1);
        }
        o.g = g;
        o.d1 = d1;
        o.d2 = d2;
    } else {
        o.g = rG<R>(t, v);
        o.d1 = rD1<R>(t, cls, v);
        o.d2 = rD2<R>(t, cls, v);
    }
    return o;
}

// The TX x TY tile of slice z with x and y stencil radius R: the same sums as xy_tile, organized
// for latency: the intensity loads of the gradient go out first, then every staging load of the
// z-filtered fields (tile plus halo) before any LDS store, and the y-filter work is spread over all
// lanes.  One tile per workgroup (no leading barrier).
template <int R, int TX, int TY>
struct XYTileR {
    static constexpr int W = TX + 2 * R, HH = TY + 2 * R;
    static constexpr int NST = 3 * HH * W;  // staged values
    static constexpr int NFY = 6 * TY * W;  // y-filtered values
};

template <int DT, int OUT_DT, int LAYOUT, int R, int TX, int TY>
__device__ __forceinline__ float xy_tile_r(const XYArgs &a, const ScaleTaps &taps, int x0, int y0, int z, float *F,
                                           float *Fy)
{
    using T = XYTileR<R, TX, TY>;
    constexpr int W = T::W, HH = T::HH, NST = T::NST;
    constexpr int PER = (NST + NT - 1) / NT;
    constexpr int NV = TX * TY / NT;
    static_assert((TX * TY) % NT == 0, "whole voxels per lane");
    const AxisTaps &tx = taps.ax[0];
    const AxisTaps &ty = taps.ax[1];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t N = plane * (uint32_t)nz;
    const int t = threadIdx.x;

    float In[NV][7];
    if (a.first) {
        Buf b = make_buf(a.vol, N * ElemSize<DT>::v);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int p = t + NT * i;
            const int yy = p / TX, xx = p - yy * TX;
            // lanes past the volume edge load an in-range voxel; their results are not stored
            const int gx = min(x0 + xx, nx - 1), gy = min(y0 + yy, ny - 1);
            const uint32_t row = (uint32_t)z * plane + (uint32_t)gy * nx;
            In[i][0] = ldv<DT>(b, row + gx);
            In[i][1] = ldv<DT>(b, row + clampi(gx + 1, 0, nx - 1));
            In[i][2] = ldv<DT>(b, row + clampi(gx - 1, 0, nx - 1));
            In[i][3] = ldv<DT>(b, (uint32_t)z * plane + (uint32_t)clampi(gy + 1, 0, ny - 1) * nx + gx);
            In[i][4] = ldv<DT>(b, (uint32_t)z * plane + (uint32_t)clampi(gy - 1, 0, ny - 1) * nx + gx);
            In[i][5] = ldv<DT>(b, (uint32_t)clampi(z + 1, 0, nz - 1) * plane + (uint32_t)gy * nx + gx);
            In[i][6] = ldv<DT>(b, (uint32_t)clampi(z - 1, 0, nz - 1) * plane + (uint32_t)gy * nx + gx);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int k = 0; k < 7; ++k) In[i][k] = 0.f;
    }

    // stage the z-filtered fields of the tile and its halo (clamped coordinates)
    float tmp[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int p = t + NT * i;
        tmp[i] = 0.f;
        if (NST % NT == 0 || p < NST) {
            const int row = p / W, xx = p - row * W;
            const int f = row / HH, yy = row - f * HH;
            const int gy = clampi(y0 - R + yy, 0, ny - 1), gx = clampi(x0 - R + xx, 0, nx - 1);
            tmp[i] = a.ws[(size_t)f * N + (size_t)z * plane + (size_t)gy * nx + gx];
        }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int p = t + NT * i;
        if (NST % NT == 0 || p < NST) F[p] = tmp[i];
    }
    __syncthreads();

    // y filters: all TY rows x W columns of the tile
    for (int p = t; p < TY * W; p += NT) {
        const int yy = p / W, xx = p - yy * W;
        const int gy = y0 + yy;
        const int cls = (gy == 0) ? 1 : (gy == ny - 1 ? 2 : 0);
        auto f0 = [&](int m) { return F[(0 * HH + yy + R + m) * W + xx]; };
        auto f1 = [&](int m) { return F[(1 * HH + yy + R + m) * W + xx]; };
        auto f2 = [&](int m) { return F[(2 * HH + yy + R + m) * W + xx]; };
        const Line3 r0 = r3<R>(ty, cls, f0);  // Gy Gz, D1y Gz, D2y Gz
        const float r1g = rG<R>(ty, f1);       // Gy D1z
        const float r1d = rD1<R>(ty, cls, f1); // D1y D1z
        const float r2 = rG<R>(ty, f2);        // Gy D2z
        Fy[0 * TY * W + p] = r0.g;
        Fy[1 * TY * W + p] = r0.d1;
        Fy[2 * TY * W + p] = r0.d2;
        Fy[3 * TY * W + p] = r1g;
        Fy[4 * TY * W + p] = r1d;
        Fy[5 * TY * W + p] = r2;
    }
    __syncthreads();

    float vmax = 0.f;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int p = t + NT * i;
        const int yy = p / TX, xx = p - yy * TX;
        const int gx = x0 + xx, gy = y0 + yy;
        const bool live = gx < nx && gy < ny;
        const int cls = (gx == 0) ? 1 : (gx == nx - 1 ? 2 : 0);
        auto fy = [&](int k) { return [=](int m) { return Fy[k * TY * W + yy * W + xx + R + m]; }; };
        float H[6];
        H[0] = rD2<R>(tx, cls, fy(0));  // Hxx = D2x Gy Gz
        H[3] = rD1<R>(tx, cls, fy(1));  // Hxy = D1x D1y Gz
        H[1] = rG<R>(tx, fy(2));        // Hyy = Gx D2y Gz
        H[4] = rD1<R>(tx, cls, fy(3));  // Hxz = D1x Gy D1z
        H[5] = rG<R>(tx, fy(4));        // Hyz = Gx D1y D1z
        H[2] = rG<R>(tx, fy(5));        // Hzz = Gx Gy D2z
        if (!live) continue;
        const uint32_t v = (uint32_t)z * plane + (uint32_t)gy * nx + gx;
        voxel_out<OUT_DT, LAYOUT>(a, taps.sigma2, H, In[i], v, N, vmax);
    }
    return vmax;
}

template <int TX, int TY>
__host__ __device__ constexpr size_t xy_lds_floats(int Rx, int Ry)
{
    return (size_t)(3 * (TY + 2 * Ry) + 6 * TY) * (size_t)(TX + 2 * Rx);
}

}  // namespace dvr
