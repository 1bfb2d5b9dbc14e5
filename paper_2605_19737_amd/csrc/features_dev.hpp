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

// Eigenvalues of a symmetric 3x3 matrix in FP32 with an accuracy of a few ulps of max|lambda| at any
// gap between them.  The closed form above takes cos(3 phi) from det(B) / p^3, whose rounding is
// amplified by ~p / gap where two roots merge.  Here the characteristic cubic of the traceless
// B = A - m I (m = tr A / 3) is solved through its two invariants J2 = tr(B^2) / 2, J3 = det B and
// its discriminant Delta = prod_{i<j} (lambda_i - lambda_j)^2 = 4 J2^3 - 27 J3^2, which is
// computed without that cancellation: Delta is the Gram determinant of the vectors I, B, B^2 under
// the Frobenius product (a Vandermonde determinant squared), so by Cauchy-Binet it is the sum of
// the squared 3x3 minors of [vec I; vec B; vec B^2] (off-diagonal coordinates weighted by sqrt 2):
//   Delta = M0^2 + 2 sum_{i<j, k} (c_k (b_jj - b_ii) - b_k (c_jj - c_ii))^2 + 12 sum_{k<l} (b_k c_l - b_l c_k)^2
// with C = B^2, M0 = c00 (b22 - b11) + c11 (b00 - b22) + c22 (b11 - b00), k, l over the
// off-diagonal entries.  Then 3 theta = atan2(sqrt Delta, 3 sqrt(3) J3) in [0, pi] and the roots
// are m + 2 p cos(theta + 2 pi j / 3), p = sqrt(J2 / 3).  B is first scaled by its largest entry
// (Delta is of degree 6 in B: no underflow or overflow), and the angle functions are polynomials
// on the ranges they are needed on (atan on [0, 1]; sin and cos on [0, pi/3]), least-squares fits
// with errors of 6e-9, 4e-11 and 8e-10, below FP32 resolution.  Returned in ascending order.
__device__ __forceinline__ float atan01(float t)
{
    const float u = t * t;
    float r = 0.0024567249f;
    r = fmaf(r, u, -0.014401361f);
    r = fmaf(r, u, 0.03978123f);
    r = fmaf(r, u, -0.07234859f);
    r = fmaf(r, u, 0.10498947f);
    r = fmaf(r, u, -0.14161229f);
    r = fmaf(r, u, 0.19985907f);
    r = fmaf(r, u, -0.33332598f);
    r = fmaf(r, u, 0.9999999f);
    return t * r;
}

__device__ __forceinline__ void eig_sym3(const float A[6], float &mu0, float &mu1, float &mu2)
{
    const float m = (A[0] + A[1] + A[2]) * (1.f / 3.f);
    const float e00 = A[0] - m, e11 = A[1] - m, e22 = A[2] - m;
    const float sc = fmaxf(fmaxf(fmaxf(fabsf(e00), fabsf(e11)), fmaxf(fabsf(e22), fabsf(A[3]))),
                           fmaxf(fabsf(A[4]), fabsf(A[5])));
    if (!(sc > 0.f)) {
        mu0 = mu1 = mu2 = m;
        return;
    }
    const float is = __builtin_amdgcn_rcpf(sc);
    const float b00 = e00 * is, b11 = e11 * is, b22 = e22 * is, b01 = A[3] * is, b02 = A[4] * is, b12 = A[5] * is;
    const float c00 = fmaf(b00, b00, fmaf(b01, b01, b02 * b02));
    const float c11 = fmaf(b01, b01, fmaf(b11, b11, b12 * b12));
    const float c22 = fmaf(b02, b02, fmaf(b12, b12, b22 * b22));
    const float c01 = fmaf(b00, b01, fmaf(b01, b11, b02 * b12));
    const float c02 = fmaf(b00, b02, fmaf(b01, b12, b02 * b22));
    const float c12 = fmaf(b01, b02, fmaf(b11, b12, b12 * b22));
    const float J2 = 0.5f * (c00 + c11 + c22);
    const float M0 = fmaf(c00, b22 - b11, fmaf(c11, b00 - b22, c22 * (b11 - b00)));
    const float db[3] = {b11 - b00, b22 - b00, b22 - b11};
    const float dc[3] = {c11 - c00, c22 - c00, c22 - c11};
    const float bo[3] = {b01, b02, b12}, co[3] = {c01, c02, c12};
    float sB = 0.f;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float t = fmaf(co[k], db[q], -bo[k] * dc[q]);
            sB = fmaf(t, t, sB);
        }
    const float t0 = fmaf(b01, c02, -b02 * c01), t1 = fmaf(b01, c12, -b12 * c01), t2 = fmaf(b02, c12, -b12 * c02);
    const float sC = fmaf(t0, t0, fmaf(t1, t1, t2 * t2));
    const float D = fmaf(M0, M0, fmaf(2.f, sB, 12.f * sC));
    const float J3 = b00 * fmaf(b11, b22, -b12 * b12) - b01 * fmaf(b01, b22, -b12 * b02) + b02 * fmaf(b01, b12, -b11 * b02);
    // 3 theta = atan2(y, x), y >= 0
    const float y = __builtin_amdgcn_sqrtf(D), x = 5.196152422706632f * J3;
    const float ax = fabsf(x), lo = fminf(ax, y), hi = fmaxf(ax, y);
    float a = hi > 0.f ? atan01(lo * __builtin_amdgcn_rcpf(hi)) : 0.f;
    if (y > ax) a = 1.5707963267948966f - a;
    if (x < 0.f) a = 3.141592653589793f - a;
    const float th = a * (1.f / 3.f), v = th * th;
    float sn = 2.6811283e-06f;
    sn = fmaf(sn, v, -0.00019833124f);
    sn = fmaf(sn, v, 0.008333295f);
    sn = fmaf(sn, v, -0.16666666f);
    sn = fmaf(sn, v, 1.f);
    sn *= th;
    float cs = 2.405656e-05f;
    cs = fmaf(cs, v, -0.0013881775f);
    cs = fmaf(cs, v, 0.04166639f);
    cs = fmaf(cs, v, -0.49999997f);
    cs = fmaf(cs, v, 1.f);
    const float p = sc * __builtin_amdgcn_sqrtf(J2 * (1.f / 3.f));
    mu2 = fmaf(2.f * p, cs, m);
    const float ps = 1.7320508075688772f * p * sn, pc = p * cs;
    mu0 = m - (pc + ps);
    mu1 = m - (pc - ps);
}

// FP64 re-solve of a near-degenerate spectrum: cyclic Jacobi rotations (each zeroes one
// off-diagonal entry), backward stable whatever the clustering of the roots (the characteristic
// polynomial of a near-triple root is too ill-conditioned to solve, even in FP64), and with no
// transcendental functions, so it stays light in registers.  Returned in ascending order.
__device__ __forceinline__ void eig_jacobi64(const float A[6], float &mu0, float &mu1, float &mu2)
{
    double d[3] = {A[0], A[1], A[2]};
    double o01 = A[3], o02 = A[4], o12 = A[5];
    // rotation in the (p, q) plane zeroing a_pq; r is the third index, a_rp and a_rq rotate with it
    auto rot = [&](double &app, double &aqq, double &apq, double &arp, double &arq) {
        if (apq == 0.0) return;
        const double th = (aqq - app) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(fma(th, th, 1.0)));
        const double c = 1.0 / sqrt(fma(t, t, 1.0)), sn = t * c;
        app -= t * apq;
        aqq += t * apq;
        apq = 0.0;
        const double rp = arp, rq = arq;
        arp = c * rp - sn * rq;
        arq = sn * rp + c * rq;
    };
    for (int sweep = 0; sweep < 6; ++sweep) {
        const double off = fabs(o01) + fabs(o02) + fabs(o12);
        if (off <= 1e-17 * (fabs(d[0]) + fabs(d[1]) + fabs(d[2]))) break;
        rot(d[0], d[1], o01, o02, o12);  // (p, q, r) = (0, 1, 2): a_r0 = a02, a_r1 = a12
        rot(d[0], d[2], o02, o01, o12);  // (0, 2, 1): a_r0 = a01, a_r2 = a12
        rot(d[1], d[2], o12, o01, o02);  // (1, 2, 0): a_r1 = a01, a_r2 = a02
    }
    const double lo = fmin(d[0], fmin(d[1], d[2])), hi = fmax(d[0], fmax(d[1], d[2]));
    mu0 = (float)lo;
    mu1 = (float)(d[0] + d[1] + d[2] - lo - hi);
    mu2 = (float)hi;
}

// |g| as the feature pass takes it (|g|_max is the largest of these; the adjoint finds its voxel with
// the same expression).  The square roots of this file are the hardware's (within 1 ulp).
__device__ __forceinline__ float grad_norm(float gx, float gy, float gz)
{
    return __builtin_amdgcn_sqrtf(gx * gx + gy * gy + gz * gz);
}

// Whether V can be non-zero at A = sigma^2 H.  With eigenvalues mu0 <= mu1 <= mu2, V != 0 exactly when
// mu1 + mu2 < 0 (that implies mu1 < 0), i.e. when tr(A) I - A, whose eigenvalues are the pair sums
// mu_i + mu_j, is negative definite: M = A - tr(A) I positive definite.  By Sylvester's criterion a
// positive definite M has positive leading principal minors m00, m00 m11 - m01^2 and det M, so a
// minor below minus a margin proves V = 0.  The margins (1e-4 s^k for the minor of order k, s the
// largest |m_ij|) are ~100 times the rounding of the minors and put mu1 + mu2 at >= 1e-5 s, far
// above the eigen-solve's error, so every voxel left out would also get V = 0 from its eigenvalues;
// the rest (about half of the voxels with tr(A) < 0) take the eigen-solve.
__device__ __forceinline__ bool maybe_vessel(const float A[6])
{
    const float t = A[0] + A[1] + A[2];
    if (!(t < 0.f)) return false;
    const float m00 = A[0] - t, m11 = A[1] - t, m22 = A[2] - t, m01 = A[3], m02 = A[4], m12 = A[5];
    const float s = fmaxf(fmaxf(fmaxf(fabsf(m00), fabsf(m11)), fmaxf(fabsf(m22), fabsf(m01))),
                          fmaxf(fabsf(m02), fabsf(m12)));
    const float e = 1e-4f * s, e2 = e * s, e3 = e2 * s;
    const float d2 = fmaf(m00, m11, -m01 * m01);
    const float c0 = fmaf(m11, m22, -m12 * m12), c1 = fmaf(m01, m22, -m12 * m02), c2 = fmaf(m01, m12, -m11 * m02);
    const float d3 = fmaf(m00, c0, fmaf(-m01, c1, m02 * c2));
    return !(m00 < -e || d2 < -e2 || d3 < -e3);
}

// 1 - exp(-x) for x >= 0 with a relative error of a few ulps: a series below 1/16, else the
// hardware exp2 (where the difference no longer cancels)
__device__ __forceinline__ float om_exp(float x)
{
    if (x < 0.0625f) {
        float t = fmaf(-x, 1.f / 7.f, 1.f);
        t = fmaf(-x * (1.f / 6.f), t, 1.f);
        t = fmaf(-x * (1.f / 5.f), t, 1.f);
        t = fmaf(-x * (1.f / 4.f), t, 1.f);
        t = fmaf(-x * (1.f / 3.f), t, 1.f);
        t = fmaf(-x * 0.5f, t, 1.f);
        return x * t;
    }
    return 1.f - __builtin_amdgcn_exp2f(-x * 1.4426950408889634f);
}

// Frangi's bright-tube vesselness of sigma^2 H (A, FP32) from its eigenvalues in ascending order.
// Sorted by (|lambda|, lambda) the eigenvalues are l1, l2, l3 with V != 0 only where l2 < 0 and
// l3 < 0: in value order mu0 <= mu1 <= mu2 that is exactly mu1 < 0 and mu1 + mu2 < 0, and then
// l3 = mu0, l2 = mu1, l1 = mu2.  The eigenvalues are re-solved in FP64 when their smallest gap is
// below tau max|mu|.  ia, ib, ic: 1 / (2 alpha^2), 1 / (2 beta^2), 1 / (2 c^2).
__device__ __forceinline__ float vesselness(const float A[6], float tau, float ia, float ib, float ic)
{
    float mu0, mu1, mu2;
    eig_sym3(A, mu0, mu1, mu2);
    const float gap = fminf(mu2 - mu1, mu1 - mu0);
    const float scl = fmaxf(fabsf(mu0), fabsf(mu2));
    if (gap < tau * scl) eig_jacobi64(A, mu0, mu1, mu2);
    if (!(mu1 < 0.f && mu1 + mu2 < 0.f)) return 0.f;
    const float Ra2 = (mu1 * mu1) * __builtin_amdgcn_rcpf(mu0 * mu0);
    const float Rb2 = (mu2 * mu2) * __builtin_amdgcn_rcpf(mu0 * mu1);
    const float S2 = fmaf(mu0, mu0, fmaf(mu1, mu1, mu2 * mu2));
    return om_exp(Ra2 * ia) * __builtin_amdgcn_exp2f(-Rb2 * ib * 1.4426950408889634f) * om_exp(S2 * ic);
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

// LDS floats of the workgroup's compaction list: the six entries of sigma^2 H of up to NT NV voxels
// (then each one's V in the first row), and the waves' counts
template <int NV>
struct Compact {
    static constexpr int kSlots = NT * NV;
    static constexpr int kFloats = 6 * kSlots + NT / 64;
};

// Epilogue of the NV voxels of one lane (every lane of the wave calls it, with the same NV): from the
// Hessian H of the smoothed volume (Hxx, Hyy, Hzz, Hxy, Hxz, Hyz) and, on the first scale, the
// intensities In = (I, I[x+1], I[x-1], I[y+1], I[y-1], I[z+1], I[z-1]) (clamped neighbours): the
// gradient (Eq. 2), k (Eq. 3), the eigenvalues of sigma^2 H and V.  Updates vmax with |g| (first
// scale) or |sigma^2 H|_F (Frangi-c pass).
// V can be non-zero only where maybe_vessel holds (a test on sigma^2 H that is exact up to a rounding
// margin), so only those voxels take the eigen-solve and Frangi: the workgroup writes them to one
// list in the LDS area cw (Compact<NV>::kFloats floats), solves the list densely, one voxel per
// lane, and reads the results back.  Elsewhere V = 0 exactly, as the full evaluation would give.
// Every thread of the workgroup must call it (it holds barriers).
template <int OUT_DT, int LAYOUT, int NV>
__device__ __forceinline__ void voxels_out(const XYArgs &a, float sigma2, const float (&H)[NV][6],
                                           const float (&In)[NV][7], const uint32_t (&v)[NV], const bool (&live)[NV],
                                           uint32_t N, float &vmax, float *cw, const float (*Vprev)[NV] = nullptr)
{
    if constexpr (LAYOUT == kHessianOut) {
        // the adjoint's recomputation: H itself, [6][N] FP32 in a.grad
        float *Ho = reinterpret_cast<float *>(a.grad);
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (live[i])
#pragma unroll
                for (int e = 0; e < 6; ++e) Ho[(size_t)e * N + v[i]] = H[i][e];
        return;
    }
    float A[NV][6];
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int e = 0; e < 6; ++e) A[i][e] = sigma2 * H[i][e];
    if (a.fro_pass) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const float f2 = A[i][0] * A[i][0] + A[i][1] * A[i][1] + A[i][2] * A[i][2] +
                             2.f * (A[i][3] * A[i][3] + A[i][4] * A[i][4] + A[i][5] * A[i][5]);
            if (live[i]) vmax = fmaxf(vmax, __builtin_amdgcn_sqrtf(f2));
        }
        return;
    }
    // V: the voxels that can have V != 0, compacted over the workgroup (a list per wave would leave
    // the lanes of a second round mostly idle)
    constexpr int NW = NT / 64;
    const int wv = threadIdx.x >> 6;
    bool need[NV];
    int slot[NV];
    int wcount = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        need[i] = live[i] && maybe_vessel(A[i]);
        const uint64_t m = __ballot(need[i]);
        slot[i] = wcount + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        wcount += __popcll(m);
    }
    int *cnt = reinterpret_cast<int *>(cw + 6 * Compact<NV>::kSlots);
    if ((threadIdx.x & 63) == 0) cnt[wv] = wcount;
    __syncthreads();
    int base = 0, count = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int c = cnt[w];
        base += (w < wv) ? c : 0;
        count += c;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        slot[i] += base;
        if (need[i])
#pragma unroll
            for (int e = 0; e < 6; ++e) cw[e * Compact<NV>::kSlots + slot[i]] = A[i][e];
    }
    // everything but V first (the gradient and k of the first scale), so that H and the intensities
    // are dead before the eigen-solves
    float kap_keep[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        kap_keep[i] = 0.f;
        if (!live[i] || !a.first) continue;
        float gx_, gy_, gz_, kap = 0.f;
        gx_ = (In[i][1] - In[i][2]) * a.inv2h[0];
        gy_ = (In[i][3] - In[i][4]) * a.inv2h[1];
        gz_ = (In[i][5] - In[i][6]) * a.inv2h[2];
        vmax = fmaxf(vmax, grad_norm(gx_, gy_, gz_));
        const float gm = fmaxf(fabsf(gx_), fmaxf(fabsf(gy_), fabsf(gz_)));
        if (gm > 0.f) {
            const float ig = __builtin_amdgcn_rcpf(gm);
            const float u0 = gx_ * ig, u1 = gy_ * ig, u2 = gz_ * ig;
            const float num = H[i][0] * u0 * u0 + H[i][1] * u1 * u1 + H[i][2] * u2 * u2 +
                              2.f * (H[i][3] * u0 * u1 + H[i][4] * u0 * u2 + H[i][5] * u1 * u2);
            kap = num * __builtin_amdgcn_rcpf(u0 * u0 + u1 * u1 + u2 * u2);  // the sum is >= 1
        }
        const uint32_t vi = v[i];
        if constexpr (LAYOUT == DVR_PLANAR) {
            st<OUT_DT>(a.grad, vi, gx_);
            st<OUT_DT>(a.grad, N + vi, gy_);
            st<OUT_DT>(a.grad, 2u * N + vi, gz_);
            st<OUT_DT>(a.kappa, vi, kap);
        } else if constexpr (LAYOUT == DVR_SPLIT) {
            if constexpr (OUT_DT == DVR_F32) {
                reinterpret_cast<float4 *>(a.grad)[vi] = make_float4(gx_, gy_, gz_, kap);
            } else {
                union { __half h[4]; uint2 u; } rec;
                rec.h[0] = __float2half_rn(gx_);
                rec.h[1] = __float2half_rn(gy_);
                rec.h[2] = __float2half_rn(gz_);
                rec.h[3] = __float2half_rn(kap);
                reinterpret_cast<uint2 *>(a.grad)[vi] = rec.u;
            }
        } else {
            // interleaved: (I, gx, gy, gz) now, (k, V, 0, 0) with V below
            if constexpr (OUT_DT == DVR_F32) {
                reinterpret_cast<float4 *>(a.grad)[2u * vi] = make_float4(In[i][0], gx_, gy_, gz_);
            } else {
                union { __half h[4]; uint2 u; } rec;
                rec.h[0] = __float2half_rn(In[i][0]);
                rec.h[1] = __float2half_rn(gx_);
                rec.h[2] = __float2half_rn(gy_);
                rec.h[3] = __float2half_rn(gz_);
                reinterpret_cast<uint2 *>(a.grad)[2u * vi] = rec.u;
            }
            kap_keep[i] = kap;
        }
    }
    __syncthreads();
    if (count > 0) {
        float c = a.c_host;
        if (!(c > 0.f)) {
            c = 0.5f * __hip_atomic_load(a.fro, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!(c > 0.f)) c = 1.f;
        }
        const float ic = 0.5f * __builtin_amdgcn_rcpf(c * c);
        for (int s = threadIdx.x; s < count; s += NT) {
            float Ai[6];
#pragma unroll
            for (int e = 0; e < 6; ++e) Ai[e] = cw[e * Compact<NV>::kSlots + s];
            cw[s] = vesselness(Ai, a.tau, a.inv2a2, a.inv2b2, ic);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (!live[i]) continue;
        float V = need[i] ? cw[slot[i]] : 0.f;
        const uint32_t vi = v[i];
        // V of the earlier scales: given by the caller (loaded ahead), or read here
        if constexpr (LAYOUT == DVR_PLANAR || LAYOUT == DVR_SPLIT) {
            if (!a.first) V = fmaxf(V, Vprev ? (*Vprev)[i] : ldo<OUT_DT>(a.ves, vi));
            st<OUT_DT>(a.ves, vi, V);
        } else {
            if (!a.first) {
                V = fmaxf(V, Vprev ? (*Vprev)[i] : ldo<OUT_DT>(a.grad, 8u * vi + 5u));
                st<OUT_DT>(a.grad, 8u * vi + 5u, V);
            } else if constexpr (OUT_DT == DVR_F32) {
                reinterpret_cast<float4 *>(a.grad)[2u * vi + 1u] = make_float4(kap_keep[i], V, 0.f, 0.f);
            } else {
                union { __half h[4]; uint2 u; } rec;
                rec.h[0] = __float2half_rn(kap_keep[i]);
                rec.h[1] = __float2half_rn(V);
                rec.h[2] = __float2half_rn(0.f);
                rec.h[3] = __float2half_rn(0.f);
                reinterpret_cast<uint2 *>(a.grad)[2u * vi + 1u] = rec.u;
            }
        }
    }
}

// y and x filters of one TX x TY tile of slice z from the staged z-filtered fields, then the
// per-voxel epilogue.  Returns this lane's contribution to |g|_max (first scale) or to
// max |sigma^2 H|_F (Frangi-c pass); the caller reduces it.  lds holds
// xy_lds_floats<TX, TY>(Rx, Ry) floats.  The taps may live in any address space (kernel
// arguments, or a device table read through the constant address space by the batched kernel).
template <int DT, int OUT_DT, int LAYOUT, int TX, int TY, typename ST>
__device__ __forceinline__ float xy_tile(const XYArgs &a, const ST &taps, int x0, int y0, int z, float *lds)
{
    const auto &tx = taps.ax[0];
    const auto &ty = taps.ax[1];
    const int Rx = tx.R, Ry = ty.R;
    const int W = TX + 2 * Rx, HH = TY + 2 * Ry;
    constexpr int kCW = Compact<TX * TY / NT>::kFloats;
    float *F = lds;                                          // [3][HH][W]; the waves' compaction lists after the y filters
    float *Fy = lds + (3 * HH * W > kCW ? 3 * HH * W : kCW);  // [6][TY][W]
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

    constexpr int NV = TX * TY / NT;
    static_assert((TX * TY) % NT == 0, "whole voxels per lane");
    float H[NV][6], In[NV][7];
    uint32_t v[NV];
    bool live[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int p = threadIdx.x + NT * i;
        const int yy = p / TX, xx = p - yy * TX;
        const int gx = x0 + xx, gy = y0 + yy;
        live[i] = gx < nx && gy < ny;
        const int cls = (gx == 0) ? 1 : (gx == nx - 1 ? 2 : 0);
        auto fy = [&](int k) { return [=](int m) { return Fy[k * TY * W + yy * W + xx + Rx + m]; }; };
        H[i][0] = filtD2(tx, cls, fy(0));   // Hxx = D2x Gy Gz
        H[i][3] = filtD1(tx, cls, fy(1));   // Hxy = D1x D1y Gz
        H[i][1] = filtG(tx, fy(2));         // Hyy = Gx D2y Gz
        H[i][4] = filtD1(tx, cls, fy(3));   // Hxz = D1x Gy D1z
        H[i][5] = filtG(tx, fy(4));         // Hyz = Gx D1y D1z
        H[i][2] = filtG(tx, fy(5));         // Hzz = Gx Gy D2z
        // lanes past the volume edge use an in-range voxel; their results are not stored
        const int cx = min(gx, nx - 1), cy = min(gy, ny - 1);
        v[i] = (uint32_t)z * plane + (uint32_t)cy * nx + cx;
#pragma unroll
        for (int k = 0; k < 7; ++k) In[i][k] = 0.f;
        if (a.first) {
            Buf b = make_buf(a.vol, N * ElemSize<DT>::v);
            const uint32_t row = (uint32_t)z * plane + (uint32_t)cy * nx;
            In[i][0] = ldv<DT>(b, v[i]);
            In[i][1] = ldv<DT>(b, row + clampi(cx + 1, 0, nx - 1));
            In[i][2] = ldv<DT>(b, row + clampi(cx - 1, 0, nx - 1));
            In[i][3] = ldv<DT>(b, (uint32_t)z * plane + (uint32_t)clampi(cy + 1, 0, ny - 1) * nx + cx);
            In[i][4] = ldv<DT>(b, (uint32_t)z * plane + (uint32_t)clampi(cy - 1, 0, ny - 1) * nx + cx);
            In[i][5] = ldv<DT>(b, (uint32_t)clampi(z + 1, 0, nz - 1) * plane + (uint32_t)cy * nx + cx);
            In[i][6] = ldv<DT>(b, (uint32_t)clampi(z - 1, 0, nz - 1) * plane + (uint32_t)cy * nx + cx);
        }
    }
    // the staged fields are dead after the y filters (the barrier above): the compaction list reuses them
    float vmax = 0.f;
    voxels_out<OUT_DT, LAYOUT, NV>(a, taps.sigma2, H, In, v, live, N, vmax, F);
    return vmax;
}

// ------------------------------------------------------------------------------------------------
// Fixed-radius filters: the same sums as filt3 / filtG / filtD1 / filtD2 with the stencil radius R a
// compile-time constant, so the loops unroll and the taps are read at constant offsets.  The
// smoothing tap G[R] is exactly zero (R = r + 1), so its term is left out.
template <int R, typename AT, typename F>
__device__ __forceinline__ float rG(const AT &t, F &&v)
{
    float g = t.G[0] * v(0);
#pragma unroll
    for (int m = 1; m < R; ++m) g = fmaf(t.G[m], v(m) + v(-m), g);
    return g;
}

template <int R, typename AT, typename F>
__device__ __forceinline__ float rD1(const AT &t, int cls, F &&v)
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

template <int R, typename AT, typename F>
__device__ __forceinline__ float rD2(const AT &t, int cls, F &&v)
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

template <int R, typename AT, typename F>
__device__ __forceinline__ Line3 r3(const AT &t, int cls, F &&v)
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
// a float in LDS, addressed with a 32-bit pointer (reads through it are LDS instructions)
typedef __attribute__((address_space(3))) float lds_f;

template <int R, int TX, int TY>
struct XYTileR {
    static constexpr int W = TX + 2 * R, HH = TY + 2 * R;
    static constexpr int NST = 3 * HH * W;  // staged values
    static constexpr int NFY = 6 * TY * W;  // y-filtered values
    static constexpr int NCW = Compact<TX * TY / NT>::kFloats;  // the workgroup's compaction list
    static constexpr int NF = NST > NCW ? NST : NCW;  // the staging area, reused by the lists
};

// One 64 x TY tile of the fixed-radius pass, for a run of z slices: the loads of a slice (its staged
// z-filtered fields with halo, the intensities of the gradient and, after the first scale, the V so
// far) are issued into registers while the previous slice is computed.
// The y-filtered fields may be written over the staged ones (F == Fy: max(NF, NFY) floats of LDS
// instead of NF + NFY): the y filters keep their results in registers until every lane has finished
// reading the staged rows, and a barrier separates the x filters from the epilogue's compaction
// lists, which reuse the staging area.  Less LDS per workgroup, more workgroups per CU.
template <int DT, int OUT_DT, int LAYOUT, int R, int TX, int TY, typename ST = ScaleTaps>
struct XYSlab {
    using T = XYTileR<R, TX, TY>;
    static constexpr int W = T::W, HH = T::HH;
    static constexpr int NW = NT / 64;    // waves
    static constexpr int NV = TY / NW;    // voxels per lane: rows wv, wv + NW, ... of the tile, x = lane
    static_assert(TX == 64 && TY % NW == 0 && W <= 128, "one tile column per lane, whole rows per wave");
    static constexpr int NROW = 3 * HH;   // staged rows (three fields)
    static constexpr int RPW = (NROW + NW - 1) / NW;

    const XYArgs &a;
    const ST &taps;
    float *F, *Fy;
    int x0, y0, nx, ny, nz;
    uint32_t plane, N;
    int lane, wv, gx, cx, c0, c1;
    bool two;
    // the slice in flight: staged rows, gradient intensities, V of the earlier scales
    float v0[RPW], v1[RPW];
    float In[NV][7];
    float Vp[NV];

    __device__ __forceinline__ XYSlab(const XYArgs &a_, const ST &t_, float *F_, float *Fy_, int x0_, int y0_)
        : a(a_), taps(t_), F(F_), Fy(Fy_), x0(x0_), y0(y0_)
    {
        nx = a.nx;
        ny = a.ny;
        nz = a.nz;
        plane = (uint32_t)nx * (uint32_t)ny;
        N = plane * (uint32_t)nz;
        lane = threadIdx.x & 63;
        // the wave index is uniform across the wave: row bases stay in scalar registers
        wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        gx = x0 + lane;              // this lane's output column
        cx = min(gx, nx - 1);        // lanes past the edge read an in-range voxel (not stored)
        c0 = clampi(x0 - R + lane, 0, nx - 1);
        c1 = clampi(x0 - R + 64 + lane, 0, nx - 1);
        two = 64 + lane < W;
    }

    // issue the loads of slice z
    __device__ __forceinline__ void load(int z)
    {
        load_rows(z);
        load_point(z);
    }

    // the staged rows of slice z (the z pass's three fields over the tile and halo)
    __device__ __forceinline__ void load_rows(int z)
    {
        // staged rows: wave wv takes rows wv, wv + NW, ...; a row is W consecutive (clamped) columns,
        // columns lane and 64 + lane, so each row adds only a scalar base to the column offsets
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
            const int r = wv + NW * k;
            v0[k] = v1[k] = 0.f;
            if (NROW % NW == 0 || r < NROW) {
                const int f = r / HH, yy = r - f * HH;
                const int gy = clampi(y0 - R + yy, 0, ny - 1);
                const float *row = a.ws + (size_t)f * N + (size_t)z * plane + (size_t)gy * nx;
                v0[k] = row[c0];
                if (two) v1[k] = row[c1];
            }
        }
    }

    // the intensities of the gradient (first scale) or the V of the earlier scales at this lane's
    // voxels of slice z
    __device__ __forceinline__ void load_point(int z)
    {
        if (a.first) {
            const Buf b = make_buf(a.vol, N * ElemSize<DT>::v);
            const int xp = min(cx + 1, nx - 1), xm = max(cx - 1, 0);
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int gy = min(y0 + wv + NW * i, ny - 1);
                const uint32_t row = (uint32_t)z * plane + (uint32_t)gy * nx;
                const uint32_t rp = (uint32_t)z * plane + (uint32_t)min(gy + 1, ny - 1) * nx;
                const uint32_t rm = (uint32_t)z * plane + (uint32_t)max(gy - 1, 0) * nx;
                const uint32_t zp = (uint32_t)min(z + 1, nz - 1) * plane + (uint32_t)gy * nx;
                const uint32_t zm = (uint32_t)max(z - 1, 0) * plane + (uint32_t)gy * nx;
                In[i][0] = ldv<DT>(b, row + cx);
                In[i][1] = ldv<DT>(b, row + xp);
                In[i][2] = ldv<DT>(b, row + xm);
                In[i][3] = ldv<DT>(b, rp + cx);
                In[i][4] = ldv<DT>(b, rm + cx);
                In[i][5] = ldv<DT>(b, zp + cx);
                In[i][6] = ldv<DT>(b, zm + cx);
                Vp[i] = 0.f;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
#pragma unroll
                for (int k = 0; k < 7; ++k) In[i][k] = 0.f;
                Vp[i] = 0.f;
                if constexpr (LAYOUT == DVR_PLANAR || LAYOUT == DVR_SPLIT || LAYOUT == DVR_INTERLEAVED) {
                    const int gy = min(y0 + wv + NW * i, ny - 1);
                    const uint32_t vi = (uint32_t)z * plane + (uint32_t)gy * nx + cx;
                    if constexpr (LAYOUT == DVR_INTERLEAVED) Vp[i] = ldo<OUT_DT>(a.grad, 8u * vi + 5u);
                    else Vp[i] = ldo<OUT_DT>(a.ves, vi);
                }
            }
        }
    }

    // write the staged rows of the slice in flight to LDS (all F readers of the previous slice done)
    __device__ __forceinline__ void store()
    {
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
            const int r = wv + NW * k;
            if (NROW % NW == 0 || r < NROW) {
                F[r * W + lane] = v0[k];
                if (two) F[r * W + 64 + lane] = v1[k];
            }
        }
    }

    // the filters and the epilogue of slice z from the staged rows in F, with that slice's intensities
    // and earlier V (In, Vp: copies taken before the next slice's loads were issued)
    __device__ __forceinline__ float compute(int z, const float (&Ic)[NV][7], const float (&Vc)[NV])
    {
        const auto &tx = taps.ax[0];
        const auto &ty = taps.ax[1];
        const int t = threadIdx.x;
        y_filters(ty, t);
        return x_filters_and_out(z, tx, Ic, Vc);
    }

    // y filters: all TY rows x W columns of the tile into registers (interior sums everywhere, then
    // the one-sided forms on the first and last row of the volume), then into Fy once every lane has
    // read the staged rows
    template <typename AT>
    __device__ __forceinline__ void y_filters(const AT &ty, int t)
    {
        constexpr int kIt = (TY * W + NT - 1) / NT;
        float ry[kIt][6];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int p = t + it * NT;
            if (p < TY * W) {
                const int yy = p / W, xx = p - yy * W;
                const lds_f *b = (const lds_f *)(F) + (yy * W + xx);
                asm volatile("" : "+v"(b));
                auto f0 = [&](int m) { return b[(0 * HH + R + m) * W]; };
                auto f1 = [&](int m) { return b[(1 * HH + R + m) * W]; };
                auto f2 = [&](int m) { return b[(2 * HH + R + m) * W]; };
                const Line3 r0 = r3<R>(ty, 0, f0);
                ry[it][0] = r0.g;
                ry[it][1] = r0.d1;
                ry[it][2] = r0.d2;
                ry[it][3] = rG<R>(ty, f1);
                ry[it][4] = rD1<R>(ty, 0, f1);
                ry[it][5] = rG<R>(ty, f2);
            }
        }
        if (y0 == 0 || y0 + TY >= ny) {
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
                const int p = t + it * NT;
                if (p < TY * W) {
                    const int yy = p / W, xx = p - yy * W;
                    const int gy = y0 + yy;
                    auto f0 = [&](int m) { return F[(0 * HH + yy + R + m) * W + xx]; };
                    auto f1 = [&](int m) { return F[(1 * HH + yy + R + m) * W + xx]; };
                    if (gy == 0) {
                        ry[it][1] = rD1<R>(ty, 1, f0);
                        ry[it][2] = rD2<R>(ty, 1, f0);
                        ry[it][4] = rD1<R>(ty, 1, f1);
                    }
                    if (gy == ny - 1) {
                        ry[it][1] = rD1<R>(ty, 2, f0);
                        ry[it][2] = rD2<R>(ty, 2, f0);
                        ry[it][4] = rD1<R>(ty, 2, f1);
                    }
                }
            }
        }
        __syncthreads();  // every lane's reads of the staged rows are done
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int p = t + it * NT;
            if (p < TY * W) {
#pragma unroll
                for (int k = 0; k < 6; ++k) Fy[k * TY * W + p] = ry[it][k];
            }
        }
        __syncthreads();
    }

    template <typename AT>
    __device__ __forceinline__ float x_filters_and_out(int z, const AT &tx, const float (&Ic)[NV][7],
                                                       const float (&Vc)[NV])
    {
        // x filters of this lane's voxels (rows wv + NW i, column lane), the same way
        float H[NV][6];
        uint32_t v[NV];
        bool live[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int yy = wv + NW * i;
            const int gy = y0 + yy;
            live[i] = gx < nx && gy < ny;
            // one opaque base per field at the start of the lane's window: every tap's offset then fits
            // the paired LDS reads' immediates
            const lds_f *b[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                b[k] = (const lds_f *)(Fy) + (k * TY * W + yy * W + lane);
                asm volatile("" : "+v"(b[k]));
            }
            auto fy = [&](int k) { return [=](int m) { return b[k][R + m]; }; };
            H[i][0] = rD2<R>(tx, 0, fy(0));  // Hxx = D2x Gy Gz
            H[i][3] = rD1<R>(tx, 0, fy(1));  // Hxy = D1x D1y Gz
            H[i][1] = rG<R>(tx, fy(2));      // Hyy = Gx D2y Gz
            H[i][4] = rD1<R>(tx, 0, fy(3));  // Hxz = D1x Gy D1z
            H[i][5] = rG<R>(tx, fy(4));      // Hyz = Gx D1y D1z
            H[i][2] = rG<R>(tx, fy(5));      // Hzz = Gx Gy D2z
            v[i] = (uint32_t)z * plane + (uint32_t)min(gy, ny - 1) * nx + cx;
        }
        // the first and last column of the volume take the one-sided differences (tiles that hold one)
        if (x0 == 0 || x0 + TX >= nx) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int yy = wv + NW * i;
                auto fy = [&](int k) { return [=](int m) { return Fy[k * TY * W + yy * W + lane + R + m]; }; };
                if (gx == 0) {
                    H[i][0] = rD2<R>(tx, 1, fy(0));
                    H[i][3] = rD1<R>(tx, 1, fy(1));
                    H[i][4] = rD1<R>(tx, 1, fy(3));
                }
                if (gx == nx - 1) {
                    H[i][0] = rD2<R>(tx, 2, fy(0));
                    H[i][3] = rD1<R>(tx, 2, fy(1));
                    H[i][4] = rD1<R>(tx, 2, fy(3));
                }
            }
        }
        // the staged fields are dead after the y filters: the compaction lists reuse them (when the
        // y-filtered fields were written over them, every lane must have read those first)
        __syncthreads();
        float vmax = 0.f;
        voxels_out<OUT_DT, LAYOUT, NV>(a, taps.sigma2, H, Ic, v, live, N, vmax, F, &Vc);
        return vmax;
    }
};

// The fixed-radius tile over slices [z0, z1), each slice's loads issued while the previous slice is
// computed.  F, Fy: XYTileR<R, TX, TY>::NF and ::NFY floats of LDS.  Returns this lane's contribution
// to |g|_max (first scale) or max |sigma^2 H|_F (Frangi-c pass).  Every thread of the workgroup must
// call it; it starts with a barrier, so the LDS may still be in use by an earlier tile.
template <int DT, int OUT_DT, int LAYOUT, int R, int TX, int TY, typename ST>
__device__ __forceinline__ float xy_run_r(const XYArgs &a, const ST &taps, int x0, int y0, int z0, int z1, float *F,
                                          float *Fy)
{
    using S = XYSlab<DT, OUT_DT, LAYOUT, R, TX, TY, ST>;
    S s(a, taps, F, Fy, x0, y0);
    float vmax = 0.f;
    s.load(z0);
    for (int z = z0; z < z1; ++z) {
        __syncthreads();  // the previous slice's readers of F (its y filters, its compaction lists) are done
        s.store();
        float Ic[S::NV][7], Vc[S::NV];
#pragma unroll
        for (int i = 0; i < S::NV; ++i) {
            Vc[i] = s.Vp[i];
#pragma unroll
            for (int k = 0; k < 7; ++k) Ic[i][k] = s.In[i][k];
        }
        if (z + 1 < z1) s.load(z + 1);
        __syncthreads();
        vmax = fmaxf(vmax, s.compute(z, Ic, Vc));
    }
    return vmax;
}

// LDS floats of the generic tile: the staged fields (whose space the four waves' compaction lists
// reuse after the y filters) and the y-filtered fields
template <int TX, int TY>
__host__ __device__ constexpr size_t xy_lds_floats(int Rx, int Ry)
{
    const size_t st = (size_t)3 * (TY + 2 * Ry) * (TX + 2 * Rx), cw = (size_t)Compact<TX * TY / NT>::kFloats;
    return (st > cw ? st : cw) + (size_t)6 * TY * (TX + 2 * Rx);
}

}  // namespace dvr
