// Device code of the raymarcher shared by the per-call kernels (render.hip) and the batched
// persistent kernel (batch.hip).  See render.hip for the design notes.
#pragma once

#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "render_args.hpp"

namespace dvr {

struct RayGeo {
    int N;               // number of segments (0 = miss)
    int64_t q0[3];       // fixed-point position of sample 0
    int64_t dq[3];       // step between full-segment samples
    int64_t dql[3];      // step from sample N-2 to the last sample
    int64_t ql[3];       // position of the last sample
    float delta, dlast;  // segment lengths (mm)
};

// ------------------------------------------------------------------------------------------------
// Double-float arithmetic for the per-ray geometry: a value is the unevaluated sum hi + lo of two
// FP32 numbers with |lo| <= ulp(hi) / 2 (about 48 significant bits), built on the error-free
// transforms TwoSum (Knuth) and TwoProd (one fused multiply-add), as in Dekker's 1971 double-length
// arithmetic.  A quotient takes three terms from the hardware reciprocal (about 1 ulp), each
// correcting the exact residual of the previous ones, and a square root one Newton step; neither
// needs a correctly rounded FP32 division.  Operation order matters: no contraction is applied to
// these (every fused multiply-add is explicit).
struct F2 {
    float hi, lo;
};

__device__ __forceinline__ F2 f2(float a) { return {a, 0.f}; }

__device__ __forceinline__ F2 two_sum(float a, float b)
{
    const float s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

// exact when |a| >= |b| (or a = 0)
__device__ __forceinline__ F2 fast_two_sum(float a, float b)
{
    const float s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ F2 two_prod(float a, float b)
{
    const float p = a * b;
    return {p, fmaf(a, b, -p)};
}

// Dekker's addition: the error is below ~2^-47 of max(|a|, |b|) (not relative to a cancelled sum,
// which is all the geometry needs: its inputs carry that absolute precision already)
__device__ __forceinline__ F2 f2_add(F2 a, F2 b)
{
    const F2 s = two_sum(a.hi, b.hi);
    return fast_two_sum(s.hi, s.lo + (a.lo + b.lo));
}

__device__ __forceinline__ F2 f2_neg(F2 a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ F2 f2_sub(F2 a, F2 b) { return f2_add(a, f2_neg(b)); }

__device__ __forceinline__ F2 f2_mul(F2 a, F2 b)
{
    const F2 p = two_prod(a.hi, b.hi);
    return fast_two_sum(p.hi, fmaf(a.hi, b.lo, fmaf(a.lo, b.hi, p.lo)));
}

__device__ __forceinline__ F2 f2_mulf(F2 a, float b)
{
    const F2 p = two_prod(a.hi, b);
    return fast_two_sum(p.hi, fmaf(a.lo, b, p.lo));
}

__device__ __forceinline__ F2 f2_half(F2 a) { return {0.5f * a.hi, 0.5f * a.lo}; }

// 1 / b (b finite and non-zero)
__device__ __forceinline__ F2 f2_recip(F2 b)
{
    const float rb = __builtin_amdgcn_rcpf(b.hi);
    const float q1 = rb;
    const F2 r1 = f2_sub(f2(1.f), f2_mulf(b, q1));
    const float q2 = r1.hi * rb;
    const F2 r2 = f2_sub(r1, f2_mulf(b, q2));
    return fast_two_sum(q1, q2 + r2.hi * rb);
}

// a > 0
__device__ __forceinline__ F2 f2_sqrt(F2 a)
{
    const float s = __builtin_amdgcn_sqrtf(a.hi);
    const F2 e = f2_sub(a, two_prod(s, s));
    return fast_two_sum(s, e.hi * (0.5f * __builtin_amdgcn_rcpf(s)));
}

__device__ __forceinline__ bool f2_lt(F2 a, F2 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

// nearest integer of a finite value of magnitude below 2^62: the integer-valued high part is split
// toward zero into a multiple of 2^32 and a remainder of the same sign below 2^32 in magnitude (both
// exact FP32 integers), each converted with a 32-bit conversion
__device__ __forceinline__ int64_t f2_rint(F2 a)
{
    const float h = rintf(a.hi);
    const float r = rintf((a.hi - h) + a.lo);
    const float hh = truncf(h * 0x1p-32f);
    const float hl = h - hh * 0x1p32f;
    const int64_t lo = hl >= 0.f ? (int64_t)(uint32_t)hl : -(int64_t)(uint32_t)(-hl);
    return (int64_t)((uint64_t)(int64_t)(int32_t)hh << 32) + lo + (int64_t)(int32_t)r;
}

// a * 2^32 to the nearest fixed-point position, clamped to [0, (n - 1) 2^32 - 1]
__device__ __forceinline__ int64_t to_fix(F2 q, int n)
{
    const int64_t hi = (int64_t)(n - 1) * 4294967296LL - 1;
    const F2 v = {q.hi * 4294967296.f, q.lo * 4294967296.f};
    if (!(v.hi > -1.f)) return 0;  // also NaN
    if (!(v.hi < 4.0e18f)) return hi;
    const int64_t r = f2_rint(v);
    return r < 0 ? 0 : (r > hi ? hi : r);
}

// Ray of pixel (pi, pj): the definition's FP64 geometry (pixel-centre ray, slab clip against
// [0, (n - 1) h], N = ceil(L / delta) segments, midpoints) evaluated in double-float FP32, which
// carries ~47 bits through these steps: N and the 32.32 fixed-point positions come out as the FP64
// definition's except where a quantity lies within ~1e-13 relative of a rounding or ceiling boundary
// (positions within one unit of 2^-32 voxel on a million-ray CPU comparison, N identical).
__device__ __forceinline__ RayGeo ray_setup(const KCam cam, int pi, int pj, const KGrid &g)
{
#pragma clang fp contract(off)
    RayGeo r;
    r.N = 0;
    const float fi = (float)pi + 0.5f, fj = (float)pj + 0.5f;  // exact below 2^23
    F2 o[3], d[3];
    if (cam.persp) {
        F2 n2 = f2(0.f);
        for (int a = 0; a < 3; ++a) {
            o[a] = f2(cam.o[a]);
            d[a] = f2_add(f2_add(f2(cam.d0[a]), two_prod(fi, cam.du[a])), two_prod(fj, cam.dv[a]));
            n2 = f2_add(n2, f2_mul(d[a], d[a]));
        }
        if (!(n2.hi > 0.f)) return r;
        const F2 inn = f2_recip(f2_sqrt(n2));
        for (int a = 0; a < 3; ++a) d[a] = f2_mul(d[a], inn);
    } else {
        for (int a = 0; a < 3; ++a) {
            o[a] = f2_add(f2_add(f2(cam.o[a]), two_prod(fi, cam.du[a])), two_prod(fj, cam.dv[a]));
            d[a] = f2(cam.d0[a]);
        }
    }
    bool any = false;
    F2 t0 = f2(0.f), t1 = f2(0.f);
    for (int a = 0; a < 3; ++a) {
        const F2 hi = two_prod((float)(g.n[a] - 1), g.h[a]);
        if (fabsf(d[a].hi) < 1e-30f) {
            // parallel to the faces of this axis (a component below 1e-30 puts both slab parameters
            // beyond 1e30 unless the origin lies on a face): outside, or on a face moving out, misses
            if (f2_lt(o[a], f2(0.f)) || f2_lt(hi, o[a])) return r;
            const bool on0 = o[a].hi == 0.f && o[a].lo == 0.f, onh = o[a].hi == hi.hi && o[a].lo == hi.lo;
            if ((on0 && d[a].hi < 0.f) || (onh && d[a].hi > 0.f)) return r;
            continue;
        }
        // the face at 0 is the entry for a positive component, the face at (n - 1) h otherwise
        const F2 id = f2_recip(d[a]);
        const F2 lo_t = f2_mul(f2_neg(o[a]), id), hi_t = f2_mul(f2_sub(hi, o[a]), id);
        const bool pos = d[a].hi > 0.f;
        const F2 ta = pos ? lo_t : hi_t, tb = pos ? hi_t : lo_t;
        if (!any || f2_lt(t0, ta)) t0 = ta;
        if (!any || f2_lt(tb, t1)) t1 = tb;
        any = true;
    }
    if (!any) return r;  // a zero direction
    const F2 tn = f2_lt(f2(0.f), t0) ? t0 : f2(0.f), tf = t1;
    if (!f2_lt(tn, tf)) return r;  // also NaN
    if (!(tf.hi < 3.0e38f)) return r;  // an unbounded chord (a direction component of ~1e-38)
    const F2 delta = {g.delta_hi, g.delta_lo};
    const F2 L = f2_sub(tf, tn);
    const F2 Lq = f2_mul(L, F2{g.idelta_hi, g.idelta_lo});
    if (!(Lq.hi <= 2.0e9f)) return r;
    // ceil(Lq): the high part's ceiling unless the high part is an integer, then that plus the low part's
    const float ch = ceilf(Lq.hi);
    const int64_t Nl = (ch != Lq.hi) ? (int64_t)ch : (int64_t)Lq.hi + (int64_t)ceilf(Lq.lo);
    if (Nl < 1 || Nl > 2000000000LL) return r;
    int N = (int)Nl;
    F2 nd, dlast;
    for (int pass = 0; pass < 2; ++pass) {
        const float nh = (float)(N - 1);
        const F2 nm1 = {nh, (float)((int64_t)(N - 1) - (int64_t)nh)};  // N - 1 exactly
        nd = f2_mul(nm1, delta);
        dlast = f2_sub(L, nd);
        // L / delta within 2^-40 above an integer (the product L (1 / delta) rounded up past an exact
        // integer, as on axis-aligned rays, or a last segment below 2^-40 L) is that integer, as the
        // FP64 quotient of an exact integer ratio is
        if (pass == 0 && N > 1 && dlast.hi <= 0x1p-40f * L.hi) --N;
        else break;
    }
    const F2 tfirst = f2_add(tn, f2_half(N == 1 ? dlast : delta));
    const F2 tlast = f2_add(f2_add(tn, nd), f2_half(dlast));
    for (int a = 0; a < 3; ++a) {
        const F2 ih = {g.ih_hi[a], g.ih_lo[a]};
        r.q0[a] = to_fix(f2_mul(f2_add(o[a], f2_mul(tfirst, d[a])), ih), g.n[a]);
        r.ql[a] = to_fix(f2_mul(f2_add(o[a], f2_mul(tlast, d[a])), ih), g.n[a]);
        const F2 sv = f2_mul(f2_mul(delta, d[a]), ih);
        int64_t st = f2_rint(F2{sv.hi * 4294967296.f, sv.lo * 4294967296.f});
        if (N >= 3) {
            // the full-segment samples lie between q0 and q0 + (N-2) st; keep that end inside
            const int64_t maxq = (int64_t)(g.n[a] - 1) * (int64_t)4294967296LL - 1;
            const int64_t end = r.q0[a] + (int64_t)(N - 2) * st;
            if (end < 0) st = (0 - r.q0[a]) / (int64_t)(N - 2);
            else if (end > maxq) st = (maxq - r.q0[a]) / (int64_t)(N - 2);
        }
        r.dq[a] = st;
        const int64_t qn2 = r.q0[a] + (int64_t)(N >= 2 ? N - 2 : 0) * st;
        r.dql[a] = r.ql[a] - qn2;
    }
    if (N == 1)
        for (int a = 0; a < 3; ++a) r.q0[a] = r.ql[a];
    r.N = N;
    r.delta = delta.hi;
    r.dlast = dlast.hi;
    return r;
}

// ------------------------------------------------------------------------------------------------
// TF in LDS: knot x, value (R, G, B, tau), slope to the next knot (0 after the last), 1/width.
// nzp: prefix counts over the extended segments e = -1 (below the first knot) .. K-1 (at or above
// the last) of "the extinction is not identically zero on e": nzp[0] = 0, nzp[j + 1] = nzp[j] + nz(j - 1).
template <int KMAX>
struct TFShared {
    float4 v[KMAX];
    float4 s[KMAX];
    float x[KMAX];
    float iw[KMAX];
    int nzp[KMAX + 2];
    int K;
};

template <int KMAX>
__device__ __forceinline__ void tf_load(TFShared<KMAX> &sh, float (&kx)[KMAX], const KTF &tf)
{
    const int K = tf.K;
    for (int i = threadIdx.x; i < KMAX; i += blockDim.x) {
        if (i < K) {
            const float4 vi = reinterpret_cast<const float4 *>(tf.rgba)[i];
            const float xi = tf.knots[i];
            sh.v[i] = vi;
            sh.x[i] = xi;
            if (i + 1 < K) {
                const float4 vn = reinterpret_cast<const float4 *>(tf.rgba)[i + 1];
                const float w = tf.knots[i + 1] - xi;
                sh.iw[i] = 1.f / w;
                sh.s[i] = make_float4((vn.x - vi.x) / w, (vn.y - vi.y) / w, (vn.z - vi.z) / w, (vn.w - vi.w) / w);
            } else {
                sh.iw[i] = 0.f;
                sh.s[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    }
    if (threadIdx.x == 0) {
        sh.K = K;
        const float4 *r = reinterpret_cast<const float4 *>(tf.rgba);
        int c = 0;
        sh.nzp[0] = 0;
        for (int e = -1; e < K; ++e) {
            const bool nz = (e < 0) ? (r[0].w != 0.f) : (e == K - 1 ? r[K - 1].w != 0.f : (r[e].w != 0.f || r[e + 1].w != 0.f));
            c += nz ? 1 : 0;
            sh.nzp[e + 2] = c;
        }
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) kx[i] = (i < K) ? tf.knots[i] : INFINITY;
}

// extended TF segment of x: -1 below the first knot, else the index of the last knot <= x
template <int KMAX>
__device__ __forceinline__ int tf_seg(const float (&kx)[KMAX], float x)
{
    int c = 0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) c += (x >= kx[i]) ? 1 : 0;
    return c - 1;
}

// True when every intensity the trilinear interpolation can produce from corner values in
// [lo, hi] falls on TF segments whose extinction is identically zero.  The interval is widened by
// 2^-18 max(|lo|, |hi|): the FP32 weights and the fma chain of the interpolation stay within
// ~2^-19 of the range of the corner values.
template <int KMAX>
__device__ __forceinline__ bool brick_empty(const TFShared<KMAX> &sh, const float (&kx)[KMAX], float lo, float hi)
{
    const float d = fmaxf(fabsf(lo), fabsf(hi)) * 3.814697265625e-6f + 1e-30f;
    const int a = tf_seg<KMAX>(kx, lo - d), b = tf_seg<KMAX>(kx, hi + d);
    return sh.nzp[b + 2] - sh.nzp[a + 1] == 0;
}

// ------------------------------------------------------------------------------------------------
// Feature fetch.  LAYOUT/DT select planar planes, interleaved records, the split layout (I and V
// planes plus a (gx, gy, gz, k) record, addressed at 4x the plane offsets), or the quad layout (the
// split records, and I and V as per-voxel (y, z) quads, also addressed at 4x the plane offsets).
template <int LAYOUT, int DT>
struct Vox {
    Buf b[6];  // planar: I, gx, gy, gz, kappa, V;  interleaved: b[0] = records;  split, quad: I, records, V
    uint32_t sx, sy, sz;  // byte strides of +1 in x, y, z (split: in the planes)

    __device__ __forceinline__ void init(const KFeat &f, const KGrid &g)
    {
        const uint32_t N = (uint32_t)g.n[0] * (uint32_t)g.n[1] * (uint32_t)g.n[2];
        uint32_t es;
        if constexpr (LAYOUT == DVR_PLANAR) {
            es = ElemSize<DT>::v;
            b[0] = make_buf(f.vol, N * es);
            const char *gp = reinterpret_cast<const char *>(f.grad);
            b[1] = make_buf(gp, N * es);
            b[2] = make_buf(gp + (size_t)N * es, N * es);
            b[3] = make_buf(gp + (size_t)2 * N * es, N * es);
            b[4] = make_buf(f.kappa, N * es);
            b[5] = make_buf(f.ves, N * es);
        } else if constexpr (LAYOUT == DVR_SPLIT || LAYOUT == DVR_QUAD) {
            es = ElemSize<DT>::v;
            const uint32_t q = (LAYOUT == DVR_QUAD) ? 4u : 1u;
            b[0] = make_buf(f.vol, N * q * es);
            b[1] = make_buf(f.grad, N * 4u * es);
            b[2] = make_buf(f.ves, N * q * es);
        } else {
            es = (DT == DVR_F32) ? 32u : 16u;
            b[0] = make_buf(f.grad, N * es);
        }
        sx = es;
        sy = es * (uint32_t)g.n[0];
        sz = sy * (uint32_t)g.n[1];
    }
};

struct Corners {
    float w[8];
    uint32_t off[4];  // byte offsets of the (y, z) = (0,0), (1,0), (0,1), (1,1) rows; +sx for x+1
};

__device__ __forceinline__ void corner_setup(const int64_t q[3], uint32_t sx, uint32_t sy, uint32_t sz, Corners &c)
{
    const float k = 2.3283064365386963e-10f;  // 2^-32
    const uint32_t cx = (uint32_t)(q[0] >> 32), cy = (uint32_t)(q[1] >> 32), cz = (uint32_t)(q[2] >> 32);
    const float fx = (float)(uint32_t)q[0] * k, fy = (float)(uint32_t)q[1] * k, fz = (float)(uint32_t)q[2] * k;
    const float gx = 1.f - fx, gy = 1.f - fy, gz = 1.f - fz;
    const float a00 = gy * gz, a10 = fy * gz, a01 = gy * fz, a11 = fy * fz;
    c.w[0] = gx * a00; c.w[1] = fx * a00;
    c.w[2] = gx * a10; c.w[3] = fx * a10;
    c.w[4] = gx * a01; c.w[5] = fx * a01;
    c.w[6] = gx * a11; c.w[7] = fx * a11;
    const uint32_t base = cx * sx + cy * sy + cz * sz;
    c.off[0] = base;
    c.off[1] = base + sy;
    c.off[2] = base + sz;
    c.off[3] = base + sy + sz;
}

// Interpolated channels of one sample.
struct Chan {
    float I, g[3], k, V;
};

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Corner values of the current cell, kept across samples: consecutive samples (half a voxel
// apart) often stay in the same cell, and then no gather is issued for that lane.  Planar
// layouts load the intensity corners first and the feature corners only for a sample whose
// extinction is non-zero; an interleaved record brings all six channels in one load per corner
// (F32: 16 + 8 bytes, F16: 12 bytes kept packed and widened at use).  F16 quad-layout corners are
// kept packed the same way, (I, gx), (gy, gz), (k, V) per corner, and widened at use.
template <int LAYOUT, int DT>
struct CornerCache {
    static constexpr bool kPacked = (LAYOUT == DVR_INTERLEAVED || LAYOUT == DVR_QUAD) && DT == DVR_F16;
    uint32_t base;  // byte offset of the cached cell's first corner, or ~0
    bool feat;      // feature corners valid for this cell
    float v[kPacked ? 1 : 8][6];
    uint32_t raw[kPacked ? 8 : 1][3];

    __device__ __forceinline__ void reset()
    {
        base = 0xffffffffu;
        feat = false;
    }

    // quad layout: the quads of voxels x and x + 1 (byte offset off and the next quad) are the
    // corners (y, z), (y+1, z), (y, z+1), (y+1, z+1) of the cell's two x-columns, channel CH; the two
    // 8-byte F16 quads are adjacent, so they come in one 16-byte load
    template <int CH>
    __device__ __forceinline__ void quad_pair(const Buf &b, uint32_t off)
    {
        if constexpr (DT == DVR_F32) {
            const f32x4 a = __builtin_bit_cast(f32x4, ld4(b, off));
            const f32x4 d = __builtin_bit_cast(f32x4, ld4(b, off + 16u));
            v[0][CH] = a.x; v[2][CH] = a.y; v[4][CH] = a.z; v[6][CH] = a.w;
            v[1][CH] = d.x; v[3][CH] = d.y; v[5][CH] = d.z; v[7][CH] = d.w;
        } else {
            const f16x8 a = __builtin_bit_cast(f16x8, ld4(b, off));
            v[0][CH] = (float)a[0]; v[2][CH] = (float)a[1]; v[4][CH] = (float)a[2]; v[6][CH] = (float)a[3];
            v[1][CH] = (float)a[4]; v[3][CH] = (float)a[5]; v[5][CH] = (float)a[6]; v[7][CH] = (float)a[7];
        }
    }

    __device__ __forceinline__ void need_I(const Vox<LAYOUT, DT> &vx, const Corners &c)
    {
        if (c.off[0] == base) return;
        base = c.off[0];
        if constexpr (LAYOUT == DVR_QUAD && DT == DVR_F16) {
            // the 8 intensity halves into the low halves of the packed words (I, gx)
            const u32x4 a = ld4(vx.b[0], c.off[0] << 2);
            raw[0][0] = a.x; raw[2][0] = a.x >> 16; raw[4][0] = a.y; raw[6][0] = a.y >> 16;
            raw[1][0] = a.z; raw[3][0] = a.z >> 16; raw[5][0] = a.w; raw[7][0] = a.w >> 16;
            feat = false;
            return;
        }
        if constexpr (LAYOUT == DVR_QUAD) {
            quad_pair<0>(vx.b[0], c.off[0] << 2);
            feat = false;
            return;
        }
        if constexpr (LAYOUT != DVR_INTERLEAVED && DT == DVR_F32) {
            // corners x and x + 1 are adjacent floats: one 8-byte load per (y, z) row of the cell
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const f32x2 p = ld2f(vx.b[0], c.off[j]);
                v[2 * j][0] = p.x;
                v[2 * j + 1][0] = p.y;
            }
            feat = false;
            return;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t off = c.off[e >> 1] + ((e & 1) ? vx.sx : 0u);
            if constexpr (LAYOUT != DVR_INTERLEAVED) {
                if constexpr (DT == DVR_F32) v[e][0] = ldf(vx.b[0], off);
                else v[e][0] = ldh(vx.b[0], off);
            } else if constexpr (DT == DVR_F32) {
                // whole-vector casts only: a bit_cast of a single ext-vector element is folded to
                // element 0 by this compiler at -O3
                const f32x4 a = __builtin_bit_cast(f32x4, ld4(vx.b[0], off));
                const f32x4 b = __builtin_bit_cast(f32x4, ld4(vx.b[0], off + 16u));
                v[e][0] = a.x;
                v[e][1] = a.y;
                v[e][2] = a.z;
                v[e][3] = a.w;
                v[e][4] = b.x;
                v[e][5] = b.y;
            } else {
                const u32x4 a = ld4(vx.b[0], off);
                raw[e][0] = a.x;
                raw[e][1] = a.y;
                raw[e][2] = a.z;
            }
        }
        feat = (LAYOUT == DVR_INTERLEAVED);
    }

    __device__ __forceinline__ void need_feat(const Vox<LAYOUT, DT> &vx, const Corners &c)
    {
        if constexpr (LAYOUT == DVR_PLANAR && DT == DVR_F32) {
            if (feat) return;
            feat = true;
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int ch = 1; ch < 6; ++ch) {
                    const f32x2 p = ld2f(vx.b[ch], c.off[j]);
                    v[2 * j][ch] = p.x;
                    v[2 * j + 1][ch] = p.y;
                }
        } else if constexpr (LAYOUT == DVR_PLANAR) {
            if (feat) return;
            feat = true;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t off = c.off[e >> 1] + ((e & 1) ? vx.sx : 0u);
#pragma unroll
                for (int ch = 1; ch < 6; ++ch) {
                    if constexpr (DT == DVR_F32) v[e][ch] = ldf(vx.b[ch], off);
                    else v[e][ch] = ldh(vx.b[ch], off);
                }
            }
        } else if constexpr (LAYOUT == DVR_QUAD && DT == DVR_F16) {
            if (feat) return;
            feat = true;
            const u32x4 vq = ld4(vx.b[2], c.off[0] << 2);
            const uint32_t V[8] = {vq.x & 0xffffu, vq.z & 0xffffu, vq.x >> 16, vq.z >> 16,
                                   vq.y & 0xffffu, vq.w & 0xffffu, vq.y >> 16, vq.w >> 16};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const u32x4 r = ld4(vx.b[1], c.off[j] << 2);  // records of corners 2j (x) and 2j + 1 (x + 1)
                const int e0 = 2 * j, e1 = 2 * j + 1;
                raw[e0][0] = (raw[e0][0] & 0xffffu) | (r.x << 16);
                raw[e0][1] = (r.x >> 16) | (r.y << 16);
                raw[e0][2] = (r.y >> 16) | (V[e0] << 16);
                raw[e1][0] = (raw[e1][0] & 0xffffu) | (r.z << 16);
                raw[e1][1] = (r.z >> 16) | (r.w << 16);
                raw[e1][2] = (r.w >> 16) | (V[e1] << 16);
            }
        } else if constexpr (LAYOUT == DVR_SPLIT || LAYOUT == DVR_QUAD) {
            if (feat) return;
            feat = true;
            if constexpr (LAYOUT == DVR_QUAD) quad_pair<5>(vx.b[2], c.off[0] << 2);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t off = c.off[e >> 1] + ((e & 1) ? vx.sx : 0u);
                if constexpr (DT == DVR_F32) {
                    const f32x4 r = __builtin_bit_cast(f32x4, ld4(vx.b[1], off << 2));
                    v[e][1] = r.x;
                    v[e][2] = r.y;
                    v[e][3] = r.z;
                    v[e][4] = r.w;
                    if (LAYOUT == DVR_SPLIT && (e & 1) == 0) {  // V of corners x and x + 1 in one 8-byte load
                        const f32x2 p = ld2f(vx.b[2], off);
                        v[e][5] = p.x;
                        v[e + 1][5] = p.y;
                    }
                } else {
                    // the 8-byte records of corners x and x + 1 are adjacent: one 16-byte load
                    if ((e & 1) == 0) {
                        const f16x8 r = __builtin_bit_cast(f16x8, ld4(vx.b[1], off << 2));
                        v[e][1] = (float)r[0];
                        v[e][2] = (float)r[1];
                        v[e][3] = (float)r[2];
                        v[e][4] = (float)r[3];
                        v[e + 1][1] = (float)r[4];
                        v[e + 1][2] = (float)r[5];
                        v[e + 1][3] = (float)r[6];
                        v[e + 1][4] = (float)r[7];
                    }
                    if constexpr (LAYOUT == DVR_SPLIT) v[e][5] = ldh(vx.b[2], off);
                }
            }
        }
        (void)vx;
        (void)c;
    }

    __device__ __forceinline__ float val(int e, int ch) const
    {
        if constexpr (kPacked) {
            const f16x2 h = __builtin_bit_cast(f16x2, raw[e][ch >> 1]);
            return (float)((ch & 1) ? h.y : h.x);
        } else {
            return v[e][ch];
        }
    }

    __device__ __forceinline__ float interp(const Corners &c, int ch) const
    {
        float acc = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) acc = fmaf(c.w[e], val(e, ch), acc);
        return acc;
    }
};

// Optical state of one sample.
struct Opt {
    float tau, c[3];  // TF value at I
    float M;          // m * w * u of Eq. 4
    float alpha, om;  // alpha and 1 - alpha
    int seg;          // TF segment; -1 below the first knot
    float dI;         // I - x_seg (0 below the first knot)
};

template <int KMAX>
__device__ __forceinline__ void tf_eval(const TFShared<KMAX> &sh, const float (&kx)[KMAX], float I, Opt &o)
{
    int seg = 0;
#pragma unroll
    for (int i = 1; i < KMAX; ++i) seg += (I >= kx[i]) ? 1 : 0;
    const bool below = I < kx[0];
    const float dI = below ? 0.f : I - sh.x[seg];
    const float4 v = sh.v[seg], s = sh.s[seg];
    o.c[0] = fmaf(dI, s.x, v.x);
    o.c[1] = fmaf(dI, s.y, v.y);
    o.c[2] = fmaf(dI, s.z, v.z);
    o.tau = fmaf(dI, s.w, v.w);
    o.seg = below ? -1 : seg;
    o.dI = dI;
}

__device__ __forceinline__ void eq4(const KRender &rp, float invg, const Chan &ch, float dk, Opt &o)
{
    const float gn = __builtin_amdgcn_sqrtf(ch.g[0] * ch.g[0] + ch.g[1] * ch.g[1] + ch.g[2] * ch.g[2]);
    const float m = fmaf(rp.lg, fminf(gn * invg, 1.f), rp.omlg);
    const float ak = fabsf(ch.k);
    const float w = fmaf(rp.lk, ak * __builtin_amdgcn_rcpf(ak + rp.k0), rp.omlk);
    const float u = fmaf(rp.lv, ch.V, 1.f);
    o.M = m * w * u;
    const float x = o.tau * o.M * dk;
    o.alpha = -expm1f(-x);
    o.om = 1.f - o.alpha;
}


// ------------------------------------------------------------------------------------------------
// One ray, front to back.  Lanes of pixels outside the image pass a ray with N = 0.
struct RayOut {
    float C0, C1, C2, A, T, Tprev;  // A = sum of T_k alpha_k (= 1 - T in exact arithmetic)
    int last, shaded;
};

// GATHER: the gather ceiling of this walk (a measurement, not the method).  The ray visits samples
// 0 .. kl only (kl = the k_last of a forward pass with the same arguments) and issues the same loads
// as the forward pass: the intensity corners of every non-skipped sample, the TF segment test, and
// the feature corners where the extinction is non-zero; Eq. 4, the exponential and the compositing
// are left out, and C0 returns a plain sum of the interpolated features that keeps the loads live.
template <int LAYOUT, int DT, int KMAX, bool GATHER = false>
__device__ __forceinline__ RayOut march_fwd(const KFeat &feat, const KGrid &g, const TFShared<KMAX> &sh,
                                            const float (&kx)[KMAX], const KRender &rp, float invg, const RayGeo &r,
                                            int kl = -1)
{
    RayOut o_;
    // the opacity is accumulated as a sum of the positive terms T_k alpha_k, relatively accurate
    // however faint the ray; 1 - T would carry an absolute error of one FP32 ulp of 1
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f, T = 1.f, Tprev = 1.f;
    int last = -1, shaded = 0;
    if (r.N > 0) {
        Vox<LAYOUT, DT> vx;
        vx.init(feat, g);
        int64_t q[3] = {r.q0[0], r.q0[1], r.q0[2]};
        int64_t dq[3] = {r.dq[0], r.dq[1], r.dq[2]};
        float dk = (r.N == 1) ? r.dlast : r.delta;
        CornerCache<LAYOUT, DT> cc;
        cc.reset();
        // empty-space skipping: a sample in a brick whose bit is set has alpha = 0 exactly; it is
        // passed with Tprev and last set as the full sample would set them, without fetching
        static_assert(DVR_BRICK == 4, "brick index = fixed-point position >> (32 + 2)");
        const bool skip = feat.bricks != nullptr;
        const int nbt = feat.nb[0] * feat.nb[1] * feat.nb[2];
        Buf bm;
        if (skip) bm = make_buf(feat.bricks + 2 * nbt, (uint32_t)((nbt + 31) / 32) * 4u);
        int cur_brick = -1;
        bool cur_empty = false;
        // the TF segment of the last full evaluation: [t_lo, t_hi) (empty before the first)
        float t_lo = INFINITY, t_hi = -INFINITY, t_x = 0.f;
        float4 t_v = make_float4(0.f, 0.f, 0.f, 0.f), t_s = t_v;
        bool t_below = false;
        const int nk = GATHER ? min(r.N, kl + 1) : r.N;
        for (int k = 0; k < nk; ++k) {
            if (skip) {
                const int bi = ((int)(q[2] >> 34) * feat.nb[1] + (int)(q[1] >> 34)) * feat.nb[0] + (int)(q[0] >> 34);
                if (bi != cur_brick) {
                    cur_brick = bi;
                    const uint32_t wd = __builtin_amdgcn_raw_buffer_load_b32(bm.r, (uint32_t)(bi >> 5) * 4u, 0, 0);
                    cur_empty = ((wd >> (bi & 31)) & 1u) != 0u;
                }
                if (cur_empty) {
                    Tprev = T;
                    last = k;
                    if (k + 1 == r.N - 1) {
                        dq[0] = r.dql[0]; dq[1] = r.dql[1]; dq[2] = r.dql[2];
                        dk = r.dlast;
                    }
                    q[0] += dq[0];
                    q[1] += dq[1];
                    q[2] += dq[2];
                    continue;
                }
            }
            Corners c;
            corner_setup(q, vx.sx, vx.sy, vx.sz, c);
            Chan ch;
            cc.need_I(vx, c);
            ch.I = cc.interp(c, 0);
            Opt o;
            if (ch.I >= t_lo && ch.I < t_hi) {
                // same TF segment as the previous evaluated sample: the same arithmetic as tf_eval
                // on the kept segment values, without the knot search and the LDS reads
                const float dI = t_below ? 0.f : ch.I - t_x;
                o.c[0] = fmaf(dI, t_s.x, t_v.x);
                o.c[1] = fmaf(dI, t_s.y, t_v.y);
                o.c[2] = fmaf(dI, t_s.z, t_v.z);
                o.tau = fmaf(dI, t_s.w, t_v.w);
            } else {
                tf_eval<KMAX>(sh, kx, ch.I, o);
                t_below = o.seg < 0;
                const int sg = t_below ? 0 : o.seg;
                t_x = sh.x[sg];
                t_v = sh.v[sg];
                t_s = sh.s[sg];
                t_lo = t_below ? -INFINITY : t_x;
                t_hi = t_below ? t_x : (sg + 1 < sh.K ? sh.x[sg + 1] : INFINITY);
            }
            Tprev = T;
            if (o.tau > 0.f) {
                ++shaded;
                cc.need_feat(vx, c);
                ch.g[0] = cc.interp(c, 1);
                ch.g[1] = cc.interp(c, 2);
                ch.g[2] = cc.interp(c, 3);
                ch.k = cc.interp(c, 4);
                ch.V = cc.interp(c, 5);
                if constexpr (GATHER) {
                    C0 += ((ch.g[0] + ch.g[1]) + (ch.g[2] + ch.k)) + (ch.V + o.tau);
                } else {
                    eq4(rp, invg, ch, dk, o);
                    const float ta = T * o.alpha;
                    C0 = fmaf(ta, o.c[0], C0);
                    C1 = fmaf(ta, o.c[1], C1);
                    C2 = fmaf(ta, o.c[2], C2);
                    A += ta;
                    T = T * o.om;
                }
            }
            last = k;
            if (T <= rp.Tstop) break;
            if (k + 1 == r.N - 1) {
                dq[0] = r.dql[0]; dq[1] = r.dql[1]; dq[2] = r.dql[2];
                dk = r.dlast;
            }
            q[0] += dq[0];
            q[1] += dq[1];
            q[2] += dq[2];
        }
    }
    o_.C0 = C0; o_.C1 = C1; o_.C2 = C2; o_.A = A; o_.T = T; o_.Tprev = Tprev; o_.last = last; o_.shaded = shaded;
    return o_;
}

// Workgroup sum of two per-lane counts (NW waves), one 64-bit atomic each per workgroup: the adds all
// go to the same two words, which the L2 serializes, so one per wave would cost a third of the
// raymarch.  Every thread of the workgroup must be here.
template <int NW>
__device__ __forceinline__ void count_samples(unsigned long long *counters, int last, int shaded)
{
    __shared__ uint32_t part[NW][2];
    uint32_t ev = (uint32_t)(last + 1), ns = (uint32_t)shaded;
    for (int o = 32; o > 0; o >>= 1) {
        ev += __shfl_xor(ev, o, 64);
        ns += __shfl_xor(ns, o, 64);
    }
    const uint32_t wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) {
        part[wv][0] = ev;
        part[wv][1] = ns;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long e = 0, n = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            e += part[w][0];
            n += part[w][1];
        }
        atomicAdd(counters, e);
        atomicAdd(counters + 1, n);
    }
}

// ------------------------------------------------------------------------------------------------
// Adjoint helpers.  TF-gradient accumulator of one lane: the register sums of the current TF segment.
// The workgroup's TF-gradient array is FP64 (see the dL/dI window on LDS atomics) and kept in
// tf_copies(KMAX) interleaved copies (entry p of copy j at p * copies + j, lane l using copy
// l % copies), so lanes of a wave that flush the same knot in the same instruction mostly add to
// different LDS words.
__host__ __device__ constexpr int tf_copies(int kmax) { return kmax <= 8 ? 16 : (kmax <= 16 ? 8 : 1); }

template <int COPIES>
struct SegAcc {
    int seg;         // current key: -1 below the first knot, 0..K-2 inside, K-1 above the last
    float lo[4], hi[4];

    __device__ __forceinline__ static void add(double *p, float v)
    {
        __hip_atomic_fetch_add(p, (double)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    // tfa: this lane's copy (workgroup array + lane % COPIES)
    __device__ __forceinline__ void flush(double *tfa, int K)
    {
        if (seg < 0 || seg >= K - 1) {
            const int kn = seg < 0 ? 0 : K - 1;
            for (int e = 0; e < 4; ++e)
                if (lo[e] != 0.f) add(tfa + (kn * 4 + e) * COPIES, lo[e]);
        } else {
            for (int e = 0; e < 4; ++e) {
                if (lo[e] != 0.f) add(tfa + (seg * 4 + e) * COPIES, lo[e]);
                if (hi[e] != 0.f) add(tfa + ((seg + 1) * 4 + e) * COPIES, hi[e]);
            }
        }
        for (int e = 0; e < 4; ++e) lo[e] = hi[e] = 0.f;
    }
};

// dL/dI scatter.  Neighbouring rays of a wave put their samples' corner weights on the same few
// voxels in the same instruction, and global float atomics on one address serialize, so each wave
// first accumulates into its own window of voxels in LDS and adds the window to dL/dI (one atomic
// per touched voxel) when a lane's cell falls outside it.  The window is re-placed around the cells
// of the lanes that need it, reaching ahead in the direction the rays walk (back to front); a lane
// whose corners do not fit adds to global memory directly.
// The window is kWin0 x kWin1 x kWin2 entries, its longest side along the volume axis the rays
// advance on fastest and its shortest along the slowest (fixed per wave at its first placement).
// Entries are FP64: LDS atomic adds on FP64 run at about the rate of integer ones on this chip,
// while FP32 LDS atomic adds are many times slower.
// With feature gradients the window holds six channels per voxel (I, gx, gy, gz, k, V) over a
// smaller box of 384 voxels, so that two workgroups' windows fit a CU; measured on the head, 8 x 8 x 6
// (2.12 ms per view) beat 6 x 8 x 8 (2.29) and 8 x 6 x 8 (2.13), while a side of 4 across the rays
// (12 x 8 x 4, 16 x 6 x 4, 4 x 8 x 12) cost 1.1-1.7x: the wave's rays do not fit it.
constexpr int kWin0 = 16, kWin1 = 12, kWin2 = 8;
constexpr int kFWin0 = 8, kFWin1 = 8, kFWin2 = 6;

__device__ __forceinline__ int wave_min_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Pairwise merge inside each quad of lanes (xor 1, then xor 2): where both lanes of a pair hold the
// same key, the lower lane adds the upper lane's values and the upper lane drops out.  Keys must be
// unique for lanes without values.  All lanes of the wave must be active.
template <int CTRL, int BIT, int NV>
__device__ __forceinline__ void quad_merge_step(bool &has, int key, float (&v)[NV])
{
    const int pk = __builtin_amdgcn_update_dpp(0, key, CTRL, 0xF, 0xF, false);
    const int ph = __builtin_amdgcn_update_dpp(0, has ? 1 : 0, CTRL, 0xF, 0xF, false);
    const bool same = (pk == key);
    const bool upper = ((threadIdx.x >> BIT) & 1u) != 0u;
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        const float pv =
            __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v[e]), CTRL, 0xF, 0xF, false));
        v[e] = same ? (upper ? 0.f : v[e] + pv) : v[e];
    }
    has = same ? (!upper && (has || ph != 0)) : has;
}

template <int NV>
__device__ __forceinline__ void quad_merge(bool &has, int key, float (&v)[NV])
{
    quad_merge_step<0xB1, 0>(has, key, v);  // quad_perm [1,0,3,2]: partner lane ^ 1
    quad_merge_step<0x4E, 1>(has, key, v);  // quad_perm [2,3,0,1]: partner lane ^ 2
}

template <int W0, int W1, int W2, int CH>
struct DWinT {
    static constexpr int kVox = W0 * W1 * W2;      // voxels of the window
    static constexpr int kEntries = kVox * CH;     // doubles in LDS
    static_assert(kVox % 64 == 0, "whole flush rounds");
    // entries are stored bank-swizzled: bits 1-3 of the index XOR bits 5-7, an involution within each
    // aligned block of 32, so that entries 32, 64, ... apart (neighbouring voxels along the window's
    // outer ranks, which the lanes of a wave add to in one instruction) fall in different LDS banks
    __device__ __forceinline__ static int swz(int e) { return e ^ (((e >> 5) & 7) << 1); }
    double *w;    // this wave's kEntries in LDS: [channel][voxel u0 + W0 (u1 + W1 u2)] (channel-major:
                  // lanes on neighbouring voxels of one channel fall in different banks)
    int o[3];     // voxel index (x, y, z) of the window's first entry; wave-uniform
    int ext[3];   // window extent along voxel axis x, y, z
    int st[3];    // window index stride of voxel axis x, y, z
    int gst[3];   // dL/dI index stride of the voxel axis on window rank 0, 1, 2
    int crn[8];   // window index offsets of the 8 cell corners (bit 0 x, bit 1 y, bit 2 z)
    bool live;    // window placed (it may hold partial sums)

    // ranks of the voxel axes by |dq| (descending), from one lane's front-to-back step
    __device__ __forceinline__ void orient(const int64_t dq[3], const KGrid &g)
    {
        const int64_t ax = dq[0] < 0 ? -dq[0] : dq[0], ay = dq[1] < 0 ? -dq[1] : dq[1], az = dq[2] < 0 ? -dq[2] : dq[2];
        int r[3];  // rank of axis x, y, z
        r[0] = (ay > ax) + (az > ax);
        r[1] = (ax >= ay) + (az > ay);
        r[2] = (ax >= az) + (ay >= az);
        const int W[3] = {W0, W1, W2};
        const int S[3] = {1, W0, W0 * W1};
        const int G[3] = {1, g.n[0], g.n[0] * g.n[1]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ext[a] = __builtin_amdgcn_readfirstlane(W[r[a]]);
            st[a] = __builtin_amdgcn_readfirstlane(S[r[a]]);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int a = (r[0] == k) ? 0 : ((r[1] == k) ? 1 : 2);
            gst[k] = __builtin_amdgcn_readfirstlane(G[a]);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) crn[e] = (e & 1) * st[0] + ((e >> 1) & 1) * st[1] + ((e >> 2) & 1) * st[2];
    }

    // add every non-zero entry to its output and clear it (all lanes of the wave): channel 0 to
    // dvol, channel c > 0 to dfeat[c - 1][.]
    __device__ __forceinline__ void flush(float *dvol, float *dfeat, const KGrid &g)
    {
        const int lane = threadIdx.x & 63;
        const int olin = o[0] + o[1] * g.n[0] + o[2] * g.n[0] * g.n[1];
        const size_t N = (size_t)g.n[0] * (size_t)g.n[1] * (size_t)g.n[2];
#pragma unroll 4
        for (int j = 0; j < kVox / 64; ++j) {
            const int e = lane + 64 * j;
            const int u0 = e % W0, u1 = (e / W0) % W1, u2 = e / (W0 * W1);
            // entries are only ever written for in-bounds voxels, so gi is in [0, N)
            const int gi = olin + u0 * gst[0] + u1 * gst[1] + u2 * gst[2];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const double v = w[c * kVox + swz(e)];
                if (v != 0.0) {
                    atomicAdd(c == 0 ? dvol + gi : dfeat + (size_t)(c - 1) * N + gi, (float)v);
                    w[c * kVox + swz(e)] = 0.0;
                }
            }
        }
    }

    __device__ __forceinline__ bool holds(const int cc[3]) const
    {
        return (uint32_t)(cc[0] - o[0]) <= (uint32_t)(ext[0] - 2) && (uint32_t)(cc[1] - o[1]) <= (uint32_t)(ext[1] - 2) &&
               (uint32_t)(cc[2] - o[2]) <= (uint32_t)(ext[2] - 2);
    }

    __device__ __forceinline__ int index(const int cc[3]) const
    {
        return (cc[0] - o[0]) * st[0] + (cc[1] - o[1]) * st[1] + (cc[2] - o[2]) * st[2];
    }

    // new origin from the cells of the lanes with need set (all lanes of the wave); dq_lead is the
    // front-to-back step of one of those lanes
    __device__ __forceinline__ void place(bool need, const int cc[3], const int64_t dq_lead[3])
    {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int lo = wave_min_i(need ? cc[a] : 0x7fffffff);
            const int hi = wave_max_i(need ? cc[a] : -0x7fffffff);
            // back to front the cells move against dq: put the window's slack on that side
            const int oa = dq_lead[a] > 0 ? hi + 2 - ext[a] : lo;
            o[a] = __builtin_amdgcn_readfirstlane(oa);
        }
        live = true;
    }
};

using DWin = DWinT<kWin0, kWin1, kWin2, 1>;
using DWinF = DWinT<kFWin0, kFWin1, kFWin2, 6>;

// Adjoint (back to front from the stored (T_last, k_last)).  With suffix colour S and suffix
// transmittance R of the samples behind k:
//   dL/dalpha_k = T_k (gC . (c_k - S) + gA R),   dL/dc_k = gC T_k alpha_k,
//   S <- alpha_k c_k + (1 - alpha_k) S,  R <- (1 - alpha_k) R,  T_{k-1} = T_k / (1 - alpha_{k-1}),
// then alpha = 1 - exp(-tau M delta_k) gives dL/dtau = dL/dalpha (1 - alpha) M delta_k; the TF is
// linear in its knot values on the sample's segment, and dL/dI_sample = sum_ch dL/dv_ch slope_ch is
// scattered to the 8 corners with the trilinear weights.
// TF-gradient accumulation: a lane adds into registers while its ray stays on one TF segment and
// flushes to a workgroup array in LDS (LDS atomics) when the segment changes; the workgroup array
// is added to the global [K][4] gradient with one atomic per parameter at the end.
//
// FG (feature gradients): with x = tau M delta_k and M = m w u, dL/dM = dL/dalpha (1 - alpha) tau delta_k
// is taken through m = (1 - lg) + lg min(|g| / gmax, 1) (to the interpolated g and to gmax, nothing
// where the ratio is clamped at 1), w = (1 - lk) + lk |k| / (|k| + k0) (nothing at k = 0) and
// u = 1 + lv V, and scattered to the 8 corners of [5][N] dfeat with the trilinear weights (global
// float atomics); the gmax part is summed in gmb.
//
// Every lane of the wave calls this (kl = -1 for a lane without a ray).  The loop runs over the
// sample index k from the wave's largest k_last down to 0, a lane taking part once k <= its own
// k_last, so at each step the lanes sit at the same sample index (the same depth for rays that
// entered through the same face) and the loop control stays wave-uniform for the dL/dI window.
template <int LAYOUT, int DT, int KMAX, bool FG>
__device__ __forceinline__ void march_bwd(const KFeat &feat, const KGrid &g, const TFShared<KMAX> &sh,
                                          const float (&kx)[KMAX], const KRender &rp, float invg, const RayGeo &r,
                                          int kl, float T_last, float4 gr, int K, double *tfa, float *dvol,
                                          double *win /* this wave's window entries of LDS, zeroed */,
                                          float *dfeat, float &gmb)
{
    const float gC0 = gr.x, gC1 = gr.y, gC2 = gr.z, gA = gr.w;
    float T = T_last;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, R = 1.f;
    Vox<LAYOUT, DT> vx;
    vx.init(feat, g);
    int64_t q[3];
    const bool at_last = (kl == r.N - 1);
    for (int a = 0; a < 3; ++a) q[a] = (kl < 0) ? 0 : (at_last ? r.ql[a] : r.q0[a] + (int64_t)kl * r.dq[a]);
    // byte offset of a corner -> voxel index (element sizes are powers of two)
    const uint32_t esh = (LAYOUT != DVR_INTERLEAVED) ? (DT == DVR_F32 ? 2u : 1u) : (DT == DVR_F32 ? 5u : 4u);
    SegAcc<tf_copies(KMAX)> sa;
    sa.seg = -2;
    for (int e = 0; e < 4; ++e) sa.lo[e] = sa.hi[e] = 0.f;
    CornerCache<LAYOUT, DT> cc;
    cc.reset();
    using Win = std::conditional_t<FG, DWinF, DWin>;
    Win dw;
    dw.w = win;
    dw.live = false;
    bool oriented = false;
    dw.o[0] = dw.o[1] = dw.o[2] = 0;
    // FG: this lane's running sums for the 8 corners of cell acell (see the loop)
    float acc[48];  // [corner][channel]
    int acell[3] = {-1, -1, -1};
    bool ahas = false;
#pragma unroll
    for (int e = 0; e < 48; ++e) acc[e] = 0.f;
    // all lanes call: lanes with flag set add acc to the window (placing it again if needed) or, when
    // their cell does not fit, to global memory
    auto emit_cell = [&](bool flag) {
        if constexpr (FG) {
            bool in = flag && dw.live && dw.holds(acell);
            const uint64_t miss = __ballot(flag && !in);
            if (miss) {
                const int lead = __ffsll((unsigned long long)miss) - 1;
                int64_t dql[3];
                for (int a = 0; a < 3; ++a) dql[a] = __shfl(r.dq[a], lead, 64);
                if (dw.live) dw.flush(dvol, dfeat, g);
                if (!oriented) {
                    dw.orient(dql, g);
                    oriented = true;
                }
                dw.place(flag, acell, dql);
                in = flag && dw.holds(acell);
            }
            if (in) {
                const int b = dw.index(acell);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    // the four lanes of a 2 x 2 pixel quad emit the corners in different orders (corner
                    // e XOR 0, 7, 3, 4): rays of one cell then add to different entries in each
                    // instruction.  Selected with bit masks, which keep the register sums out of scratch.
                    const int c0 = (threadIdx.x & 1u) ? -1 : 0, c1 = (threadIdx.x & 2u) ? -1 : 0;
                    const uint32_t m0 = (uint32_t)c0, m1 = (uint32_t)c1;
                    const int e7 = e ^ 7, e3 = e ^ 3, e4 = e ^ 4;
                    const int ca = (dw.crn[e] & ~c0) | (dw.crn[e7] & c0), cb = (dw.crn[e3] & ~c0) | (dw.crn[e4] & c0);
                    double *p = win + DWinF::swz(b + ((ca & ~c1) | (cb & c1)));
#pragma unroll
                    for (int ch6 = 0; ch6 < 6; ++ch6) {
                        const uint32_t va = (__builtin_bit_cast(uint32_t, acc[e * 6 + ch6]) & ~m0) |
                                            (__builtin_bit_cast(uint32_t, acc[e7 * 6 + ch6]) & m0);
                        const uint32_t vb = (__builtin_bit_cast(uint32_t, acc[e3 * 6 + ch6]) & ~m0) |
                                            (__builtin_bit_cast(uint32_t, acc[e4 * 6 + ch6]) & m0);
                        const float val = __builtin_bit_cast(float, (va & ~m1) | (vb & m1));
                        if (val != 0.f)
                            __hip_atomic_fetch_add(p + ch6 * DWinF::kVox, (double)val, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
                    }
                }
            } else if (flag) {
                const uint32_t nx = (uint32_t)g.n[0], plane = nx * (uint32_t)g.n[1];
                const size_t N = (size_t)plane * (size_t)g.n[2];
                const uint32_t v0 = (uint32_t)acell[2] * plane + (uint32_t)acell[1] * nx + (uint32_t)acell[0];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t vi = v0 + (e & 1) + ((e >> 1) & 1) * nx + ((e >> 2) & 1) * plane;
                    if (acc[e * 6] != 0.f) atomicAdd(dvol + vi, acc[e * 6]);
#pragma unroll
                    for (int f = 1; f < 6; ++f)
                        if (acc[e * 6 + f] != 0.f) atomicAdd(dfeat + (size_t)(f - 1) * N + vi, acc[e * 6 + f]);
                }
            }
        }
    };
    const int kmax = __builtin_amdgcn_readfirstlane(wave_max_i(kl));
    for (int k = kmax; k >= 0; --k) {
        const bool act = (k <= kl);
        float Ib = 0.f;
        float fv[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // FG: this sample's dL/d(gx, gy, gz, k, V)
        Corners c;
        int cell[3] = {0, 0, 0};
        if (act) {
            const float dk = (k == r.N - 1) ? r.dlast : r.delta;
            corner_setup(q, vx.sx, vx.sy, vx.sz, c);
            cell[0] = (int)(q[0] >> 32);
            cell[1] = (int)(q[1] >> 32);
            cell[2] = (int)(q[2] >> 32);
            Chan ch;
            cc.need_I(vx, c);
            ch.I = cc.interp(c, 0);
            Opt o;
            tf_eval<KMAX>(sh, kx, ch.I, o);
            // unlike the forward pass, a sample with zero extinction is not skipped: its alpha is 0,
            // but dalpha/dtau = (1 - alpha) M delta is not, so the TF-value gradient needs M
            cc.need_feat(vx, c);
            ch.g[0] = cc.interp(c, 1);
            ch.g[1] = cc.interp(c, 2);
            ch.g[2] = cc.interp(c, 3);
            ch.k = cc.interp(c, 4);
            ch.V = cc.interp(c, 5);
            eq4(rp, invg, ch, dk, o);
            if (k < kl) T = T / o.om;
            const float Ta = T * o.alpha;
            const float dal = T * (gC0 * (o.c[0] - S0) + gC1 * (o.c[1] - S1) + gC2 * (o.c[2] - S2) + gA * R);
            float vb[4];
            vb[0] = gC0 * Ta;
            vb[1] = gC1 * Ta;
            vb[2] = gC2 * Ta;
            vb[3] = dal * o.om * o.M * dk;
            if constexpr (FG) {
                const float Mb = dal * o.om * o.tau * dk;
                if (Mb != 0.f) {
                    const float gn = __builtin_amdgcn_sqrtf(ch.g[0] * ch.g[0] + ch.g[1] * ch.g[1] + ch.g[2] * ch.g[2]);
                    const float t = gn * invg;
                    const float m = fmaf(rp.lg, fminf(t, 1.f), rp.omlg);
                    const float ak = fabsf(ch.k);
                    const float rk = 1.f / (ak + rp.k0);
                    const float w = fmaf(rp.lk, ak * rk, rp.omlk);
                    const float u = fmaf(rp.lv, ch.V, 1.f);
                    float gs = 0.f;
                    if (t < 1.f && gn > 0.f) {
                        const float mb = Mb * w * u * rp.lg;
                        gs = mb * invg / gn;
                        gmb -= mb * t * invg;
                    }
                    const float sk = ch.k > 0.f ? 1.f : (ch.k < 0.f ? -1.f : 0.f);
                    fv[0] = gs * ch.g[0];
                    fv[1] = gs * ch.g[1];
                    fv[2] = gs * ch.g[2];
                    fv[3] = Mb * m * u * rp.lk * rp.k0 * sk * rk * rk;
                    fv[4] = Mb * m * w * rp.lv;
                }
            }
            S0 = fmaf(o.om, S0, o.alpha * o.c[0]);
            S1 = fmaf(o.om, S1, o.alpha * o.c[1]);
            S2 = fmaf(o.om, S2, o.alpha * o.c[2]);
            R = o.om * R;
            const int key = o.seg < 0 ? -1 : o.seg;
            if (key != sa.seg) {
                if (sa.seg != -2) sa.flush(tfa, K);
                sa.seg = key;
            }
            if (key < 0 || key >= K - 1) {
#pragma unroll
                for (int e = 0; e < 4; ++e) sa.lo[e] += vb[e];
            } else {
                const float t = o.dI * sh.iw[key];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    sa.lo[e] = fmaf(1.f - t, vb[e], sa.lo[e]);
                    sa.hi[e] = fmaf(t, vb[e], sa.hi[e]);
                }
                const float4 s = sh.s[key];
                Ib = vb[0] * s.x + vb[1] * s.y + vb[2] * s.z + vb[3] * s.w;
            }
        }
        if constexpr (FG) {
            // six channels (I, gx, gy, gz, k, V): a lane sums its cell's 8 corners in registers while
            // its ray stays in that cell and emits them when the cell changes (neighbouring rays in
            // one cell would otherwise add to the same LDS entries in the same instruction)
            const float val[6] = {dvol ? Ib : 0.f, fv[0], fv[1], fv[2], fv[3], fv[4]};
            const bool nz = act && (val[0] != 0.f || val[1] != 0.f || val[2] != 0.f || val[3] != 0.f ||
                                    val[4] != 0.f || val[5] != 0.f);
            const bool moved = act && (cell[0] != acell[0] || cell[1] != acell[1] || cell[2] != acell[2]);
            emit_cell(ahas && moved);
            if (moved) {
#pragma unroll
                for (int e = 0; e < 48; ++e) acc[e] = 0.f;
                acell[0] = cell[0];
                acell[1] = cell[1];
                acell[2] = cell[2];
                ahas = false;
            }
            if (nz) {
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                    for (int ch6 = 0; ch6 < 6; ++ch6) acc[e * 6 + ch6] = fmaf(c.w[e], val[ch6], acc[e * 6 + ch6]);
                ahas = true;
            }
        } else if (dvol) {
            bool need = act && Ib != 0.f;
            float cw[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) cw[e] = need ? c.w[e] * Ib : 0.f;
            // LDS atomics on one address from several lanes of an instruction are serialized; the
            // lanes of a quad (2 x 2 pixels) that sit in the same cell merge their corner values
            // first (the lower lane of each pair takes the sum).
            quad_merge(need, need ? (int)(c.off[0] >> esh) : (int)(0x80000000u | threadIdx.x), cw);
            bool in = need && dw.live && dw.holds(cell);
            const uint64_t miss = __ballot(need && !in);
            if (miss) {
                const int lead = __ffsll((unsigned long long)miss) - 1;
                int64_t dql[3];
                for (int a = 0; a < 3; ++a) dql[a] = __shfl(r.dq[a], lead, 64);
                if (dw.live) dw.flush(dvol, dfeat, g);
                if (!oriented) {
                    dw.orient(dql, g);
                    oriented = true;
                }
                dw.place(need, cell, dql);
                in = need && dw.holds(cell);
            }
            if (in) {
                const int b = dw.index(cell);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    // wave scope: only this wave touches its window
                    __hip_atomic_fetch_add(win + DWin::swz(b + dw.crn[e]), (double)cw[e], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
            } else if (need) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t off = c.off[e >> 1] + ((e & 1) ? vx.sx : 0u);
                    atomicAdd(dvol + (off >> esh), cw[e]);
                }
            }
        }
        if (act && k > 0) {
            const bool from_last = (k == r.N - 1) && r.N >= 2;
            q[0] -= from_last ? r.dql[0] : r.dq[0];
            q[1] -= from_last ? r.dql[1] : r.dq[1];
            q[2] -= from_last ? r.dql[2] : r.dq[2];
        }
    }
    if constexpr (FG) emit_cell(ahas);
    if ((FG || dvol) && dw.live) dw.flush(dvol, dfeat, g);
    if (sa.seg != -2) sa.flush(tfa, K);
}

}  // namespace dvr
