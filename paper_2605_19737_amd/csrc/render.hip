// Front-to-back raymarcher (Sec. 2.4 Eq. 4-6) and its adjoint, for gfx950.
//
// Mapping: one lane per ray; a wave covers an 8 x 8 pixel tile and a 256-lane workgroup a
// 16 x 16 tile, so the lanes of a wave gather neighbouring voxels.  A lane leaves the sample loop
// when its ray ends or terminates early; the wave leaves when every lane has (the exec mask of the
// loop empties), which is the wave-ballot early termination.
//
// Ray geometry.  The camera ray, the slab clip against [0,(n-1)h] and the segment count are
// computed once per ray in IEEE double with the same operation order as the FP64 definition (no
// FMA contraction), so N and the segment lengths agree with it.  Sample positions in voxel units
// are then carried in 32.32 fixed point: q_k = q_0 + k dq for the full segments and the midpoint
// of the shorter last segment separately.  Integer steps are exact and reversible, so the adjoint
// walks the same positions back to front, and the clamp of the first and last positions (plus a
// one-time check of the last full step) keeps every cell index inside [0, n-2] without per-sample
// clamping.  FP32 positions would be off by up to 1e-4 voxel at a perspective camera two box
// diagonals away, which moves the image by more than the 1e-5 parity budget.
//
// Per sample: trilinear I (8 gathers); the TF segment (knots in scalar registers, values and
// slopes in LDS); when the extinction is zero the sample is exactly transparent and the feature
// gathers are skipped; otherwise g, k, V (planar: 5 x 8 gathers; interleaved record: the same
// loads merged), Eq. 4 factors, alpha = -expm1(-sigma delta_k), C += T alpha c, T *= 1 - alpha.
#include <math.h>

#include "common.hpp"
#include "render_args.hpp"

namespace dvr {

constexpr double kS32 = 4294967296.0;

struct RayGeo {
    int N;               // number of segments (0 = miss)
    int64_t q0[3];       // fixed-point position of sample 0
    int64_t dq[3];       // step between full-segment samples
    int64_t dql[3];      // step from sample N-2 to the last sample
    int64_t ql[3];       // position of the last sample
    float delta, dlast;  // segment lengths (mm)
};

__device__ __forceinline__ int64_t to_fix(double q, int n)
{
    double v = q * kS32;
    const double hi = (double)(n - 1) * kS32 - 1.0;
    v = v < 0.0 ? 0.0 : (v > hi ? hi : v);
    return (int64_t)__double2ll_rn(v);
}

__device__ __forceinline__ RayGeo ray_setup(const KCam cam, int pi, int pj, const KGrid &g)
{
#pragma clang fp contract(off)
    RayGeo r;
    r.N = 0;
    const double fi = pi + 0.5, fj = pj + 0.5;
    double o[3], d[3];
    if (cam.persp) {
        double n2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            o[a] = cam.o[a];
            d[a] = (double)cam.d0[a] + fi * (double)cam.du[a] + fj * (double)cam.dv[a];
            n2 += d[a] * d[a];
        }
        const double nn = sqrt(n2);
        for (int a = 0; a < 3; ++a) d[a] /= nn;
    } else {
        for (int a = 0; a < 3; ++a) {
            o[a] = (double)cam.o[a] + fi * (double)cam.du[a] + fj * (double)cam.dv[a];
            d[a] = cam.d0[a];
        }
    }
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double hi = (double)(g.n[a] - 1) * (double)g.h[a];
        if (d[a] == 0.0) {
            if (o[a] < 0.0 || o[a] > hi) return r;
            continue;
        }
        double ta = (0.0 - o[a]) / d[a], tb = (hi - o[a]) / d[a];
        if (ta > tb) { const double t = ta; ta = tb; tb = t; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    const double tn = t0 > 0.0 ? t0 : 0.0, tf = t1;
    if (!(tf > tn)) return r;
    const double delta = g.delta;
    const double L = tf - tn;
    const double Nd = ceil(L / delta);
    if (!(Nd >= 1.0) || Nd > 2.0e9) return r;
    const int N = (int)Nd;
    const double dlast = L - (double)(N - 1) * delta;
    const double tfirst = tn + 0.0 * delta + 0.5 * (N == 1 ? dlast : delta);
    const double tlast = tn + (double)(N - 1) * delta + 0.5 * dlast;
    for (int a = 0; a < 3; ++a) {
        const double h = g.h[a];
        r.q0[a] = to_fix((o[a] + tfirst * d[a]) / h, g.n[a]);
        r.ql[a] = to_fix((o[a] + tlast * d[a]) / h, g.n[a]);
        int64_t st = (int64_t)__double2ll_rn(delta * d[a] / h * kS32);
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
    r.delta = (float)delta;
    r.dlast = (float)dlast;
    return r;
}

// ------------------------------------------------------------------------------------------------
// TF in LDS: knot x, value (R, G, B, tau), slope to the next knot (0 after the last), 1/width.
template <int KMAX>
struct TFShared {
    float4 v[KMAX];
    float4 s[KMAX];
    float x[KMAX];
    float iw[KMAX];
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
#pragma unroll
    for (int i = 0; i < KMAX; ++i) kx[i] = (i < K) ? tf.knots[i] : INFINITY;
}

// ------------------------------------------------------------------------------------------------
// Feature fetch.  LAYOUT/DT select planar planes or interleaved records.
template <int LAYOUT, int DT>
struct Vox {
    Buf b[6];  // planar: I, gx, gy, gz, kappa, V;  interleaved: b[0] = records
    uint32_t sx, sy, sz;  // byte strides of +1 in x, y, z

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
// (F32: 16 + 8 bytes, F16: 12 bytes kept packed and widened at use).
template <int LAYOUT, int DT>
struct CornerCache {
    static constexpr bool kPacked = (LAYOUT == DVR_INTERLEAVED && DT == DVR_F16);
    uint32_t base;  // byte offset of the cached cell's first corner, or ~0
    bool feat;      // feature corners valid for this cell
    float v[kPacked ? 1 : 8][6];
    uint32_t raw[kPacked ? 8 : 1][3];

    __device__ __forceinline__ void reset()
    {
        base = 0xffffffffu;
        feat = false;
    }

    __device__ __forceinline__ void need_I(const Vox<LAYOUT, DT> &vx, const Corners &c)
    {
        if (c.off[0] == base) return;
        base = c.off[0];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t off = c.off[e >> 1] + ((e & 1) ? vx.sx : 0u);
            if constexpr (LAYOUT == DVR_PLANAR) {
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
        if constexpr (LAYOUT == DVR_PLANAR) {
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
// The camera index is uniform over the workgroup; copying the record field by field keeps the
// by-value kernel argument block in the constant segment (taking its address would make the
// compiler copy the whole block to per-lane scratch).
__device__ __forceinline__ KCam load_cam(const KLaunch &L, uint32_t cam)
{
    cam = __builtin_amdgcn_readfirstlane(cam);
    KCam c;
    c.persp = L.cams[cam].persp;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.o[a] = L.cams[cam].o[a];
        c.d0[a] = L.cams[cam].d0[a];
        c.du[a] = L.cams[cam].du[a];
        c.dv[a] = L.cams[cam].dv[a];
    }
    return c;
}

__device__ __forceinline__ void pixel_of(const KLaunch &L, uint32_t &cam, int &pi, int &pj, bool &valid)
{
    // XCD-aware order: consecutive dispatch slots go to different XCDs, so logical tile t is placed
    // at slot (t % per) * 8 + t / per; each XCD then walks a contiguous range of tiles.
    const uint32_t b = blockIdx.x;
    const uint32_t per = gridDim.x / 8u;
    const uint32_t t = (b & 7u) * per + (b >> 3);
    const uint32_t tiles_x = (L.W + 15) / 16, tiles_y = (L.H + 15) / 16;
    const uint32_t tpv = tiles_x * tiles_y;
    cam = t / tpv;
    const uint32_t tt = t - cam * tpv;
    const uint32_t ty = tt / tiles_x, tx = tt - ty * tiles_x;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    pi = (int)(tx * 16u + (wv & 1u) * 8u + (lane & 7u));
    pj = (int)(ty * 16u + (wv >> 1) * 8u + (lane >> 3));
    valid = cam < (uint32_t)L.ncam && pi < L.W && pj < L.H;
}

template <int LAYOUT, int DT, int KMAX>
__global__ __launch_bounds__(256) void k_render(KFeat feat, KGrid g, KTF tf, KRender rp, KLaunch L)
{
    __shared__ TFShared<KMAX> sh;
    float kx[KMAX];
    tf_load<KMAX>(sh, kx, tf);
    __syncthreads();
    uint32_t cam;
    int pi, pj;
    bool valid;
    pixel_of(L, cam, pi, pj, valid);
    const float gm = *feat.gmax;
    const float invg = gm > 0.f ? 1.f / gm : 0.f;
    RayGeo r;
    r.N = 0;
    if (valid) r = ray_setup(load_cam(L, cam), pi, pj, g);
    const size_t pix = valid ? ((size_t)(L.cam_base + cam) * L.H + pj) * L.W + pi : 0;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f, Tprev = 1.f;
    int last = -1, shaded = 0;
    if (r.N > 0) {
        Vox<LAYOUT, DT> vx;
        vx.init(feat, g);
        int64_t q[3] = {r.q0[0], r.q0[1], r.q0[2]};
        int64_t dq[3] = {r.dq[0], r.dq[1], r.dq[2]};
        float dk = (r.N == 1) ? r.dlast : r.delta;
        CornerCache<LAYOUT, DT> cc;
        cc.reset();
        for (int k = 0; k < r.N; ++k) {
            Corners c;
            corner_setup(q, vx.sx, vx.sy, vx.sz, c);
            Chan ch;
            cc.need_I(vx, c);
            ch.I = cc.interp(c, 0);
            Opt o;
            tf_eval<KMAX>(sh, kx, ch.I, o);
            Tprev = T;
            if (o.tau > 0.f) {
                ++shaded;
                cc.need_feat(vx, c);
                ch.g[0] = cc.interp(c, 1);
                ch.g[1] = cc.interp(c, 2);
                ch.g[2] = cc.interp(c, 3);
                ch.k = cc.interp(c, 4);
                ch.V = cc.interp(c, 5);
                eq4(rp, invg, ch, dk, o);
                const float ta = T * o.alpha;
                C0 = fmaf(ta, o.c[0], C0);
                C1 = fmaf(ta, o.c[1], C1);
                C2 = fmaf(ta, o.c[2], C2);
                T = T * o.om;
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
    if (valid) {
        reinterpret_cast<float4 *>(L.out)[pix] = make_float4(C0, C1, C2, 1.f - T);
        if (L.T_last) L.T_last[pix] = Tprev;
        if (L.k_last) L.k_last[pix] = last;
    }
    if (L.counters) {
        // every lane of the wave is here (no early exit): one atomic per wave
        uint32_t ev = (uint32_t)(last + 1), ns = (uint32_t)shaded;
        for (int o = 32; o > 0; o >>= 1) {
            ev += __shfl_xor(ev, o, 64);
            ns += __shfl_xor(ns, o, 64);
        }
        if ((threadIdx.x & 63u) == 0) {
            atomicAdd(L.counters, (unsigned long long)ev);
            atomicAdd(L.counters + 1, (unsigned long long)ns);
        }
    }
}

// ------------------------------------------------------------------------------------------------
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
struct SegAcc {
    int seg;         // current key: -1 below the first knot, 0..K-2 inside, K-1 above the last
    float lo[4], hi[4];

    __device__ __forceinline__ void flush(float *tfa, int K)
    {
        if (seg < 0 || seg >= K - 1) {
            const int kn = seg < 0 ? 0 : K - 1;
            for (int e = 0; e < 4; ++e)
                if (lo[e] != 0.f) atomicAdd(tfa + kn * 4 + e, lo[e]);
        } else {
            for (int e = 0; e < 4; ++e) {
                if (lo[e] != 0.f) atomicAdd(tfa + seg * 4 + e, lo[e]);
                if (hi[e] != 0.f) atomicAdd(tfa + (seg + 1) * 4 + e, hi[e]);
            }
        }
        for (int e = 0; e < 4; ++e) lo[e] = hi[e] = 0.f;
    }
};

template <int LAYOUT, int DT, int KMAX>
__global__ __launch_bounds__(256) void k_render_bwd(KFeat feat, KGrid g, KTF tf, KRender rp, KLaunch L)
{
    __shared__ TFShared<KMAX> sh;
    __shared__ float tfa[KMAX * 4];
    float kx[KMAX];
    tf_load<KMAX>(sh, kx, tf);
    for (int p = threadIdx.x; p < KMAX * 4; p += 256) tfa[p] = 0.f;
    __syncthreads();
    const int K = tf.K;
    uint32_t cam;
    int pi, pj;
    bool valid;
    pixel_of(L, cam, pi, pj, valid);
    const size_t pix = valid ? ((size_t)(L.cam_base + cam) * L.H + pj) * L.W + pi : 0;
    const int kl = valid ? L.k_last[pix] : -1;
    if (kl >= 0) {
        const float gm = *feat.gmax;
        const float invg = gm > 0.f ? 1.f / gm : 0.f;
        const RayGeo r = ray_setup(load_cam(L, cam), pi, pj, g);
        const float4 gr = reinterpret_cast<const float4 *>(L.dout)[pix];
        const float gC0 = gr.x, gC1 = gr.y, gC2 = gr.z, gA = gr.w;
        float T = L.T_last[pix];
        float S0 = 0.f, S1 = 0.f, S2 = 0.f, R = 1.f;
        Vox<LAYOUT, DT> vx;
        vx.init(feat, g);
        int64_t q[3];
        const bool at_last = (kl == r.N - 1);
        for (int a = 0; a < 3; ++a) q[a] = at_last ? r.ql[a] : r.q0[a] + (int64_t)kl * r.dq[a];
        // byte offset of a corner -> voxel index (element sizes are powers of two)
        const uint32_t esh = (LAYOUT == DVR_PLANAR) ? (DT == DVR_F32 ? 2u : 1u) : (DT == DVR_F32 ? 5u : 4u);
        SegAcc sa;
        sa.seg = -2;
        for (int e = 0; e < 4; ++e) sa.lo[e] = sa.hi[e] = 0.f;
        CornerCache<LAYOUT, DT> cc;
        cc.reset();
        for (int k = kl; k >= 0; --k) {
            const float dk = (k == r.N - 1) ? r.dlast : r.delta;
            Corners c;
            corner_setup(q, vx.sx, vx.sy, vx.sz, c);
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
                if (L.dvol) {
                    const float4 s = sh.s[key];
                    const float Ib = vb[0] * s.x + vb[1] * s.y + vb[2] * s.z + vb[3] * s.w;
                    if (Ib != 0.f) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const uint32_t off = c.off[e >> 1] + ((e & 1) ? vx.sx : 0u);
                            atomicAdd(L.dvol + (off >> esh), c.w[e] * Ib);
                        }
                    }
                }
            }
            if (k > 0) {
                const bool from_last = (k == r.N - 1) && r.N >= 2;
                q[0] -= from_last ? r.dql[0] : r.dq[0];
                q[1] -= from_last ? r.dql[1] : r.dq[1];
                q[2] -= from_last ? r.dql[2] : r.dq[2];
            }
        }
        if (sa.seg != -2) sa.flush(tfa, K);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < K * 4; p += 256)
        if (tfa[p] != 0.f) atomicAdd(L.dtf + p, tfa[p]);
}

// ------------------------------------------------------------------------------------------------
template <int LAYOUT, int DT, int KMAX>
static hipError_t launch_fwd_t(const KFeat &f, const KGrid &g, const KTF &tf, const KRender &rp, const KLaunch &L,
                               uint32_t blocks, hipStream_t st, bool bwd)
{
    if (bwd)
        hipLaunchKernelGGL((k_render_bwd<LAYOUT, DT, KMAX>), dim3(blocks), dim3(256), 0, st, f, g, tf, rp, L);
    else
        hipLaunchKernelGGL((k_render<LAYOUT, DT, KMAX>), dim3(blocks), dim3(256), 0, st, f, g, tf, rp, L);
    return hipGetLastError();
}

template <int LAYOUT, int DT>
static hipError_t launch_k(const KFeat &f, const KGrid &g, const KTF &tf, const KRender &rp, const KLaunch &L,
                           uint32_t blocks, hipStream_t st, bool bwd)
{
    if (tf.K <= 8) return launch_fwd_t<LAYOUT, DT, 8>(f, g, tf, rp, L, blocks, st, bwd);
    if (tf.K <= 16) return launch_fwd_t<LAYOUT, DT, 16>(f, g, tf, rp, L, blocks, st, bwd);
    return launch_fwd_t<LAYOUT, DT, 64>(f, g, tf, rp, L, blocks, st, bwd);
}

static hipError_t launch_any(const RenderArgs &a, hipStream_t st, bool bwd)
{
    for (int c0 = 0; c0 < a.ncam; c0 += kCamChunk) {
        KLaunch L = a.launch;
        L.ncam = a.ncam - c0 < kCamChunk ? a.ncam - c0 : kCamChunk;
        L.cam_base = c0;
        for (int i = 0; i < L.ncam; ++i) L.cams[i] = a.cams[c0 + i];
        const uint32_t tiles = (uint32_t)((L.W + 15) / 16) * (uint32_t)((L.H + 15) / 16) * (uint32_t)L.ncam;
        const uint32_t blocks = (tiles + 7u) / 8u * 8u;
        hipError_t e;
        const int lay = a.feat.layout, dt = a.feat.dtype;
        if (lay == DVR_PLANAR && dt == DVR_F32) e = launch_k<DVR_PLANAR, DVR_F32>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, bwd);
        else if (lay == DVR_PLANAR && dt == DVR_F16) e = launch_k<DVR_PLANAR, DVR_F16>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, bwd);
        else if (lay == DVR_INTERLEAVED && dt == DVR_F32) e = launch_k<DVR_INTERLEAVED, DVR_F32>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, bwd);
        else if (lay == DVR_INTERLEAVED && dt == DVR_F16) e = launch_k<DVR_INTERLEAVED, DVR_F16>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, bwd);
        else e = hipErrorInvalidValue;
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_render(const RenderArgs &a, hipStream_t st) { return launch_any(a, st, false); }
hipError_t launch_render_backward(const RenderArgs &a, hipStream_t st) { return launch_any(a, st, true); }

}  // namespace dvr

namespace dvr {

__global__ __launch_bounds__(256) void k_fill_zero(float *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.f;
}

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t st)
{
    const int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace dvr
