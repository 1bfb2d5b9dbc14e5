// Batched persistent launch: the feature pass of many volumes and the raymarch of many views, in
// one persistent kernel recorded in a HIP graph, with tile shapes chosen by an autotuner.
//
// Work queue.  Items are taken in a fixed order from one atomic counter:
//   Z  (volume, scale, slab of z slices): z filters of the slab into the volume's workspace;
//   XY (volume, scale, 2-D tile, run of z slices): y/x filters, Hessian, eigenvalues, k, V, g;
//   Q  (volume, slab of z slices; quad layout only): the V and intensity quads of the slab;
//   RAY (view, 16x16 pixel tile): one ray per lane, front to back.
// An XY item waits until every Z item of its (volume, scale) is done (and, for scale s > 0, every
// XY item of scale s-1, whose vesselness it max-accumulates); a RAY item waits until every XY item
// of its volume is done (features and |g|_max complete; with quad-layout features, every Q item of
// its volume, which itself waits for the volume's last XY scale).  Completion is a per-(volume, scale)
// counter incremented after a device-scope release (every wave writes its L2 back); the waiter
// polls, then acquires (invalidates its L2) once per volume per workgroup.  An item only waits for
// items earlier in the queue, which were taken by running workgroups that never wait for later
// items, so the launch makes progress at any grid size; each wait is still bounded and sets an
// error flag instead of hanging.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"
#include "features_dev.hpp"
#include "host.hpp"
#include "render_args.hpp"
#include "render_dev.hpp"

namespace dvr {

enum { IT_Z = 0, IT_XY = 1, IT_RAY = 2, IT_Q = 3 };
constexpr unsigned kMaxSpin = 1u << 23;  // polls of ~0.5 us: a wait gives up after several seconds
constexpr int kMaxVolScale = 8192;       // volumes x scales per plan (LDS bitmaps of acquired counters)

struct BItem {
    int32_t type_scale;  // type | scale << 8
    int32_t v;           // volume (Z, XY, Q) or view (RAY)
    int32_t a;           // Z, Q: first slice; XY: tile index; RAY: tile index
    int32_t b;           // Z, Q: end slice; XY: first slice of the run
};

struct BVol {
    const void *vol;
    void *grad, *kappa, *ves;
    float *gmax;
    float *ws;  // [nsigma][3][N] z-filtered fields
    void *iquad;  // quad layout: the intensity quads
    void *vtmp;   // quad layout: V as a plain field (features dtype) until the Q items build its quads
    int32_t n[3];
    int32_t tiles_x;
    KGrid grid;  // extents, spacings and segment length for the ray setup
    float inv2h[3];
};

struct BView {
    KCam cam;
    int32_t vol, W, H, tiles_x;
    float *rgba;
    float *T_last;
    int32_t *k_last;
};

// Read-only tables are addressed through the constant address space so that the uniform loads
// of their fields become scalar loads (held in SGPRs) rather than per-lane vector loads.
template <typename T>
using CP = const __attribute__((address_space(4))) T *;

struct BatchArgs {
    uint64_t items;  // BItem[nitems]
    int32_t nitems, ns, zrun, ray_tile;
    uint64_t vols;   // BVol[nvol]
    uint64_t views;  // BView[nview]
    uint64_t taps;   // ScaleTaps[volume * ns + scale]
    unsigned *head, *zdone, *xydone, *err;
    const unsigned *nz_items, *nxy_items;
    unsigned *qdone;           // per volume: Q items done (quad layout)
    const unsigned *nq_items;  // per volume: Q items
    const unsigned *ray_need;  // count a ray tile waits for (= nxy_items, see the timeout test hook)
    unsigned max_spin;  // bound of every dependency wait (polls)
    float c, inv2a2, inv2b2, tau;
    KTF tf;
    KRender rp;
};

__device__ __forceinline__ bool bit_test_set(unsigned *bits, int i)
{
    const unsigned m = 1u << (i & 31);
    if (bits[i >> 5] & m) return true;
    bits[i >> 5] |= m;
    return false;
}

// Thread 0: wait until *ctr >= target (bounded); then acquire once per (workgroup, counter).
__device__ __forceinline__ void wait_for(unsigned *ctr, unsigned target, unsigned *err, unsigned *acq, int idx,
                                         unsigned max_spin)
{
    if (threadIdx.x != 0) return;
    if (acq[idx >> 5] & (1u << (idx & 31))) return;
    unsigned n = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++n > max_spin) {
            atomicOr(err, 1u);
            break;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    bit_test_set(acq, idx);
}

// Every wave releases its writes at device scope, then one lane bumps the completion counter.
__device__ __forceinline__ void release_done(unsigned *ctr)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int TXY>
struct XYShape;
template <> struct XYShape<0> { static constexpr int TX = 64, TY = 8; };
template <> struct XYShape<1> { static constexpr int TX = 32, TY = 16; };
template <> struct XYShape<2> { static constexpr int TX = 128, TY = 4; };

__device__ __forceinline__ void ray_pixel(int ray_tile, int tiles_x, int tile, int &pi, int &pj)
{
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int ox, oy;
    if (ray_tile == 1) {         // 16 x 4 per wave, waves stacked in y
        ox = lane & 15;
        oy = wv * 4 + (lane >> 4);
    } else if (ray_tile == 2) {  // 4 x 16 per wave, waves side by side in x
        ox = wv * 4 + (lane & 3);
        oy = lane >> 2;
    } else {                     // 8 x 8 per wave, 2 x 2 waves
        ox = (wv & 1) * 8 + (lane & 7);
        oy = (wv >> 1) * 8 + (lane >> 3);
    }
    pi = tx * 16 + ox;
    pj = ty * 16 + oy;
}

// Quads of slices [z0, z1) of one volume (the workgroup's 256 lanes over the slices' voxels):
// dst[v] = (src(x,y,z), src(x,y+1,z), src(x,y,z+1), src(x,y+1,z+1)), 0 past the last row or slice,
// as bit copies of the features dtype, for V (from the plain field) and for the intensity.
template <typename T, typename T4>
__device__ __forceinline__ void quads_slab(const T *__restrict__ src, T4 *__restrict__ dst, uint32_t nx, uint32_t ny,
                                           uint32_t nz, int z0, int z1)
{
    const uint32_t plane = nx * ny;
    const uint32_t end = (uint32_t)z1 * plane;
    for (uint32_t v = (uint32_t)z0 * plane + threadIdx.x; v < end; v += 256u) {
        const uint32_t row = v / nx, y = row % ny, z = row / ny;
        const bool yi = y + 1u < ny, zi = z + 1u < nz;
        T4 q;
        q.x = src[v];
        q.y = yi ? src[v + nx] : T(0);
        q.z = zi ? src[v + plane] : T(0);
        q.w = (yi && zi) ? src[v + plane + nx] : T(0);
        dst[v] = q;
    }
}

// The fixed-radius tile for radius Rr (a uniform value) over slices [z0, z1), if 2 <= Rr <= 10.
template <int DT, int LAYOUT, int TX, int TY, int R, typename ST>
__device__ __forceinline__ bool xy_fixed(const XYArgs &a, const ST &taps, int Rr, int x0, int y0, int z0, int z1,
                                         float *lds, float &vmax)
{
    if constexpr (R > 10) {
        return false;
    } else {
        if (Rr != R) return xy_fixed<DT, LAYOUT, TX, TY, R + 1>(a, taps, Rr, x0, y0, z0, z1, lds, vmax);
        vmax = xy_run_r<DT, DT, LAYOUT, R, TX, TY>(a, taps, x0, y0, z0, z1, lds, lds);
        return true;
    }
}

template <int LAYOUT, int DT, int KMAX, int TXY>
__global__ __launch_bounds__(256, 3) void k_batch(BatchArgs A)
{
    constexpr int TX = XYShape<TXY>::TX, TY = XYShape<TXY>::TY;
    extern __shared__ float lds[];
    __shared__ TFShared<KMAX> sh;
    __shared__ unsigned acq_z[kMaxVolScale / 32], acq_xy[kMaxVolScale / 32], acq_q[kMaxVolScale / 32];
    // the quad layout computes its features as the split layout, with V into the volume's plain field
    constexpr int FLAYOUT = (LAYOUT == DVR_QUAD) ? DVR_SPLIT : LAYOUT;
    __shared__ int item_sh;
    float kx[KMAX];
    tf_load<KMAX>(sh, kx, A.tf);
    for (int i = threadIdx.x; i < kMaxVolScale / 32; i += 256) acq_z[i] = acq_xy[i] = acq_q[i] = 0u;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) item_sh = (int)atomicAdd(A.head, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(item_sh);
        __syncthreads();
        if (it >= A.nitems) break;
        const CP<BItem> items = (CP<BItem>)A.items;
        const CP<BVol> vols = (CP<BVol>)A.vols;
        const CP<BView> views = (CP<BView>)A.views;
        const CP<ScaleTaps> tapt = (CP<ScaleTaps>)A.taps;
        BItem w;
        w.type_scale = items[it].type_scale;
        w.v = items[it].v;
        w.a = items[it].a;
        w.b = items[it].b;
        const int type = w.type_scale & 0xff, s = w.type_scale >> 8;
        if (type == IT_Z) {
            const auto &V = vols[w.v];
            const uint32_t plane = (uint32_t)V.n[0] * (uint32_t)V.n[1];
            const uint32_t N = plane * (uint32_t)V.n[2];
            float *ws = V.ws + (size_t)s * 3u * N;
            const auto &tz = tapt[w.v * A.ns + s].ax[2];
            for (int z = w.a; z < w.b; ++z)
                for (uint32_t e = threadIdx.x; e < plane; e += 256u)
                    zpass_voxel<DT>(V.vol, ws, V.n[0], V.n[1], V.n[2], tz, e, z);
            release_done(A.zdone + w.v * A.ns + s);
        } else if (type == IT_XY) {
            const int vs = w.v * A.ns + s;
            wait_for(A.zdone + vs, A.nz_items[vs], A.err, acq_z, vs, A.max_spin);
            if (s > 0) wait_for(A.xydone + vs - 1, A.nxy_items[vs - 1], A.err, acq_xy, vs - 1, A.max_spin);
            __syncthreads();
            const auto &V = vols[w.v];
            const uint32_t N = (uint32_t)V.n[0] * (uint32_t)V.n[1] * (uint32_t)V.n[2];
            XYArgs a;
            a.ws = V.ws + (size_t)s * 3u * N;
            a.vol = V.vol;
            a.grad = V.grad;
            a.kappa = V.kappa;
            a.ves = (LAYOUT == DVR_QUAD) ? V.vtmp : V.ves;
            a.gmax = V.gmax;
            a.fro = nullptr;
            a.nx = V.n[0];
            a.ny = V.n[1];
            a.nz = V.n[2];
            a.inv2h[0] = V.inv2h[0];
            a.inv2h[1] = V.inv2h[1];
            a.inv2h[2] = V.inv2h[2];
            a.c_host = A.c;
            a.inv2a2 = A.inv2a2;
            a.inv2b2 = A.inv2b2;
            a.tau = A.tau;
            a.first = (s == 0);
            a.fro_pass = 0;
            const auto &taps = tapt[vs];
            const int bx = w.a % V.tiles_x, by = w.a / V.tiles_x;
            const int z1 = min(w.b + A.zrun, V.n[2]);
            float vmax = 0.f;
            // the fixed-radius tile (equal x and y radius 2..10) for the split-layout features of the
            // split and quad launches; the generic tile otherwise
            bool done = false;
            if constexpr (TXY == 0 && FLAYOUT == DVR_SPLIT)
                if (taps.ax[0].R == taps.ax[1].R)
                    done = xy_fixed<DT, FLAYOUT, TX, TY, 2>(a, taps, taps.ax[0].R, bx * TX, by * TY, w.b, z1, lds, vmax);
            if (!done)
                for (int z = w.b; z < z1; ++z)
                    vmax = fmaxf(vmax, xy_tile<DT, DT, FLAYOUT, TX, TY>(a, taps, bx * TX, by * TY, z, lds));
            if (s == 0) {
                vmax = wave_max(vmax);
                if ((threadIdx.x & 63) == 0) atomic_max_pos(V.gmax, vmax);
            }
            release_done(A.xydone + vs);
        } else if (type == IT_Q) {
            if constexpr (LAYOUT == DVR_QUAD) {
                const int vs = w.v * A.ns + A.ns - 1;
                wait_for(A.xydone + vs, A.nxy_items[vs], A.err, acq_xy, vs, A.max_spin);
                __syncthreads();
                const auto &V = vols[w.v];
                const uint32_t nx = (uint32_t)V.n[0], ny = (uint32_t)V.n[1], nz = (uint32_t)V.n[2];
                if constexpr (DT == DVR_F32) {
                    quads_slab(static_cast<const uint32_t *>(V.vtmp), static_cast<uint4 *>(V.ves), nx, ny, nz, w.a, w.b);
                    quads_slab(static_cast<const uint32_t *>(V.vol), static_cast<uint4 *>(V.iquad), nx, ny, nz, w.a, w.b);
                } else {
                    quads_slab(static_cast<const uint16_t *>(V.vtmp), static_cast<ushort4 *>(V.ves), nx, ny, nz, w.a, w.b);
                    quads_slab(static_cast<const uint16_t *>(V.vol), static_cast<ushort4 *>(V.iquad), nx, ny, nz, w.a,
                               w.b);
                }
                release_done(A.qdone + w.v);
            }
        } else {
            const auto &Vw = views[w.v];
            const int vol = Vw.vol;
            const int vs = vol * A.ns + A.ns - 1;
            if constexpr (LAYOUT == DVR_QUAD)
                wait_for(A.qdone + vol, A.nq_items[vol], A.err, acq_q, vol, A.max_spin);
            else
                wait_for(A.xydone + vs, A.ray_need[vs], A.err, acq_xy, vs, A.max_spin);
            __syncthreads();
            const auto &V = vols[vol];
            KFeat f;
            f.vol = (LAYOUT == DVR_QUAD) ? V.iquad : V.vol;
            f.grad = V.grad;
            f.kappa = V.kappa;
            f.ves = V.ves;
            f.gmax = V.gmax;
            f.dtype = DT;
            f.layout = LAYOUT;
            f.bricks = nullptr;  // the batched launch builds no brick tables
            f.nb[0] = f.nb[1] = f.nb[2] = 0;
            KGrid g;  // field by field: V lives in the constant address space
            for (int k = 0; k < 3; ++k) {
                g.n[k] = V.grid.n[k];
                g.h[k] = V.grid.h[k];
                g.ih_hi[k] = V.grid.ih_hi[k];
                g.ih_lo[k] = V.grid.ih_lo[k];
            }
            g.delta_hi = V.grid.delta_hi;
            g.delta_lo = V.grid.delta_lo;
            g.idelta_hi = V.grid.idelta_hi;
            g.idelta_lo = V.grid.idelta_lo;
            const float gm = __hip_atomic_load(V.gmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const float invg = gm > 0.f ? 1.f / gm : 0.f;
            int pi, pj;
            ray_pixel(A.ray_tile, Vw.tiles_x, w.a, pi, pj);
            const bool valid = pi < Vw.W && pj < Vw.H;
            RayGeo r;
            r.N = 0;
            KCam cam;
            cam.persp = Vw.cam.persp;
            for (int k = 0; k < 3; ++k) {
                cam.o[k] = Vw.cam.o[k];
                cam.d0[k] = Vw.cam.d0[k];
                cam.du[k] = Vw.cam.du[k];
                cam.dv[k] = Vw.cam.dv[k];
            }
            if (valid) r = ray_setup(cam, pi, pj, g);
            const RayOut o = march_fwd<LAYOUT, DT, KMAX>(f, g, sh, kx, A.rp, invg, r);
            if (valid) {
                const size_t pix = (size_t)pj * Vw.W + pi;
                reinterpret_cast<float4 *>(Vw.rgba)[pix] = make_float4(o.C0, o.C1, o.C2, o.A);
                if (Vw.T_last) {
                    Vw.T_last[pix] = o.Tprev;
                    if (Vw.k_last) Vw.k_last[pix] = o.last;
                }
            }
        }
    }
}

// Reset the queue, counters, error flag and every volume's |g|_max (no memset nodes in the graph).
__global__ void k_batch_init(BatchArgs A, int nvs, int nvol)
{
    const int n = 2 * nvs + 2;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (i == 0) *A.head = 0u;
        else if (i == 1) *A.err = 0u;
        else if (i < 2 + nvs) A.zdone[i - 2] = 0u;
        else A.xydone[i - 2 - nvs] = 0u;
    }
    const BVol *vols = (const BVol *)A.vols;
    for (int v = threadIdx.x; v < nvol; v += blockDim.x) {
        *vols[v].gmax = 0.f;
        A.qdone[v] = 0u;
    }
}

// ------------------------------------------------------------------------------------------------
// host side

static hipError_t launch_batch_kernel(const BatchArgs &A, int layout, int dt, int tf_k, int txy, unsigned grid,
                                      size_t lds, hipStream_t st)
{
#define DVR_B(L, D, KM, T)                                                                                     \
    if (layout == L && dt == D && (KM == 16 ? tf_k <= 16 : tf_k > 16) && txy == T) {                            \
        hipLaunchKernelGGL((k_batch<L, D, KM, T>), dim3(grid), dim3(256), lds, st, A);                          \
        return hipGetLastError();                                                                               \
    }
#define DVR_B3(L, D, KM) DVR_B(L, D, KM, 0) DVR_B(L, D, KM, 1) DVR_B(L, D, KM, 2)
#define DVR_B6(L, D) DVR_B3(L, D, 16) DVR_B3(L, D, 64)
    DVR_B6(DVR_PLANAR, DVR_F32)
    DVR_B6(DVR_PLANAR, DVR_F16)
    DVR_B6(DVR_INTERLEAVED, DVR_F32)
    DVR_B6(DVR_INTERLEAVED, DVR_F16)
    DVR_B6(DVR_SPLIT, DVR_F32)
    DVR_B6(DVR_SPLIT, DVR_F16)
    DVR_B6(DVR_QUAD, DVR_F32)
    DVR_B6(DVR_QUAD, DVR_F16)
#undef DVR_B6
#undef DVR_B3
#undef DVR_B
    return hipErrorInvalidValue;
}

}  // namespace dvr

using namespace dvr;
using namespace dvr::host;

struct dvr_batch {
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> allocs;
    unsigned *d_err = nullptr;
    dvr_tune tune;
};

static void plan_free(dvr_batch *p)
{
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->stream) hipStreamDestroy(p->stream);
    for (void *a : p->allocs) hipFree(a);
    delete p;
}

static dvr_tune default_tune()
{
    dvr_tune t;
    t.wg_per_cu = 4;
    t.xy_tile = 0;
    // long z runs: every item ends with a device-scope release, which writes the XCD's L2 back; 32
    // slices per item took the 64-volume feature phase from 27.8 to 12.0 ms (4 slices per item)
    t.xy_zrun = 32;
    t.z_chunk = 8;
    t.ray_tile = 0;
    return t;
}

static dvr_status check_tune(const dvr_tune &t)
{
    if (t.wg_per_cu < 1 || t.wg_per_cu > 8) return fail(DVR_E_INVALID_ARG, "tune.wg_per_cu must be in [1, 8]");
    if (t.xy_tile < 0 || t.xy_tile > 2) return fail(DVR_E_INVALID_ARG, "tune.xy_tile must be 0, 1 or 2");
    if (t.xy_zrun < 1 || t.xy_zrun > 32) return fail(DVR_E_INVALID_ARG, "tune.xy_zrun must be in [1, 32]");
    if (t.z_chunk < 1 || t.z_chunk > 64) return fail(DVR_E_INVALID_ARG, "tune.z_chunk must be in [1, 64]");
    if (t.ray_tile < 0 || t.ray_tile > 2) return fail(DVR_E_INVALID_ARG, "tune.ray_tile must be 0, 1 or 2");
    return DVR_OK;
}

static const int kTXs[3] = {64, 32, 128}, kTYs[3] = {8, 16, 4};

extern "C" dvr_status dvr_batch_create(const dvr_batch_desc *d, dvr_batch **plan_out)
{
    if (!d || !plan_out) return fail(DVR_E_NULL, "desc and plan must be non-NULL");
    *plan_out = nullptr;
    if (d->nvol < 1 || !d->vols) return fail(DVR_E_INVALID_ARG, "need at least one volume");
    if (d->nview < 0 || (d->nview > 0 && !d->views)) return fail(DVR_E_INVALID_ARG, "bad view array");
    const dvr_tune tune = d->tune ? *d->tune : default_tune();
    dvr_status s = check_tune(tune);
    if (s) return s;
    const dvr_feature_params &fp = d->fp;
    if (!(fp.c > 0.f)) return fail(DVR_E_UNSUPPORTED, "batched launches need an explicit Frangi c > 0");
    const int ns = fp.nsigma;
    if ((int64_t)d->nvol * (ns > 0 ? ns : 1) > kMaxVolScale)
        return fail(DVR_E_INVALID_ARG, "volumes x scales must not exceed %d", kMaxVolScale);
    const int layout = d->vols[0].feat.layout, fdt = d->vols[0].feat.dtype;
    const int TX = kTXs[tune.xy_tile], TY = kTYs[tune.xy_tile];

    std::vector<BVol> vols(d->nvol);
    std::vector<ScaleTaps> taps((size_t)d->nvol * (ns > 0 ? ns : 1));
    std::vector<unsigned> nz_items((size_t)d->nvol * ns, 0u), nxy_items((size_t)d->nvol * ns, 0u);
    size_t lds_floats = 0;
    size_t ws_total = 0;
    for (int v = 0; v < d->nvol; ++v) {
        const dvr_batch_volume &bv = d->vols[v];
        if ((s = check_grid(&bv.grid))) return fail(s, "volume %d: %s", v, g_err.c_str());
        if ((s = check_fparams(&bv.grid, &fp))) return fail(s, "volume %d: %s", v, g_err.c_str());
        if ((s = check_feat_buf(&bv.feat, true))) return fail(s, "volume %d: %s", v, g_err.c_str());
        if (bv.feat.layout != layout || bv.feat.dtype != fdt)
            return fail(DVR_E_UNSUPPORTED, "all volumes must share the feature dtype and layout");
        if (bv.vol_dtype != fdt) return fail(DVR_E_UNSUPPORTED, "volume %d: vol dtype must equal the feature dtype", v);
        if (!bv.vol || !aligned16(bv.vol)) return fail(bv.vol ? DVR_E_ALIGN : DVR_E_NULL, "volume %d: bad vol pointer", v);
        const double h[3] = {bv.grid.hx, bv.grid.hy, bv.grid.hz};
        BVol &B = vols[v];
        B.vol = bv.vol;
        B.grad = bv.feat.grad;
        B.kappa = bv.feat.kappa;
        B.ves = bv.feat.ves;
        B.gmax = bv.feat.gmax;
        B.iquad = bv.feat.iquad;
        B.vtmp = nullptr;
        B.n[0] = bv.grid.nx;
        B.n[1] = bv.grid.ny;
        B.n[2] = bv.grid.nz;
        B.tiles_x = (bv.grid.nx + TX - 1) / TX;
        for (int a = 0; a < 3; ++a) B.inv2h[a] = (float)(1.0 / (2.0 * h[a]));
        const float hf[3] = {bv.grid.hx, bv.grid.hy, bv.grid.hz};
        B.grid.n[0] = bv.grid.nx;
        B.grid.n[1] = bv.grid.ny;
        B.grid.n[2] = bv.grid.nz;
        set_grid_steps(B.grid, hf, d->rp.step_vox);
        for (int sc = 0; sc < ns; ++sc) {
            ScaleTaps &t = taps[(size_t)v * ns + sc];
            for (int a = 0; a < 3; ++a) axis_taps((double)fp.sigma_mm[sc] / h[a], h[a], t.ax[a]);
            t.sigma2 = (float)((double)fp.sigma_mm[sc] * fp.sigma_mm[sc]);
            const size_t st = (size_t)3 * (TY + 2 * t.ax[1].R) * (TX + 2 * t.ax[0].R),
                         cw = (size_t)Compact<2>::kFloats;
            lds_floats = std::max(lds_floats, std::max(st, cw) + (size_t)6 * TY * (TX + 2 * t.ax[0].R));
        }
        ws_total += (size_t)ns * 12u * (size_t)nvox(&bv.grid);
        if (layout == DVR_QUAD) ws_total += ((size_t)4u * (size_t)nvox(&bv.grid) + 255u) & ~(size_t)255u;
    }
    if (lds_floats * 4 > 60 * 1024)
        return fail(DVR_E_UNSUPPORTED, "feature tile with halo needs %zu bytes of LDS (limit 60 KB)", lds_floats * 4);
    // views
    std::vector<BView> views(d->nview);
    for (int w = 0; w < d->nview; ++w) {
        const dvr_batch_view &bw = d->views[w];
        if (bw.volume < 0 || bw.volume >= d->nvol) return fail(DVR_E_INVALID_ARG, "view %d: bad volume index", w);
        const dvr_batch_volume &bv = d->vols[bw.volume];
        dvr::RenderArgs ra;
        dvr::KCam kc;
        if ((s = build_render_args(bv.vol, bv.vol_dtype, &bv.grid, &bv.feat, &d->tf, &d->rp, &bw.cam, 1, ra, &kc)))
            return fail(s, "view %d: %s", w, g_err.c_str());
        if (!bw.rgba || !aligned16(bw.rgba)) return fail(bw.rgba ? DVR_E_ALIGN : DVR_E_NULL, "view %d: bad rgba", w);
        BView &V = views[w];
        V.cam = kc;
        V.vol = bw.volume;
        V.W = bw.cam.width;
        V.H = bw.cam.height;
        V.tiles_x = (V.W + 15) / 16;
        V.rgba = bw.rgba;
        V.T_last = bw.T_last;
        V.k_last = bw.T_last ? bw.k_last : nullptr;
    }
    // work items in queue order: every Z item, then XY by scale, then rays
    std::vector<BItem> items;
    for (int v = 0; v < d->nvol; ++v)
        for (int sc = 0; sc < ns; ++sc)
            for (int z = 0; z < vols[v].n[2]; z += tune.z_chunk) {
                items.push_back({IT_Z | (sc << 8), v, z, std::min(z + tune.z_chunk, vols[v].n[2])});
                nz_items[(size_t)v * ns + sc]++;
            }
    for (int sc = 0; sc < ns; ++sc)
        for (int v = 0; v < d->nvol; ++v) {
            const int tx = vols[v].tiles_x, ty = (vols[v].n[1] + TY - 1) / TY;
            for (int z = 0; z < vols[v].n[2]; z += tune.xy_zrun)
                for (int t = 0; t < tx * ty; ++t) {
                    items.push_back({IT_XY | (sc << 8), v, t, z});
                    nxy_items[(size_t)v * ns + sc]++;
                }
        }
    std::vector<unsigned> nq_items((size_t)d->nvol, 0u);
    if (layout == DVR_QUAD)
        for (int v = 0; v < d->nvol; ++v)
            for (int z = 0; z < vols[v].n[2]; z += tune.z_chunk) {
                items.push_back({IT_Q, v, z, std::min(z + tune.z_chunk, vols[v].n[2])});
                nq_items[v]++;
            }
    for (int w = 0; w < d->nview; ++w) {
        const int nt = views[w].tiles_x * ((views[w].H + 15) / 16);
        for (int t = 0; t < nt; ++t) items.push_back({IT_RAY, w, t, 0});
    }
    if (items.size() > 0x7fffffffu) return fail(DVR_E_INVALID_ARG, "too many work items");

    dvr_batch *P = new (std::nothrow) dvr_batch();
    if (!P) return fail(DVR_E_NOMEM, "host allocation");
    P->tune = tune;
    auto dalloc = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) return nullptr;
        P->allocs.push_back(p);
        return p;
    };
    const int nvs = d->nvol * ns;
    BItem *d_items = (BItem *)dalloc(sizeof(BItem) * items.size());
    BVol *d_vols = (BVol *)dalloc(sizeof(BVol) * vols.size());
    BView *d_views = (BView *)dalloc(sizeof(BView) * std::max<size_t>(views.size(), 1));
    ScaleTaps *d_taps = (ScaleTaps *)dalloc(sizeof(ScaleTaps) * taps.size());
    unsigned *d_ctr = (unsigned *)dalloc(sizeof(unsigned) * (size_t)(2 + 5 * nvs + 2 * d->nvol));
    float *d_ws = (float *)dalloc(ws_total);
    if (!d_items || !d_vols || !d_views || !d_taps || !d_ctr || !d_ws) {
        plan_free(P);
        return fail(DVR_E_DEVICE, "device allocation of %zu bytes of workspace failed", ws_total);
    }
    size_t off = 0;
    for (int v = 0; v < d->nvol; ++v) {
        vols[v].ws = d_ws + off / 4;
        off += (size_t)ns * 12u * (size_t)nvox(&d->vols[v].grid);
        if (layout == DVR_QUAD) {
            vols[v].vtmp = d_ws + off / 4;
            off += ((size_t)4u * (size_t)nvox(&d->vols[v].grid) + 255u) & ~(size_t)255u;
        }
    }
    BatchArgs A;
    memset(&A, 0, sizeof A);
    A.items = (uint64_t)(uintptr_t)d_items;
    A.nitems = (int32_t)items.size();
    A.ns = ns;
    A.zrun = tune.xy_zrun;
    A.ray_tile = tune.ray_tile;
    A.vols = (uint64_t)(uintptr_t)d_vols;
    A.views = (uint64_t)(uintptr_t)d_views;
    A.taps = (uint64_t)(uintptr_t)d_taps;
    A.head = d_ctr;
    A.err = d_ctr + 1;
    A.zdone = d_ctr + 2;
    A.xydone = d_ctr + 2 + nvs;
    unsigned *d_nz = d_ctr + 2 + 2 * nvs, *d_nxy = d_ctr + 2 + 3 * nvs;
    A.nz_items = d_nz;
    A.nxy_items = d_nxy;
    unsigned *d_need = d_ctr + 2 + 4 * nvs;
    A.ray_need = d_need;
    A.qdone = d_ctr + 2 + 5 * nvs;
    unsigned *d_nq = d_ctr + 2 + 5 * nvs + d->nvol;
    A.nq_items = d_nq;
    A.max_spin = kMaxSpin;
    // Test hook (DVR_BATCH_TEST_TIMEOUT=1): the rays of volume 0 wait for one feature item more than
    // exist, with a short bound, so the launch exercises the timeout path and still exits normally.
    std::vector<unsigned> need(nxy_items);
    if (getenv("DVR_BATCH_TEST_TIMEOUT") && atoi(getenv("DVR_BATCH_TEST_TIMEOUT")) == 1) {
        need[(size_t)ns - 1] += 1;
        A.max_spin = 2000;
    }
    A.c = fp.c;
    A.inv2a2 = (float)(1.0 / (2.0 * (double)fp.alpha * fp.alpha));
    A.inv2b2 = (float)(1.0 / (2.0 * (double)fp.beta * fp.beta));
    A.tau = fp.eig_gap_fp64;
    {
        dvr::RenderArgs ra;
        dvr::KCam kc;
        const dvr_batch_volume &bv = d->vols[0];
        dvr_camera dummy;
        memset(&dummy, 0, sizeof dummy);
        dummy.width = dummy.height = 1;
        dummy.d0[2] = 1.f;
        if ((s = build_render_args(bv.vol, bv.vol_dtype, &bv.grid, &bv.feat, &d->tf, &d->rp, &dummy, 1, ra, &kc))) {
            plan_free(P);
            return s;
        }
        A.tf = ra.tf;
        A.rp = ra.rp;
    }
    P->d_err = A.err;
    hipError_t e = hipMemcpy(d_items, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_vols, vols.data(), sizeof(BVol) * vols.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !views.empty())
        e = hipMemcpy(d_views, views.data(), sizeof(BView) * views.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_taps, taps.data(), sizeof(ScaleTaps) * taps.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_nz, nz_items.data(), sizeof(unsigned) * nvs, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_nxy, nxy_items.data(), sizeof(unsigned) * nvs, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_need, need.data(), sizeof(unsigned) * nvs, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_nq, nq_items.data(), sizeof(unsigned) * d->nvol, hipMemcpyHostToDevice);
    int dev = 0, ncu = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        plan_free(P);
        return dev_fail(e, "batch plan setup");
    }
    const unsigned grid = (unsigned)(ncu * tune.wg_per_cu);
    const size_t lds = lds_floats * 4;
    e = hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(256), 0, P->stream, A, nvs, d->nvol);
        hipError_t e1 = hipGetLastError();
        hipError_t e2 = launch_batch_kernel(A, layout, fdt, d->tf.K, tune.xy_tile, grid, lds, P->stream);
        hipError_t e3 = hipStreamEndCapture(P->stream, &P->graph);
        e = e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        plan_free(P);
        return dev_fail(e, "batch graph capture");
    }
    *plan_out = P;
    return DVR_OK;
}

extern "C" dvr_status dvr_batch_launch(dvr_batch *plan, hipStream_t stream)
{
    if (!plan || !plan->exec) return fail(DVR_E_NULL, "plan is NULL");
    const hipError_t e = hipGraphLaunch(plan->exec, stream);
    return e == hipSuccess ? DVR_OK : dev_fail(e, "batch graph launch");
}

extern "C" dvr_status dvr_batch_check(dvr_batch *plan, hipStream_t stream)
{
    if (!plan) return fail(DVR_E_NULL, "plan is NULL");
    hipError_t e = hipStreamSynchronize(stream);
    unsigned err = 0;
    if (e == hipSuccess) e = hipMemcpy(&err, plan->d_err, sizeof err, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail(e, "batch check");
    if (err) return fail(DVR_E_TIMEOUT, "a dependency wait of the batched launch expired");
    return DVR_OK;
}

extern "C" dvr_status dvr_batch_destroy(dvr_batch *plan)
{
    if (!plan) return DVR_OK;
    hipStreamSynchronize(plan->stream);
    plan_free(plan);
    return DVR_OK;
}

// ------------------------------------------------------------------------------------------------
// autotuner: time candidate tile shapes on the batch itself; JSON cache keyed by shape class

static std::string tune_key(const dvr_batch_desc *d)
{
    double vox = 0, pix = 0;
    for (int v = 0; v < d->nvol; ++v) vox += (double)nvox(&d->vols[v].grid);
    for (int w = 0; w < d->nview; ++w) pix += (double)d->views[w].cam.width * d->views[w].cam.height;
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    std::ostringstream k;
    k << arch.substr(0, arch.find(':')) << "|dt" << d->vols[0].feat.dtype << "|lay" << d->vols[0].feat.layout << "|ns"
      << d->fp.nsigma << "|K" << (d->tf.K <= 16 ? 16 : 64) << "|vox2^" << (int)floor(log2(std::max(vox, 1.0)))
      << "|pix2^" << (int)floor(log2(std::max(pix, 1.0))) << "|nvol2^" << (int)floor(log2((double)d->nvol));
    return k.str();
}

static std::map<std::string, dvr_tune> read_cache(const char *path)
{
    std::map<std::string, dvr_tune> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // "key": [wg_per_cu, xy_tile, xy_zrun, z_chunk, ray_tile],
        const size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1), b0 = line.find('['), b1 = line.find(']');
        if (q0 == std::string::npos || q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos)
            continue;
        dvr_tune t;
        if (sscanf(line.c_str() + b0 + 1, "%d , %d , %d , %d , %d", &t.wg_per_cu, &t.xy_tile, &t.xy_zrun, &t.z_chunk,
                   &t.ray_tile) == 5 &&
            check_tune(t) == DVR_OK)
            m[line.substr(q0 + 1, q1 - q0 - 1)] = t;
    }
    return m;
}

static void write_cache(const char *path, const std::map<std::string, dvr_tune> &m)
{
    std::ofstream f(path);
    f << "{\n";
    size_t i = 0;
    for (const auto &kv : m) {
        const dvr_tune &t = kv.second;
        f << "  \"" << kv.first << "\": [" << t.wg_per_cu << ", " << t.xy_tile << ", " << t.xy_zrun << ", " << t.z_chunk
          << ", " << t.ray_tile << "]" << (++i < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
}

extern "C" dvr_status dvr_batch_autotune(const dvr_batch_desc *desc, const char *cache_path, dvr_tune *best)
{
    if (!desc || !best) return fail(DVR_E_NULL, "desc and best must be non-NULL");
    const std::string key = tune_key(desc);
    std::map<std::string, dvr_tune> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *best = it->second;
            return DVR_OK;
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(DVR_E_DEVICE, "event creation");
    dvr_status last = DVR_OK;
    // one candidate: build the plan, one warm replay, then two timed replays
    auto time_tune = [&](const dvr_tune &t) -> float {
        dvr_batch_desc d = *desc;
        d.tune = &t;
        dvr_batch *p = nullptr;
        dvr_status s = dvr_batch_create(&d, &p);
        if (s != DVR_OK) {
            last = s;
            return INFINITY;  // e.g. a tile whose halo does not fit in LDS
        }
        float ms = INFINITY;
        if (dvr_batch_launch(p, p->stream) == DVR_OK && dvr_batch_check(p, p->stream) == DVR_OK) {
            hipEventRecord(e0, p->stream);
            dvr_batch_launch(p, p->stream);
            dvr_batch_launch(p, p->stream);
            hipEventRecord(e1, p->stream);
            if (dvr_batch_check(p, p->stream) == DVR_OK) {
                hipEventElapsedTime(&ms, e0, e1);
                ms *= 0.5f;
            }
        }
        dvr_batch_destroy(p);
        return ms;
    };
    // coordinate descent from the defaults, two sweeps: each field in turn over its candidate values
    // with the others at the best so far (the fields interact weakly: the feature items use xy_tile,
    // xy_zrun and z_chunk, the ray items ray_tile, and wg_per_cu sets the occupancy of both)
    const std::vector<int> vals[5] = {{2, 3, 4, 6, 8}, {0, 1, 2}, {8, 16, 32}, {4, 8, 16, 32}, {0, 1, 2}};
    auto field = [](dvr_tune &t, int f) -> int & {
        return f == 0 ? t.wg_per_cu : (f == 1 ? t.xy_tile : (f == 2 ? t.xy_zrun : (f == 3 ? t.z_chunk : t.ray_tile)));
    };
    std::map<std::vector<int>, float> seen;
    auto key_of = [](const dvr_tune &t) {
        return std::vector<int>{t.wg_per_cu, t.xy_tile, t.xy_zrun, t.z_chunk, t.ray_tile};
    };
    dvr_tune best_t = default_tune();
    float best_ms = time_tune(best_t);
    seen[key_of(best_t)] = best_ms;
    for (int sweep = 0; sweep < 2; ++sweep)
        for (int f = 0; f < 5; ++f)
            for (int v : vals[f]) {
                dvr_tune t = best_t;
                field(t, f) = v;
                const auto k = key_of(t);
                if (seen.count(k)) continue;
                const float ms = time_tune(t);
                seen[k] = ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    best_t = t;
                }
            }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!isfinite(best_ms)) return last != DVR_OK ? last : fail(DVR_E_DEVICE, "no candidate tune ran");
    *best = best_t;
    if (cache_path) {
        cache[key] = best_t;
        write_cache(cache_path, cache);
    }
    return DVR_OK;
}
