// Front-to-back raymarcher (Sec. 2.4 Eq. 4-6) and its adjoint, for gfx950.
//
// Mapping: one lane per ray; a wave covers an 8 x 8 pixel tile and a 256-lane workgroup a
// 16 x 16 tile, so the lanes of a wave gather neighbouring voxels.  A lane leaves the sample loop
// when its ray ends or terminates early; the wave leaves when every lane has (the exec mask of the
// loop empties), which is the wave-ballot early termination.
//
// Ray geometry.  The camera ray, the slab clip against [0,(n-1)h] and the segment count are
// computed once per ray in double-float FP32 (pairs of FP32 numbers, ~48 bits, from error-free
// transforms), following the FP64 definition's steps, so N and the segment lengths agree with it
// (plain FP32 here moves the head's perspective images by ~6e-4).  Sample positions in voxel units
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
#include "render_dev.hpp"

namespace dvr {

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

// MORTON: the 64 lanes of a wave take their 8 x 8 pixels in Morton order (lane bits x0 y0 x1 y1 x2
// y2), so each quad of lanes is a 2 x 2 pixel block; otherwise row-major.
template <bool MORTON = false>
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
    uint32_t lx, ly;
    if (MORTON) {
        lx = (lane & 1u) | ((lane >> 1) & 2u) | ((lane >> 2) & 4u);
        ly = ((lane >> 1) & 1u) | ((lane >> 2) & 2u) | ((lane >> 3) & 4u);
    } else {
        lx = lane & 7u;
        ly = lane >> 3;
    }
    pi = (int)(tx * 16u + (wv & 1u) * 8u + lx);
    pj = (int)(ty * 16u + (wv >> 1) * 8u + ly);
    valid = cam < (uint32_t)L.ncam && pi < L.W && pj < L.H;
}

// The FP16 quad layout keeps a corner's six values packed in three registers (104 VGPRs, four waves
// per SIMD); held to five waves (96 VGPRs, a few spilled values) it runs 7 % faster on the head
// (0.296 against 0.318 ms per view).  The FP32 layouts and the other FP16 ones spill far more at
// five waves and are slower, so they keep the default.
template <int LAYOUT, int DT, int KMAX>
__global__ __launch_bounds__(256, (LAYOUT == DVR_QUAD && DT == DVR_F16) ? 5 : 1) void k_render(KFeat feat, KGrid g,
                                                                                            KTF tf, KRender rp,
                                                                                            KLaunch L)
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
    const RayOut o = march_fwd<LAYOUT, DT, KMAX>(feat, g, sh, kx, rp, invg, r);
    if (valid) {
        const size_t pix = ((size_t)(L.cam_base + cam) * L.H + pj) * L.W + pi;
        reinterpret_cast<float4 *>(L.out)[pix] = make_float4(o.C0, o.C1, o.C2, o.A);
        if (L.T_last) L.T_last[pix] = o.Tprev;
        if (L.k_last) L.k_last[pix] = o.last;
    }
    if (L.counters) count_samples<4>(L.counters, o.last, o.shaded);
}

// Gather ceiling of k_render (dvr_render_gather): the same rays, samples and loads, without the
// optics; sink[pixel] keeps the loads live, counters count the samples walked and those whose
// feature corners were fetched (equal to the forward pass's counts by construction).
template <int LAYOUT, int DT, int KMAX>
__global__ __launch_bounds__(256) void k_render_gather(KFeat feat, KGrid g, KTF tf, KRender rp, KLaunch L)
{
    __shared__ TFShared<KMAX> sh;
    float kx[KMAX];
    tf_load<KMAX>(sh, kx, tf);
    __syncthreads();
    uint32_t cam;
    int pi, pj;
    bool valid;
    pixel_of(L, cam, pi, pj, valid);
    const size_t pix = valid ? ((size_t)(L.cam_base + cam) * L.H + pj) * L.W + pi : 0;
    const int kl = valid ? L.k_last[pix] : -1;
    RayGeo r;
    r.N = 0;
    if (kl >= 0) r = ray_setup(load_cam(L, cam), pi, pj, g);
    const RayOut o = march_fwd<LAYOUT, DT, KMAX, true>(feat, g, sh, kx, rp, 0.f, r, kl);
    if (valid) L.out[pix] = o.C0;
    if (L.counters) count_samples<4>(L.counters, o.last, o.shaded);
}

template <int LAYOUT, int DT, int KMAX, bool FG>
__global__ __launch_bounds__(256) void k_render_bwd(KFeat feat, KGrid g, KTF tf, KRender rp, KLaunch L)
{
    __shared__ TFShared<KMAX> sh;
    constexpr int kCopies = tf_copies(KMAX);
    __shared__ double tfa[KMAX * 4 * kCopies];
    using Win = std::conditional_t<FG, DWinF, DWin>;
    __shared__ double win[4][Win::kEntries];  // one accumulation window per wave
    // the ray first, before anything else is live: set up after the TF load (with the knots held in
    // registers across it) the kernel took 182 VGPRs instead of 166, one wave per SIMD fewer
    uint32_t cam;
    int pi, pj;
    bool valid;
    pixel_of<true>(L, cam, pi, pj, valid);
    const size_t pix = valid ? ((size_t)(L.cam_base + cam) * L.H + pj) * L.W + pi : 0;
    const int kl = valid ? L.k_last[pix] : -1;
    RayGeo r;
    r.N = 0;
    if (kl >= 0) r = ray_setup(load_cam(L, cam), pi, pj, g);
    float kx[KMAX];
    tf_load<KMAX>(sh, kx, tf);
    for (int p = threadIdx.x; p < KMAX * 4 * kCopies; p += 256) tfa[p] = 0.0;
    double *wwin = win[threadIdx.x >> 6];
    if (FG || L.dvol)
        for (int p = threadIdx.x & 63; p < Win::kEntries; p += 64) wwin[p] = 0.0;
    __syncthreads();
    const int K = tf.K;
    const float gm = *feat.gmax;
    const float invg = gm > 0.f ? 1.f / gm : 0.f;
    float4 gr = make_float4(0.f, 0.f, 0.f, 0.f);
    float Tl = 0.f;
    if (kl >= 0) {
        gr = reinterpret_cast<const float4 *>(L.dout)[pix];
        Tl = L.T_last[pix];
    }
    // every lane of the wave takes part (the dL/dI window is managed wave-wide)
    float gmb = 0.f;
    march_bwd<LAYOUT, DT, KMAX, FG>(feat, g, sh, kx, rp, invg, r, kl, Tl, gr, K, tfa + (threadIdx.x % kCopies), L.dvol,
                                    wwin, L.dfeat, gmb);
    if constexpr (FG) {
        for (int o = 32; o > 0; o >>= 1) gmb += __shfl_xor(gmb, o, 64);
        if ((threadIdx.x & 63) == 0 && gmb != 0.f) atomicAdd(L.dgmax, gmb);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < K * 4; p += 256) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kCopies; ++j) acc += tfa[p * kCopies + j];
        if (acc != 0.0) atomicAdd(L.dtf + p, (float)acc);
    }
}

// ------------------------------------------------------------------------------------------------
enum { kFwd = 0, kBwd = 1, kGather = 2 };

template <int LAYOUT, int DT, int KMAX>
static hipError_t launch_fwd_t(const KFeat &f, const KGrid &g, const KTF &tf, const KRender &rp, const KLaunch &L,
                               uint32_t blocks, hipStream_t st, int mode)
{
    const bool bwd = mode == kBwd;
    if (mode == kGather)
        hipLaunchKernelGGL((k_render_gather<LAYOUT, DT, KMAX>), dim3(blocks), dim3(256), 0, st, f, g, tf, rp, L);
    else if (bwd && L.dfeat)
        hipLaunchKernelGGL((k_render_bwd<LAYOUT, DT, KMAX, true>), dim3(blocks), dim3(256), 0, st, f, g, tf, rp, L);
    else if (bwd)
        hipLaunchKernelGGL((k_render_bwd<LAYOUT, DT, KMAX, false>), dim3(blocks), dim3(256), 0, st, f, g, tf, rp, L);
    else
        hipLaunchKernelGGL((k_render<LAYOUT, DT, KMAX>), dim3(blocks), dim3(256), 0, st, f, g, tf, rp, L);
    return hipGetLastError();
}

template <int LAYOUT, int DT>
static hipError_t launch_k(const KFeat &f, const KGrid &g, const KTF &tf, const KRender &rp, const KLaunch &L,
                           uint32_t blocks, hipStream_t st, int mode)
{
    if (tf.K <= 8) return launch_fwd_t<LAYOUT, DT, 8>(f, g, tf, rp, L, blocks, st, mode);
    if (tf.K <= 16) return launch_fwd_t<LAYOUT, DT, 16>(f, g, tf, rp, L, blocks, st, mode);
    return launch_fwd_t<LAYOUT, DT, 64>(f, g, tf, rp, L, blocks, st, mode);
}

static hipError_t launch_any(const RenderArgs &a, hipStream_t st, int mode)
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
        if (lay == DVR_PLANAR && dt == DVR_F32) e = launch_k<DVR_PLANAR, DVR_F32>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, mode);
        else if (lay == DVR_PLANAR && dt == DVR_F16) e = launch_k<DVR_PLANAR, DVR_F16>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, mode);
        else if (lay == DVR_INTERLEAVED && dt == DVR_F32) e = launch_k<DVR_INTERLEAVED, DVR_F32>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, mode);
        else if (lay == DVR_INTERLEAVED && dt == DVR_F16) e = launch_k<DVR_INTERLEAVED, DVR_F16>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, mode);
        else if (lay == DVR_SPLIT && dt == DVR_F32) e = launch_k<DVR_SPLIT, DVR_F32>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, mode);
        else if (lay == DVR_SPLIT && dt == DVR_F16) e = launch_k<DVR_SPLIT, DVR_F16>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, mode);
        else if (lay == DVR_QUAD && dt == DVR_F32) e = launch_k<DVR_QUAD, DVR_F32>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, mode);
        else if (lay == DVR_QUAD && dt == DVR_F16) e = launch_k<DVR_QUAD, DVR_F16>(a.feat, a.grid, a.tf, a.rp, L, blocks, st, mode);
        else e = hipErrorInvalidValue;
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Empty-brick bits for one TF: brick i is empty when brick_empty() holds for its (min, max); a wave
// covers 64 bricks and writes the two 32-bit words of its ballot.
__global__ __launch_bounds__(256) void k_brick_mask(const float *__restrict__ bricks, int nb, KTF tf)
{
    __shared__ TFShared<64> sh;
    float kx[64];
    tf_load<64>(sh, kx, tf);
    __syncthreads();
    const int i = (int)(blockIdx.x * 256u + threadIdx.x);
    bool e = false;
    if (i < nb) e = brick_empty<64>(sh, kx, bricks[2 * i], bricks[2 * i + 1]);
    const uint64_t bal = __ballot(e);
    const int w0 = (int)(blockIdx.x * 256u + (threadIdx.x & ~63u)) / 32;  // first word of this wave
    const int nw = (nb + 31) / 32;
    uint32_t *mask = reinterpret_cast<uint32_t *>(const_cast<float *>(bricks) + 2 * nb);
    const int lane = threadIdx.x & 63;
    if (lane == 0 && w0 < nw) mask[w0] = (uint32_t)bal;
    if (lane == 1 && w0 + 1 < nw) mask[w0 + 1] = (uint32_t)(bal >> 32);
}

hipError_t launch_brick_mask(const RenderArgs &a, hipStream_t st)
{
    const int nb = a.feat.nb[0] * a.feat.nb[1] * a.feat.nb[2];
    hipLaunchKernelGGL(k_brick_mask, dim3((nb + 255) / 256), dim3(256), 0, st, a.feat.bricks, nb, a.tf);
    return hipGetLastError();
}

hipError_t launch_render(const RenderArgs &a, hipStream_t st)
{
    if (a.feat.bricks) {
        const hipError_t e = launch_brick_mask(a, st);
        if (e != hipSuccess) return e;
    }
    return launch_any(a, st, kFwd);
}
hipError_t launch_render_backward(const RenderArgs &a, hipStream_t st) { return launch_any(a, st, kBwd); }
hipError_t launch_render_gather(const RenderArgs &a, hipStream_t st)
{
    if (a.feat.bricks) {
        const hipError_t e = launch_brick_mask(a, st);
        if (e != hipSuccess) return e;
    }
    return launch_any(a, st, kGather);
}

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
