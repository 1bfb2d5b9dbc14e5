// Feature pass for gfx950: central-difference gradient (Sec. 2.3 Eq. 2), Gaussian-scale Hessian
// (Sec. 1 "multi-scale Hessian analysis"; Sec. 2.3), its eigenvalues, directional curvature
// (Sec. 2.3 Eq. 3) and Frangi vesselness (Sec. 1 "vesselness measures").
//
// The Hessian of the Gaussian-smoothed volume by clamped central differences is a linear
// operator on I; it is applied here as six separable derivative-of-Gaussian filters
//     Hxx = D2x Gy Gz, Hyy = Gx D2y Gz, Hzz = Gx Gy D2z,
//     Hxy = D1x D1y Gz, Hxz = D1x Gy D1z, Hyz = Gx D1y D1z,
// with exact one-sided variants on the first and last voxel of each axis.  Smoothing first and
// differencing afterwards in FP32 cancels away ~1e-5 of the Hessian's range; the combined taps
// keep it at a few 1e-7.
//
// Two kernels per scale:
//   k_zpass   one voxel per lane: (Gz, D1z, D2z) of I along z -> workspace, 12 B/voxel;
//   k_xypass  one 64 x 8 (x, y) tile of one z slice per 256-lane workgroup: the three z-filtered
//             fields of the tile plus halo are staged in LDS, the y filters produce six fields
//             (kept in LDS), the x filters give H per voxel, and the epilogue computes the
//             gradient (first scale), |g|_max, k, the eigenvalues of sigma^2 H and V.
#include <math.h>

#include "common.hpp"
#include "features_dev.hpp"

namespace dvr {

// z pass: (Gz, D1z, D2z) of I for every voxel.  The grid covers each z plane in 256-voxel runs
// (blockIdx.x) and the planes (blockIdx.y), so lanes read consecutive x and the boundary class of
// z is uniform per workgroup.
template <int DT>
__global__ __launch_bounds__(256) void k_zpass(const void *__restrict__ vol, float *__restrict__ ws, int nx, int ny,
                                               int nz, AxisTaps tz)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= plane) return;
    zpass_voxel<DT>(vol, ws, nx, ny, nz, tz, e, (int)blockIdx.y);
}

// Fixed-radius z pass: a lane takes TZ consecutive voxels of one (x, y) column and keeps the
// TZ + 2R inputs it needs in registers, so each input is loaded (TZ + 2R) / TZ times instead of
// 2R + 1 times.
template <int DT, int R, int TZ>
__global__ __launch_bounds__(256) void k_zpass_r(const void *__restrict__ vol, float *__restrict__ ws, int nx, int ny,
                                                 int nz, AxisTaps tz)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= plane) return;
    const int z0 = (int)blockIdx.y * TZ;
    const uint32_t N = plane * (uint32_t)nz;
    const Buf b = make_buf(vol, N * ElemSize<DT>::v);
    float col[TZ + 2 * R];
#pragma unroll
    for (int i = 0; i < TZ + 2 * R; ++i) col[i] = ldv<DT>(b, (uint32_t)clampi(z0 - R + i, 0, nz - 1) * plane + e);
#pragma unroll
    for (int k = 0; k < TZ; ++k) {
        const int z = z0 + k;
        if (z >= nz) break;
        const int cls = (z == 0) ? 1 : (z == nz - 1 ? 2 : 0);
        const Line3 o = r3<R>(tz, cls, [&](int m) { return col[k + R + m]; });
        const uint32_t i = (uint32_t)z * plane + e;
        ws[i] = o.g;
        ws[N + i] = o.d1;
        ws[2u * N + i] = o.d2;
    }
}

constexpr int kTZ = 16;  // slices per lane of the fixed-radius z pass (8: 2-16 % slower on the head)

template <int DT, int R>
static hipError_t launch_z_r(const void *vol, float *ws, const dvr_grid &g, const AxisTaps &tz, hipStream_t st)
{
    if constexpr (R > 10) {
        return hipErrorInvalidValue;
    } else {
        if (tz.R != R) return launch_z_r<DT, R + 1>(vol, ws, g, tz, st);
        const uint32_t plane = (uint32_t)g.nx * (uint32_t)g.ny;
        dim3 grid((plane + 255) / 256, (g.nz + kTZ - 1) / kTZ);
        hipLaunchKernelGGL((k_zpass_r<DT, R, kTZ>), grid, dim3(256), 0, st, vol, ws, g.nx, g.ny, g.nz, tz);
        return hipGetLastError();
    }
}

constexpr int TX = 64, TY = 8;

template <int DT, int OUT_DT, int LAYOUT>
__global__ __launch_bounds__(NT) void k_xypass(XYArgs a, ScaleTaps taps)
{
    extern __shared__ float lds[];
    float vmax = xy_tile<DT, OUT_DT, LAYOUT, TX, TY>(a, taps, blockIdx.x * TX, blockIdx.y * TY, blockIdx.z, lds);
    if (a.fro_pass || a.first) {
        vmax = wave_max(vmax);
        if ((threadIdx.x & 63) == 0) atomic_max_pos(a.fro_pass ? a.fro : a.gmax, vmax);
    }
}

// Fixed-radius variant (x and y stencil radius R, equal) for the layouts the workloads use: one
// workgroup per (x, y) tile and run of kZRun z slices, each slice's loads in flight while the previous
// slice is computed.
constexpr int kZRun = 1;

// One slice per workgroup, the y-filtered fields written over the staged ones (one LDS area of
// max(NF, NFY) floats): 25 instead of 41 KB at radius 10, six workgroups a CU instead of three.  At
// radii 6-9 the compiler otherwise takes 103-128 VGPRs (four waves per SIMD) for the y filters'
// registers; held to six waves it needs 57-64, without spills (radius 7: 0.142 -> 0.127 ms on the head).
template <int DT, int OUT_DT, int LAYOUT, int R>
__global__ __launch_bounds__(NT, (R >= 6 && R <= 9) ? 6 : 1) void k_xypass_r(XYArgs a, ScaleTaps taps)
{
    using T = XYTileR<R, TX, TY>;
    using S = XYSlab<DT, OUT_DT, LAYOUT, R, TX, TY>;
    __shared__ float F[T::NF > T::NFY ? T::NF : T::NFY];
    float vmax;
    if constexpr (kZRun == 1) {
        S s(a, taps, F, F, blockIdx.x * TX, blockIdx.y * TY);
        const int z = blockIdx.z;
        s.load(z);
        s.store();
        __syncthreads();
        vmax = s.compute(z, s.In, s.Vp);
    } else {
        const int z0 = blockIdx.z * kZRun, z1 = min(z0 + kZRun, a.nz);
        vmax = xy_run_r<DT, OUT_DT, LAYOUT, R, TX, TY>(a, taps, blockIdx.x * TX, blockIdx.y * TY, z0, z1, F, F);
    }
    if (a.fro_pass || a.first) {
        vmax = wave_max(vmax);
        if ((threadIdx.x & 63) == 0) atomic_max_pos(a.fro_pass ? a.fro : a.gmax, vmax);
    }
}

constexpr int kRFastMin = 2, kRFastMax = 10;

template <int DT, int OUT_DT, int LAYOUT, int R>
static hipError_t launch_xy_r(const XYArgs &a, const ScaleTaps &taps, hipStream_t st)
{
    if constexpr (R > kRFastMax) {
        return hipErrorInvalidValue;
    } else {
        if (taps.ax[0].R != R) return launch_xy_r<DT, OUT_DT, LAYOUT, R + 1>(a, taps, st);
        dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY, (a.nz + kZRun - 1) / kZRun);
        hipLaunchKernelGGL((k_xypass_r<DT, OUT_DT, LAYOUT, R>), grid, dim3(NT), 0, st, a, taps);
        return hipGetLastError();
    }
}

// Brick table: one lane per brick (consecutive lanes on consecutive bricks along x), each reading its
// (DVR_BRICK + 1)^3 voxels.  SRC: 0 F32 volume, 1 F16 volume, 2 F32 records (I at stride 8), 3 F16
// records.
template <int SRC>
__global__ __launch_bounds__(256) void k_bricks(const void *__restrict__ src, float2 *__restrict__ out, int nx, int ny,
                                                int nz, int nbx, int nby, int nbz)
{
    const int i = (int)(blockIdx.x * 256u + threadIdx.x);
    if (i >= nbx * nby * nbz) return;
    const int bx = i % nbx, by = (i / nbx) % nby, bz = i / (nbx * nby);
    const int x0 = bx * DVR_BRICK, y0 = by * DVR_BRICK, z0 = bz * DVR_BRICK;
    const int x1 = min(x0 + DVR_BRICK, nx - 1), y1 = min(y0 + DVR_BRICK, ny - 1), z1 = min(z0 + DVR_BRICK, nz - 1);
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    float mn = INFINITY, mx = -INFINITY;
    for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const uint32_t v = (uint32_t)z * plane + (uint32_t)y * nx + x;
                float f;
                if constexpr (SRC == 0) f = reinterpret_cast<const float *>(src)[v];
                else if constexpr (SRC == 1) f = __half2float(reinterpret_cast<const __half *>(src)[v]);
                else if constexpr (SRC == 2) f = reinterpret_cast<const float *>(src)[8u * v];
                else f = __half2float(reinterpret_cast<const __half *>(src)[8u * v]);
                mn = fminf(mn, f);
                mx = fmaxf(mx, f);
            }
    out[i] = make_float2(mn, mx);
}

// One lane per voxel, x fastest: the four rows are read coalesced (mostly from L2), the quad is
// written as one 16- (F32) or 8-byte (F16) store.
template <typename T, typename T4>
__global__ void __launch_bounds__(256) k_quads(const T *__restrict__ src, T4 *__restrict__ dst, uint32_t nx,
                                               uint32_t ny, uint32_t nz)
{
    const uint32_t v = blockIdx.x * 256u + threadIdx.x;
    const uint32_t sz = nx * ny;
    if (v >= sz * nz) return;
    const uint32_t row = v / nx, y = row % ny, z = row / ny;
    const bool yi = y + 1u < ny, zi = z + 1u < nz;
    T4 q;
    q.x = src[v];
    q.y = yi ? src[v + nx] : T(0);
    q.z = zi ? src[v + sz] : T(0);
    q.w = (yi && zi) ? src[v + sz + nx] : T(0);
    dst[v] = q;
}

hipError_t launch_quads(const void *src, void *dst, const dvr_grid &g, int dtype, hipStream_t st)
{
    const uint32_t n = (uint32_t)g.nx * (uint32_t)g.ny * (uint32_t)g.nz;
    const dim3 grid((n + 255u) / 256u);
    if (dtype == DVR_F32)
        hipLaunchKernelGGL((k_quads<uint32_t, uint4>), grid, dim3(256), 0, st, static_cast<const uint32_t *>(src),
                           static_cast<uint4 *>(dst), (uint32_t)g.nx, (uint32_t)g.ny, (uint32_t)g.nz);
    else
        hipLaunchKernelGGL((k_quads<uint16_t, ushort4>), grid, dim3(256), 0, st, static_cast<const uint16_t *>(src),
                           static_cast<ushort4 *>(dst), (uint32_t)g.nx, (uint32_t)g.ny, (uint32_t)g.nz);
    return hipGetLastError();
}

hipError_t launch_bricks(const void *vol, int vol_dt, const dvr_grid &g, const dvr_features_buf &out, hipStream_t st)
{
    const int nbx = (g.nx - 1 + DVR_BRICK - 1) / DVR_BRICK, nby = (g.ny - 1 + DVR_BRICK - 1) / DVR_BRICK,
              nbz = (g.nz - 1 + DVR_BRICK - 1) / DVR_BRICK;
    const int nb = nbx * nby * nbz;
    dim3 grid((nb + 255) / 256);
    float2 *o = reinterpret_cast<float2 *>(out.bricks);
    // the records' I is the volume itself when the dtypes agree (read the contiguous volume then)
    if (out.layout == DVR_INTERLEAVED && out.dtype != vol_dt) {
        if (out.dtype == DVR_F32)
            hipLaunchKernelGGL(k_bricks<2>, grid, dim3(256), 0, st, out.grad, o, g.nx, g.ny, g.nz, nbx, nby, nbz);
        else
            hipLaunchKernelGGL(k_bricks<3>, grid, dim3(256), 0, st, out.grad, o, g.nx, g.ny, g.nz, nbx, nby, nbz);
    } else if (vol_dt == DVR_F32) {
        hipLaunchKernelGGL(k_bricks<0>, grid, dim3(256), 0, st, vol, o, g.nx, g.ny, g.nz, nbx, nby, nbz);
    } else {
        hipLaunchKernelGGL(k_bricks<1>, grid, dim3(256), 0, st, vol, o, g.nx, g.ny, g.nz, nbx, nby, nbz);
    }
    return hipGetLastError();
}

__global__ void k_init_scalars(float *gmax, float *fro)
{
    if (threadIdx.x == 0) {
        if (gmax) *gmax = 0.f;
        if (fro) *fro = 0.f;
    }
}

hipError_t launch_init_scalars(float *gmax, float *ws_scalars, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, st, gmax, ws_scalars);
    return hipGetLastError();
}

template <int DT, int OUT_DT, int LAYOUT>
static hipError_t launch_xy(const XYArgs &a, const ScaleTaps &taps, hipStream_t st)
{
    const size_t lds = sizeof(float) * xy_lds_floats<TX, TY>(taps.ax[0].R, taps.ax[1].R);
    dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY, a.nz);
    hipLaunchKernelGGL((k_xypass<DT, OUT_DT, LAYOUT>), grid, dim3(NT), lds, st, a, taps);
    return hipGetLastError();
}

static hipError_t launch_z_any(const void *vol, int vol_dt, const dvr_grid &g, const AxisTaps &tz, float *ws_fields,
                               hipStream_t st)
{
    if (tz.R >= 2 && tz.R <= 10)
        return (vol_dt == DVR_F32) ? launch_z_r<DVR_F32, 2>(vol, ws_fields, g, tz, st)
                                   : launch_z_r<DVR_F16, 2>(vol, ws_fields, g, tz, st);
    const uint32_t plane = (uint32_t)g.nx * (uint32_t)g.ny;
    dim3 zgrid((plane + 255) / 256, g.nz);
    if (vol_dt == DVR_F32)
        hipLaunchKernelGGL(k_zpass<DVR_F32>, zgrid, dim3(256), 0, st, vol, ws_fields, g.nx, g.ny, g.nz, tz);
    else
        hipLaunchKernelGGL(k_zpass<DVR_F16>, zgrid, dim3(256), 0, st, vol, ws_fields, g.nx, g.ny, g.nz, tz);
    return hipGetLastError();
}

hipError_t launch_hessian(const void *vol, int vol_dt, const dvr_grid &g, const ScaleTaps &taps, float *ws_fields,
                          float *H, hipStream_t st)
{
    hipError_t e = launch_z_any(vol, vol_dt, g, taps.ax[2], ws_fields, st);
    if (e != hipSuccess) return e;
    XYArgs a = {};
    a.ws = ws_fields;
    a.vol = vol;
    a.grad = H;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.first = 0;
    a.fro_pass = 0;
    const int R = taps.ax[0].R;
    if (R == taps.ax[1].R && R >= kRFastMin && R <= kRFastMax)
        return (vol_dt == DVR_F32) ? launch_xy_r<DVR_F32, DVR_F32, kHessianOut, kRFastMin>(a, taps, st)
                                   : launch_xy_r<DVR_F16, DVR_F32, kHessianOut, kRFastMin>(a, taps, st);
    if (vol_dt == DVR_F32) return launch_xy<DVR_F32, DVR_F32, kHessianOut>(a, taps, st);
    return launch_xy<DVR_F16, DVR_F32, kHessianOut>(a, taps, st);
}

hipError_t launch_features_scale(const void *vol, int vol_dt, const dvr_grid &g, const ScaleTaps &taps,
                                 int scale_index, bool last_scale, const dvr_feature_params &fp,
                                 const dvr_features_buf &out, float *ws_fields, float *ws_scalars,
                                 bool fro_pass, hipStream_t st)
{
    (void)last_scale;
    const uint32_t plane = (uint32_t)g.nx * (uint32_t)g.ny;
    dim3 zgrid((plane + 255) / 256, g.nz);
    hipError_t e;
    if (taps.ax[2].R >= 2 && taps.ax[2].R <= 10) {
        e = (vol_dt == DVR_F32) ? launch_z_r<DVR_F32, 2>(vol, ws_fields, g, taps.ax[2], st)
                                : launch_z_r<DVR_F16, 2>(vol, ws_fields, g, taps.ax[2], st);
    } else {
        if (vol_dt == DVR_F32)
            hipLaunchKernelGGL(k_zpass<DVR_F32>, zgrid, dim3(256), 0, st, vol, ws_fields, g.nx, g.ny, g.nz, taps.ax[2]);
        else
            hipLaunchKernelGGL(k_zpass<DVR_F16>, zgrid, dim3(256), 0, st, vol, ws_fields, g.nx, g.ny, g.nz, taps.ax[2]);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;

    XYArgs a;
    a.ws = ws_fields;
    a.vol = vol;
    a.grad = out.grad;
    a.kappa = out.kappa;
    a.ves = out.ves;
    a.gmax = out.gmax;
    a.fro = ws_scalars;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.inv2h[0] = (float)(1.0 / (2.0 * (double)g.hx));
    a.inv2h[1] = (float)(1.0 / (2.0 * (double)g.hy));
    a.inv2h[2] = (float)(1.0 / (2.0 * (double)g.hz));
    a.c_host = fp.c;
    a.inv2a2 = (float)(1.0 / (2.0 * (double)fp.alpha * fp.alpha));
    a.inv2b2 = (float)(1.0 / (2.0 * (double)fp.beta * fp.beta));
    a.tau = fp.eig_gap_fp64;
    a.first = (scale_index == 0) && !fro_pass;
    a.fro_pass = fro_pass;
    const int odt = out.dtype, lay = out.layout;
    const int R = taps.ax[0].R;
    if (R == taps.ax[1].R && R >= kRFastMin && R <= kRFastMax) {
        if (vol_dt == DVR_F32 && odt == DVR_F32 && lay == DVR_PLANAR)
            return launch_xy_r<DVR_F32, DVR_F32, DVR_PLANAR, kRFastMin>(a, taps, st);
        if (vol_dt == DVR_F16 && odt == DVR_F16 && lay == DVR_INTERLEAVED)
            return launch_xy_r<DVR_F16, DVR_F16, DVR_INTERLEAVED, kRFastMin>(a, taps, st);
        if (vol_dt == DVR_F32 && odt == DVR_F32 && lay == DVR_SPLIT)
            return launch_xy_r<DVR_F32, DVR_F32, DVR_SPLIT, kRFastMin>(a, taps, st);
        if (vol_dt == DVR_F16 && odt == DVR_F16 && lay == DVR_SPLIT)
            return launch_xy_r<DVR_F16, DVR_F16, DVR_SPLIT, kRFastMin>(a, taps, st);
    }
#define DVR_XY(D, O, L) \
    if (vol_dt == D && odt == O && lay == L) return launch_xy<D, O, L>(a, taps, st);
    DVR_XY(DVR_F32, DVR_F32, DVR_PLANAR)
    DVR_XY(DVR_F32, DVR_F32, DVR_INTERLEAVED)
    DVR_XY(DVR_F32, DVR_F16, DVR_PLANAR)
    DVR_XY(DVR_F32, DVR_F16, DVR_INTERLEAVED)
    DVR_XY(DVR_F16, DVR_F32, DVR_PLANAR)
    DVR_XY(DVR_F16, DVR_F32, DVR_INTERLEAVED)
    DVR_XY(DVR_F16, DVR_F16, DVR_PLANAR)
    DVR_XY(DVR_F16, DVR_F16, DVR_INTERLEAVED)
    DVR_XY(DVR_F32, DVR_F32, DVR_SPLIT)
    DVR_XY(DVR_F32, DVR_F16, DVR_SPLIT)
    DVR_XY(DVR_F16, DVR_F32, DVR_SPLIT)
    DVR_XY(DVR_F16, DVR_F16, DVR_SPLIT)
#undef DVR_XY
    return hipErrorInvalidValue;
}

}  // namespace dvr
