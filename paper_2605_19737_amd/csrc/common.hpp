// Internal declarations shared by the HIP sources of libdvr (not part of the C ABI).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dvr.h"

namespace dvr {

// ---------------------------------------------------------------------------------------------
// Raw buffer loads.  Every gather of the render and feature kernels goes through a buffer
// resource whose num_records is the byte size of the array, so an out-of-range offset returns 0
// in hardware instead of touching memory outside the array.  Word 3 is the gfx9-family raw
// buffer descriptor (32-bit data format, no swizzle).
constexpr int kRsrcWord3 = 0x00020000;

struct Buf {
    __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ Buf make_buf(const void *p, uint32_t bytes)
{
    Buf b;
    b.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3);
    return b;
}

__device__ __forceinline__ float ldf(Buf b, uint32_t byte_off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, byte_off, 0, 0));
}

__device__ __forceinline__ float ldh(Buf b, uint32_t byte_off)
{
    uint16_t v = __builtin_amdgcn_raw_buffer_load_b16(b.r, byte_off, 0, 0);
    return __half2float(__builtin_bit_cast(__half, v));
}

// 16-byte load (4 dwords) used for interleaved records.  Reinterpret the loaded vector as a
// whole (f32x4 / f16x8); a bit_cast of one ext-vector element is miscompiled at -O3.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 ld4(Buf b, uint32_t byte_off)
{
    return __builtin_amdgcn_raw_buffer_load_b128(b.r, byte_off, 0, 0);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
// two consecutive floats (byte_off 4-byte aligned; both must lie inside the buffer)
__device__ __forceinline__ f32x2 ld2f(Buf b, uint32_t byte_off)
{
    return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(b.r, byte_off, 0, 0));
}

// Load one element of a volume stored as F32 or F16.
template <int DT>
__device__ __forceinline__ float ldv(Buf b, uint32_t idx)
{
    if constexpr (DT == DVR_F32) return ldf(b, idx * 4u);
    else return ldh(b, idx * 2u);
}

template <int DT>
struct ElemSize {
    static constexpr uint32_t v = (DT == DVR_F32) ? 4u : 2u;
};

// ---------------------------------------------------------------------------------------------
// Derivative-of-Gaussian filter taps for one axis and one scale, computed on the host in double
// from the sampled, normalized Gaussian w_j (radius r, zero outside) and rounded to float.
// R = r + 1 is the stencil radius of the combined filters.
//   G[j]   = w_j                                 (j = 0..R)        smoothing
//   D1[j]  = (w_{j-1} - w_{j+1}) / (2h)          (j = 1..R)        central first difference of s
//   D2[j]  = (w_{j-1} - 2 w_j + w_{j+1}) / h^2   (j = 0..R)        central second difference of s
//   E1[m]  = (w_{m-1} - w_m) / (2h)              (m = -R..R+1)     one-sided first difference
//   E2[m]  = (w_{m-1} - w_m) / h^2               (m = -R..R+1)     one-sided second difference
// At the low face (i = 0) the clamped stencil of s gives s[1] - s[0], i.e. E applied at i = 0; at
// the high face (i = n-1) it gives s[n-2] - s[n-1], i.e. -E shifted by one (see features.hip).
struct AxisTaps {
    int R;
    float G[DVR_MAX_RADIUS + 2];
    float D1[DVR_MAX_RADIUS + 2];
    float D2[DVR_MAX_RADIUS + 2];
    float E1[2 * DVR_MAX_RADIUS + 4];  // index m + R
    float E2[2 * DVR_MAX_RADIUS + 4];
};

// Output mode of the feature kernels next to the layouts of dvr_layout: write the six Hessian entries
// of each voxel ([6][N] FP32) and nothing else.
constexpr int kHessianOut = 16;

struct ScaleTaps {
    AxisTaps ax[3];  // x, y, z
    float sigma2;    // sigma^2 (mm^2): scale normalization of the Hessian for the eigenvalues
};

// Launchers (host side, defined in the .hip files).
hipError_t launch_features_scale(const void *vol, int vol_dt, const dvr_grid &g, const ScaleTaps &taps,
                                 int scale_index, bool last_scale, const dvr_feature_params &fp,
                                 const dvr_features_buf &out, float *ws_fields, float *ws_scalars,
                                 bool fro_pass, hipStream_t st);
hipError_t launch_init_scalars(float *gmax, float *ws_scalars, hipStream_t st);
// The six Hessian entries of one scale, [6][N] FP32 in H (z-filtered fields staged in ws_fields, 3N).
hipError_t launch_hessian(const void *vol, int vol_dt, const dvr_grid &g, const ScaleTaps &taps, float *ws_fields,
                          float *H, hipStream_t st);
// Feature-pass adjoint (features_bwd.hip); the arguments are validated by the caller.
struct FeatBwdPlan {
    int nsigma;
    ScaleTaps taps[DVR_MAX_SIGMA];
    double sigma2[DVR_MAX_SIGMA];
    double inv2a2, inv2b2, inv2c2;  // 1 / (2 alpha^2), 1 / (2 beta^2), 1 / (2 c^2)
    double inv2h[3];                // 1 / (2 h_a)
};
size_t features_bwd_ws_bytes(const dvr_grid &g, const FeatBwdPlan &p);
hipError_t launch_features_backward(const void *vol, int vol_dt, const dvr_grid &g, const FeatBwdPlan &p,
                                    const float *dfeat, const float *dgmax, float *dvol, void *ws, hipStream_t st);
hipError_t launch_bricks(const void *vol, int vol_dt, const dvr_grid &g, const dvr_features_buf &out, hipStream_t st);
// dst[v] = (src(x,y,z), src(x,y+1,z), src(x,y,z+1), src(x,y+1,z+1)) with 0 past the last row or slice
// (bit copies of dtype elements): the quads of the QUAD feature layout
hipError_t launch_quads(const void *src, void *dst, const dvr_grid &g, int dtype, hipStream_t st);

hipError_t launch_normalize(const void *raw, int raw_dt, void *out, int out_dt, int64_t n, uint32_t *ws,
                            hipStream_t st);
// The allocation-free normalize's scratch (normalize.hip): its size, and this device's address of it.
size_t normalize_scratch_bytes();
hipError_t normalize_scratch(void **ptr);

hipError_t launch_histogram(const void *vol, int dt, int64_t n, float floor_, uint32_t *hist, uint32_t *used,
                            hipStream_t st);
hipError_t launch_peaks(const uint32_t *hist, int min_sep, dvr_peaks *out, hipStream_t st);
hipError_t launch_tissue_tf(const dvr_peaks *pk, const dvr_tissue_tf_params &p, float *knots, float *rgba,
                            hipStream_t st);

hipError_t launch_denoise(const void *vol, int dt, const dvr_grid &g, int mode, const int r[3],
                          const float w[3][DVR_MAX_RADIUS + 1], void *out, float *ws, hipStream_t st);

struct RenderArgs;
hipError_t launch_render(const RenderArgs &a, hipStream_t st);
hipError_t launch_render_backward(const RenderArgs &a, hipStream_t st);
hipError_t launch_render_gather(const RenderArgs &a, hipStream_t st);

}  // namespace dvr
