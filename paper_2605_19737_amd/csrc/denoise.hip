// Optional denoise pre-pass (Sec. 5.3: lightweight spatial smoothing or median filtering as an
// optional compute pass before the morphology pass).
//   k_median3   3x3x3 median, clamp-to-edge: a lane loads its 27 neighbours and selects the 14th
//               smallest by forgetful selection (keep 15, then repeatedly move the smallest and the
//               largest of the kept values to the ends, drop both and take in the next neighbour;
//               the median of the last three is the answer).  All indices are compile-time, so the
//               values stay in registers.  The result is one of the inputs (exact).
//   k_smooth    one axis of the separable sampled, normalized Gaussian (radius floor(3 sigma/h + 1/2),
//               clamp-to-edge), FP32 accumulation; three launches (x, y, z) through FP32 workspaces.
#include "common.hpp"

namespace dvr {

template <int DT>
__device__ __forceinline__ float ld_any(const void *p, uint32_t i)
{
    if constexpr (DT == DVR_F32) return reinterpret_cast<const float *>(p)[i];
    else return __half2float(reinterpret_cast<const __half *>(p)[i]);
}

template <int DT>
__device__ __forceinline__ void st_any(void *p, uint32_t i, float v)
{
    if constexpr (DT == DVR_F32) reinterpret_cast<float *>(p)[i] = v;
    else reinterpret_cast<__half *>(p)[i] = __float2half_rn(v);
}

__device__ __forceinline__ void cswap(float &a, float &b)
{
    const float lo = fminf(a, b), hi = fmaxf(a, b);
    a = lo;
    b = hi;
}

// After this, b[0] is the smallest and b[N-1] the largest of b[0..N-1].
template <int N>
__device__ __forceinline__ void min_max_to_ends(float (&b)[15])
{
#pragma unroll
    for (int i = 0; i < N - 1; ++i) cswap(b[i], b[i + 1]);  // largest to N-1
#pragma unroll
    for (int i = N - 3; i >= 0; --i) cswap(b[i], b[i + 1]);  // smallest of 0..N-2 to 0
}

// one forgetful-selection step on a kept set of N values: drop the ends, take in x
template <int N>
__device__ __forceinline__ void forget_step(float (&b)[15], float x)
{
    min_max_to_ends<N>(b);
#pragma unroll
    for (int i = 0; i < N - 2; ++i) b[i] = b[i + 1];
    b[N - 2] = x;
}

template <int DT>
__global__ __launch_bounds__(256) void k_median3(const void *__restrict__ in, void *__restrict__ out, int nx, int ny,
                                                 int nz)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= plane) return;
    const int z = (int)blockIdx.y;
    const int y = (int)(e / (uint32_t)nx), x = (int)(e - (uint32_t)y * nx);
    float v[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) {
        const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
        const int zz = min(max(z + dz, 0), nz - 1), yy = min(max(y + dy, 0), ny - 1), xx = min(max(x + dx, 0), nx - 1);
        v[k] = ld_any<DT>(in, (uint32_t)zz * plane + (uint32_t)yy * nx + xx);
    }
    float b[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) b[i] = v[i];
    forget_step<15>(b, v[15]);
    forget_step<14>(b, v[16]);
    forget_step<13>(b, v[17]);
    forget_step<12>(b, v[18]);
    forget_step<11>(b, v[19]);
    forget_step<10>(b, v[20]);
    forget_step<9>(b, v[21]);
    forget_step<8>(b, v[22]);
    forget_step<7>(b, v[23]);
    forget_step<6>(b, v[24]);
    forget_step<5>(b, v[25]);
    forget_step<4>(b, v[26]);
    // three left: their median
    const float m = fmaxf(fminf(b[0], b[1]), fminf(fmaxf(b[0], b[1]), b[2]));
    st_any<DT>(out, (uint32_t)z * plane + e, m);
}

struct GaussTaps {
    int r;
    float w[DVR_MAX_RADIUS + 1];
};

// out = G_axis * in along one axis (stride in elements, n the axis length)
template <int DTI, int DTO>
__global__ __launch_bounds__(256) void k_smooth(const void *__restrict__ in, void *__restrict__ out, int nx, int ny,
                                                int nz, int axis, GaussTaps t)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= plane) return;
    const int z = (int)blockIdx.y;
    const int y = (int)(e / (uint32_t)nx), x = (int)(e - (uint32_t)y * nx);
    const int pos = axis == 0 ? x : (axis == 1 ? y : z);
    const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const uint32_t st = axis == 0 ? 1u : (axis == 1 ? (uint32_t)nx : plane);
    const uint32_t base = (uint32_t)z * plane + e - (uint32_t)pos * st;
    float acc = t.w[0] * ld_any<DTI>(in, base + (uint32_t)pos * st);
    for (int m = 1; m <= t.r; ++m) {
        const int a = min(pos + m, n - 1), b = max(pos - m, 0);
        acc = fmaf(t.w[m], ld_any<DTI>(in, base + (uint32_t)a * st) + ld_any<DTI>(in, base + (uint32_t)b * st), acc);
    }
    st_any<DTO>(out, (uint32_t)z * plane + e, acc);
}

hipError_t launch_denoise(const void *vol, int dt, const dvr_grid &g, int mode, const int r[3],
                          const float w[3][DVR_MAX_RADIUS + 1], void *out, float *ws, hipStream_t st)
{
    const uint32_t plane = (uint32_t)g.nx * (uint32_t)g.ny;
    const dim3 grid((plane + 255) / 256, g.nz);
    if (mode == DVR_DENOISE_MEDIAN3) {
        if (dt == DVR_F32) hipLaunchKernelGGL(k_median3<DVR_F32>, grid, dim3(256), 0, st, vol, out, g.nx, g.ny, g.nz);
        else hipLaunchKernelGGL(k_median3<DVR_F16>, grid, dim3(256), 0, st, vol, out, g.nx, g.ny, g.nz);
        return hipGetLastError();
    }
    GaussTaps t[3];
    for (int a = 0; a < 3; ++a) {
        t[a].r = r[a];
        for (int j = 0; j <= DVR_MAX_RADIUS; ++j) t[a].w[j] = w[a][j];
    }
    const size_t N = (size_t)plane * g.nz;
    float *w0 = ws, *w1 = ws + N;
    if (dt == DVR_F32)
        hipLaunchKernelGGL((k_smooth<DVR_F32, DVR_F32>), grid, dim3(256), 0, st, vol, w0, g.nx, g.ny, g.nz, 0, t[0]);
    else
        hipLaunchKernelGGL((k_smooth<DVR_F16, DVR_F32>), grid, dim3(256), 0, st, vol, w0, g.nx, g.ny, g.nz, 0, t[0]);
    hipLaunchKernelGGL((k_smooth<DVR_F32, DVR_F32>), grid, dim3(256), 0, st, w0, w1, g.nx, g.ny, g.nz, 1, t[1]);
    if (dt == DVR_F32)
        hipLaunchKernelGGL((k_smooth<DVR_F32, DVR_F32>), grid, dim3(256), 0, st, w1, out, g.nx, g.ny, g.nz, 2, t[2]);
    else
        hipLaunchKernelGGL((k_smooth<DVR_F32, DVR_F16>), grid, dim3(256), 0, st, w1, out, g.nx, g.ny, g.nz, 2, t[2]);
    return hipGetLastError();
}

}  // namespace dvr
