// Global min-max normalization (Sec. 2.2 Eq. 1): out = (I - min) / (max - min), 0 where max == min.
// Pass 1 reduces min and max (wave reduction, then one atomic per wave on an order-preserving
// unsigned encoding), pass 2 scales and stores (F16 rounded to nearest even, or F32).
#include "common.hpp"

namespace dvr {

// order-preserving map of a float onto uint32 (total order of non-NaN values)
__device__ __forceinline__ uint32_t f2ord(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

template <int DT>
__device__ __forceinline__ uint32_t load_ord(const void *p, int64_t i)
{
    if constexpr (DT == DVR_U16) return reinterpret_cast<const uint16_t *>(p)[i];
    else if constexpr (DT == DVR_F32) return f2ord(reinterpret_cast<const float *>(p)[i]);
    else return f2ord(__half2float(reinterpret_cast<const __half *>(p)[i]));
}

__global__ void k_norm_init(uint32_t *ws)
{
    if (threadIdx.x == 0) {
        ws[0] = 0xffffffffu;  // min
        ws[1] = 0u;           // max
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_norm_reduce(const void *__restrict__ raw, int64_t n, uint32_t *ws)
{
    uint32_t mn = 0xffffffffu, mx = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t v = load_ord<DT>(raw, i);
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(ws + 0, mn);
        atomicMax(ws + 1, mx);
    }
}

template <int DT, int ODT>
__global__ __launch_bounds__(256) void k_norm_scale(const void *__restrict__ raw, void *__restrict__ out, int64_t n,
                                                    const uint32_t *ws)
{
    float mn, mx;
    if constexpr (DT == DVR_U16) {
        mn = (float)ws[0];
        mx = (float)ws[1];
    } else {
        mn = ord2f(ws[0]);
        mx = ord2f(ws[1]);
    }
    const float den = mx - mn;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float x;
        if constexpr (DT == DVR_U16) x = (float)reinterpret_cast<const uint16_t *>(raw)[i];
        else if constexpr (DT == DVR_F32) x = reinterpret_cast<const float *>(raw)[i];
        else x = __half2float(reinterpret_cast<const __half *>(raw)[i]);
        const float y = den > 0.f ? (x - mn) / den : 0.f;
        if constexpr (ODT == DVR_F16) reinterpret_cast<__half *>(out)[i] = __float2half_rn(y);
        else reinterpret_cast<float *>(out)[i] = y;
    }
}

template <int DT>
static hipError_t launch_norm_t(const void *raw, void *out, int out_dt, int64_t n, uint32_t *ws, hipStream_t st)
{
    const int64_t blocks64 = (n + 255) / 256;
    const unsigned blocks = (unsigned)(blocks64 < 8192 ? blocks64 : 8192);
    hipLaunchKernelGGL(k_norm_init, dim3(1), dim3(64), 0, st, ws);
    hipLaunchKernelGGL(k_norm_reduce<DT>, dim3(blocks), dim3(256), 0, st, raw, n, ws);
    if (out_dt == DVR_F16)
        hipLaunchKernelGGL((k_norm_scale<DT, DVR_F16>), dim3(blocks), dim3(256), 0, st, raw, out, n, ws);
    else
        hipLaunchKernelGGL((k_norm_scale<DT, DVR_F32>), dim3(blocks), dim3(256), 0, st, raw, out, n, ws);
    return hipGetLastError();
}

hipError_t launch_normalize(const void *raw, int raw_dt, void *out, int out_dt, int64_t n, uint32_t *ws,
                            hipStream_t st)
{
    if (raw_dt == DVR_U16) return launch_norm_t<DVR_U16>(raw, out, out_dt, n, ws, st);
    if (raw_dt == DVR_F32) return launch_norm_t<DVR_F32>(raw, out, out_dt, n, ws, st);
    return launch_norm_t<DVR_F16>(raw, out, out_dt, n, ws, st);
}

}  // namespace dvr
