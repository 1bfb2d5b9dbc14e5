// Global min-max normalization (Sec. 2.2 Eq. 1): out = (I - min) / (max - min), 0 where max == min.
// Pass 1 reduces min and max: 16-byte loads in a grid-stride loop, a wave and then a workgroup
// reduction, and one atomic per workgroup on an order-preserving unsigned encoding, skipped when it
// cannot change the global value (device-scope atomics on one address serialize).  Pass 2 scales and
// stores 16 input bytes per lane and step (F16 rounded to nearest even, or F32).
#include <mutex>

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

template <int DT>
struct NormVec {
    static constexpr int k = (DT == DVR_F32) ? 4 : 8;  // elements per 16-byte load
};

// the k elements of 16-byte vector j as floats (U16 and F16 exactly representable)
template <int DT>
__device__ __forceinline__ void load_vec(const void *p, int64_t j, float (&x)[NormVec<DT>::k])
{
    const uint4 u = reinterpret_cast<const uint4 *>(p)[j];
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
    if constexpr (DT == DVR_F32) {
        for (int e = 0; e < 4; ++e) x[e] = __uint_as_float(w[e]);
    } else {
        for (int e = 0; e < 8; ++e) {
            const uint16_t h = (uint16_t)(w[e >> 1] >> ((e & 1) * 16));
            if constexpr (DT == DVR_U16) x[e] = (float)h;
            else x[e] = __half2float(__builtin_bit_cast(__half, h));
        }
    }
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
    constexpr int K = NormVec<DT>::k;
    uint32_t mn = 0xffffffffu, mx = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nv = n / K;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nv; j += stride) {
        float x[K];
        load_vec<DT>(raw, j, x);
        for (int e = 0; e < K; ++e) {
            const uint32_t v = (DT == DVR_U16) ? (uint32_t)x[e] : f2ord(x[e]);
            mn = v < mn ? v : mn;
            mx = v > mx ? v : mx;
        }
    }
    for (int64_t i = nv * K + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t v = load_ord<DT>(raw, i);
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    __shared__ uint32_t smn[4], smx[4];
    if ((threadIdx.x & 63) == 0) {
        smn[threadIdx.x >> 6] = mn;
        smx[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            mn = smn[w] < mn ? smn[w] : mn;
            mx = smx[w] > mx ? smx[w] : mx;
        }
        if (mn < __hip_atomic_load(ws + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(ws + 0, mn);
        if (mx > __hip_atomic_load(ws + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(ws + 1, mx);
    }
}

template <int DT, int ODT>
__device__ __forceinline__ void norm_store(void *out, int64_t i, float y)
{
    if constexpr (ODT == DVR_F16) reinterpret_cast<__half *>(out)[i] = __float2half_rn(y);
    else reinterpret_cast<float *>(out)[i] = y;
}

template <int DT, int ODT>
__global__ __launch_bounds__(256) void k_norm_scale(const void *__restrict__ raw, void *__restrict__ out, int64_t n,
                                                    const uint32_t *ws)
{
    constexpr int K = NormVec<DT>::k;
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
    const int64_t nv = n / K;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nv; j += stride) {
        float x[K];
        load_vec<DT>(raw, j, x);
        float y[K];
        for (int e = 0; e < K; ++e) y[e] = den > 0.f ? (x[e] - mn) / den : 0.f;
        if constexpr (ODT == DVR_F16) {
            // K = 8 (U16/F16 input) or 4 (F32 input): K halves per store
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            for (int e = 0; e < K; ++e)
                w[e >> 1] |= (uint32_t)__builtin_bit_cast(uint16_t, __float2half_rn(y[e])) << ((e & 1) * 16);
            if constexpr (K == 8) reinterpret_cast<uint4 *>(out)[j] = make_uint4(w[0], w[1], w[2], w[3]);
            else reinterpret_cast<uint2 *>(out)[j] = make_uint2(w[0], w[1]);
        } else {
            for (int e = 0; e < K; e += 4)
                reinterpret_cast<float4 *>(out)[j * (K / 4) + e / 4] = make_float4(y[e], y[e + 1], y[e + 2], y[e + 3]);
        }
    }
    for (int64_t i = nv * K + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float x;
        if constexpr (DT == DVR_U16) x = (float)reinterpret_cast<const uint16_t *>(raw)[i];
        else if constexpr (DT == DVR_F32) x = reinterpret_cast<const float *>(raw)[i];
        else x = __half2float(reinterpret_cast<const __half *>(raw)[i]);
        norm_store<DT, ODT>(out, i, den > 0.f ? (x - mn) / den : 0.f);
    }
}

template <int DT>
static hipError_t launch_norm_t(const void *raw, void *out, int out_dt, int64_t n, uint32_t *ws, hipStream_t st)
{
    // enough workgroups to fill the chip a few times over; each lane then loops over 16-byte vectors
    const int64_t blocks64 = (n / NormVec<DT>::k + 255) / 256;
    const unsigned blocks = (unsigned)(blocks64 < 2048 ? (blocks64 > 0 ? blocks64 : 1) : 2048);
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

// ------------------------------------------------------------------------------------------------
// Library-owned scratch of the allocation-free entry point (dvr_normalize_noalloc): the two
// reduction words, in a file-scope device array that every GPU the library runs on holds until the
// process ends.  Host code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept here.
constexpr size_t kNormScratchBytes = 256;
static __device__ __align__(256) uint32_t scratch[kNormScratchBytes / sizeof(uint32_t)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

size_t normalize_scratch_bytes() { return kNormScratchBytes; }

// Device address of this device's scratch (the current device); hipSuccess and *ptr set, or the
// HIP error of the lookup.
hipError_t normalize_scratch(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace dvr
