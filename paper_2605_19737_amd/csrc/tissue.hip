// Automatic tissue windows (Sec. 2.2 "256-bin density analysis" and tissue peaks; Sec. 3.1 Table 2):
//   k_hist       256-bin counts of a normalized volume, privatized per workgroup in LDS (integer LDS
//                atomics) in kHistCopies interleaved copies (lane mod copies), so that lanes hitting
//                one bin at once (a volume's background fills one bin) spread over several addresses
//                and banks; one global atomic per non-empty bin per workgroup;
//   k_peaks      the three tissue peaks of the [1, 2, 1]-smoothed counts: local maxima taken greedily
//                by height at least min_sep bins apart, as three workgroup arg-max reductions (the
//                first is the highest maximum, the next the highest one far enough from those taken,
//                which is what the greedy pass over the sorted maxima selects), ordered by bin, each
//                checked against its Table 2 window;
//   k_tissue_tf  an 8-knot TF from the peaks (zero extinction below the CSF window).
#include "common.hpp"

namespace dvr {

constexpr int kHistCopies = 8;

// h: this lane's copy, bin b at h[b * kHistCopies]
template <int DT>
__device__ __forceinline__ void hist_add(uint32_t *h, float x, float floor_, uint32_t &used)
{
    if (x > floor_) {
        int b = (int)floorf(x * 256.f);
        b = b < 0 ? 0 : (b > 255 ? 255 : b);
        atomicAdd(h + b * kHistCopies, 1u);
        ++used;
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_hist(const void *__restrict__ vol, int64_t n, float floor_, uint32_t *hist,
                                              uint32_t *used_out)
{
    __shared__ uint32_t hs[256 * kHistCopies];
    __shared__ uint32_t wu[4];
    for (int i = threadIdx.x; i < 256 * kHistCopies; i += 256) hs[i] = 0u;
    __syncthreads();
    uint32_t *h = hs + (threadIdx.x % kHistCopies);
    constexpr int K = (DT == DVR_F32) ? 4 : 8;  // values per 16-byte load
    const int64_t nv = n / K;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t used = 0u;
    auto add16 = [&](const uint4 &u) {
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
        if constexpr (DT == DVR_F32) {
            for (int e = 0; e < 4; ++e) hist_add<DT>(h, __uint_as_float(w[e]), floor_, used);
        } else {
            for (int e = 0; e < 8; ++e)
                hist_add<DT>(h, __half2float(__builtin_bit_cast(__half, (uint16_t)(w[e >> 1] >> ((e & 1) * 16)))), floor_,
                             used);
        }
    };
    const uint4 *v4 = reinterpret_cast<const uint4 *>(vol);
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // four 16-byte loads in flight per lane, then their values
    for (; j + 3 * stride < nv; j += 4 * stride) {
        const uint4 u0 = v4[j], u1 = v4[j + stride], u2 = v4[j + 2 * stride], u3 = v4[j + 3 * stride];
        add16(u0);
        add16(u1);
        add16(u2);
        add16(u3);
    }
    for (; j < nv; j += stride) add16(v4[j]);
    for (int64_t i = nv * K + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float x = (DT == DVR_F32) ? reinterpret_cast<const float *>(vol)[i]
                                        : __half2float(reinterpret_cast<const __half *>(vol)[i]);
        hist_add<DT>(h, x, floor_, used);
    }
    for (int o = 32; o > 0; o >>= 1) used += __shfl_xor(used, o, 64);
    if ((threadIdx.x & 63) == 0) wu[threadIdx.x >> 6] = used;
    __syncthreads();
    uint32_t tot_b = 0u;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) tot_b += hs[threadIdx.x * kHistCopies + c];
    if (tot_b != 0u) atomicAdd(hist + threadIdx.x, tot_b);
    if (threadIdx.x == 0 && used_out) {
        const uint32_t tot = wu[0] + wu[1] + wu[2] + wu[3];
        if (tot) atomicAdd(used_out, tot);
    }
}

__global__ void k_zero_u32(uint32_t *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// workgroup maximum of a 64-bit key (every thread of the 256 must call)
__device__ __forceinline__ uint64_t block_max_u64(uint64_t v, uint64_t *red)
{
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t m = red[0];
    for (int i = 1; i < 4; ++i) m = red[i] > m ? red[i] : m;
    return m;
}

__global__ __launch_bounds__(256) void k_peaks(const uint32_t *__restrict__ hist, int min_sep, dvr_peaks *out)
{
    __shared__ uint64_t S[256];
    __shared__ uint64_t red[4];
    const int b = threadIdx.x;
    const uint64_t hl = hist[b > 0 ? b - 1 : 0], hc = hist[b], hr = hist[b < 255 ? b + 1 : 255];
    S[b] = hl + 2u * hc + hr;
    __syncthreads();
    const uint64_t s = S[b];
    const bool left_ok = (b == 0) || s > S[b - 1];
    const bool right_ok = (b == 255) || s >= S[b + 1];
    const bool cand = s > 0u && left_ok && right_ok;
    int taken[3] = {-1, -1, -1};
    int nt = 0;
    for (int i = 0; i < 3; ++i) {
        bool far = cand;
        for (int j = 0; j < nt; ++j) far = far && (b - taken[j] >= min_sep || taken[j] - b >= min_sep);
        // larger count first, then the lower bin (the key is never 0 for a candidate: s > 0)
        const uint64_t key = far ? ((s << 8) | (uint64_t)(255 - b)) : 0u;
        const uint64_t m = block_max_u64(key, red);
        if (m == 0u) break;
        taken[nt++] = 255 - (int)(m & 255u);
    }
    if (threadIdx.x == 0) {
        // order by bin (at most three)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2 - i; ++j) {
                const bool swap = (taken[j] < 0 && taken[j + 1] >= 0) || (taken[j + 1] >= 0 && taken[j + 1] < taken[j]);
                if (swap) {
                    const int t = taken[j];
                    taken[j] = taken[j + 1];
                    taken[j + 1] = t;
                }
            }
        // Table 2 windows: CSF [0.05, 0.12), GM [0.12, 0.18), WM (0.18, 1]
        const double lo[3] = {0.05, 0.12, 0.18}, hi[3] = {0.12, 0.18, 1.0};
        for (int c = 0; c < 3; ++c) {
            const int bb = taken[c];
            out->bin[c] = bb;
            const float p = bb >= 0 ? ((float)bb + 0.5f) / 256.f : -1.f;
            out->peak[c] = p;
            const double d = p;
            out->in_window[c] = bb >= 0 && (c < 2 ? (d >= lo[c] && d < hi[c]) : (d > lo[c] && d <= hi[c]));
        }
    }
}

struct TissueTFArgs {
    float rgb[3][3];
    float tau[3];
    float rgb_hi[3];
    float tau_hi;
};

__global__ void k_tissue_tf(const dvr_peaks *__restrict__ pk, TissueTFArgs p, float *knots, float *rgba)
{
    if (threadIdx.x != 0) return;
    const float fb[3] = {0.085f, 0.15f, 0.24f};  // a missing peak: its window's centre (WM: edge + GM width)
    float m[3];
    for (int c = 0; c < 3; ++c) m[c] = pk->bin[c] >= 0 ? ((float)pk->bin[c] + 0.5f) / 256.f : fb[c];
    const float lo = 0.05f, s = 1.f / 256.f;
    // strictly increasing knots, at least one bin apart; the WM peak at most three bins below 1
    m[0] = fmaxf(m[0], lo + s);
    m[1] = fmaxf(m[1], m[0] + s);
    m[2] = fmaxf(m[2], m[1] + s);
    m[2] = fminf(m[2], 1.f - 3.f * s);
    m[1] = fminf(m[1], m[2] - s);
    m[0] = fminf(m[0], m[1] - s);
    const float u = fminf(fmaxf(2.f * m[2] - m[1], m[2] + s), 1.f - 2.f * s);
    const float kx[8] = {0.f, lo, m[0], m[1], m[2], u, u + s, 1.f};
    const int col[8] = {0, 0, 0, 1, 2, 2, 3, 3};
    const float tau[8] = {0.f, 0.f, p.tau[0], p.tau[1], p.tau[2], p.tau[2], p.tau_hi, p.tau_hi};
    for (int k = 0; k < 8; ++k) {
        knots[k] = kx[k];
        const float *c = col[k] < 3 ? p.rgb[col[k]] : p.rgb_hi;
        rgba[4 * k + 0] = c[0];
        rgba[4 * k + 1] = c[1];
        rgba[4 * k + 2] = c[2];
        rgba[4 * k + 3] = tau[k];
    }
}

hipError_t launch_histogram(const void *vol, int dt, int64_t n, float floor_, uint32_t *hist, uint32_t *used,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, hist, 256);
    if (used) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, used, 1);
    const int K = dt == DVR_F32 ? 4 : 8;
    const int64_t b64 = (n / K + 255) / 256;
    // 1024 workgroups: enough to fill the chip, and each bin's global counter takes one add per
    // workgroup (same-address atomics serialize at the L2)
    const unsigned blocks = (unsigned)(b64 < 1024 ? (b64 > 0 ? b64 : 1) : 1024);
    if (dt == DVR_F32)
        hipLaunchKernelGGL(k_hist<DVR_F32>, dim3(blocks), dim3(256), 0, st, vol, n, floor_, hist, used);
    else
        hipLaunchKernelGGL(k_hist<DVR_F16>, dim3(blocks), dim3(256), 0, st, vol, n, floor_, hist, used);
    return hipGetLastError();
}

hipError_t launch_peaks(const uint32_t *hist, int min_sep, dvr_peaks *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_peaks, dim3(1), dim3(256), 0, st, hist, min_sep, out);
    return hipGetLastError();
}

hipError_t launch_tissue_tf(const dvr_peaks *pk, const dvr_tissue_tf_params &p, float *knots, float *rgba,
                            hipStream_t st)
{
    TissueTFArgs a;
    for (int c = 0; c < 3; ++c) {
        for (int k = 0; k < 3; ++k) a.rgb[c][k] = p.rgb[c][k];
        a.tau[c] = p.tau[c];
        a.rgb_hi[c] = p.rgb_hi[c];
    }
    a.tau_hi = p.tau_hi;
    hipLaunchKernelGGL(k_tissue_tf, dim3(1), dim3(64), 0, st, pk, a, knots, rgba);
    return hipGetLastError();
}

}  // namespace dvr
