// LDS atomic-add rate on gfx950, FP32 (ds_add_f32) against FP64 (ds_add_f64), for six lane-to-address
// patterns.  This decides the entry type of the adjoint raymarch's LDS accumulation windows.
// A standalone program (not part of the library):
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o lds_atomic_rate lds_atomic_rate.hip && ./lds_atomic_rate
// Each 256-lane workgroup adds 1 to LDS words 4096 times per lane; both types use the same 64 KB
// of LDS (the same occupancy), and every index is masked into the array, so every access is in bounds.
// The printed cycles are per wave-instruction per CU at 2.4 GHz.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
constexpr int NE = 2048;  // entries per wave region
template <typename T, int PAT>
__global__ __launch_bounds__(256) void k(T *out, int iters, const int *tab)
{
    __shared__ double raw[4][NE];  // same LDS bytes (and occupancy) for both types
    T *ww = reinterpret_cast<T *>(raw[threadIdx.x >> 6]);
    for (int i = threadIdx.x & 63; i < NE; i += 64) ww[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    int base = 0;
    for (int it = 0; it < iters; ++it) {
        int a;
        if (PAT == 0) a = lane;                       // consecutive
        else if (PAT == 1) a = lane * 2;              // stride 2
        else if (PAT == 2) a = lane * 32;             // stride 32
        else if (PAT == 3) a = 0;                     // one address
        else if (PAT == 4) a = (lane & 7) * 6 + (lane >> 3) * 48;  // window-like 6/48 strides
        else a = tab[(it & 63) * 64 + lane];          // random
        a = (a + base) & (NE - 1);
        __hip_atomic_fetch_add(ww + a, (T)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        base += 7;
    }
    __syncthreads();
    out[blockIdx.x * 256 + threadIdx.x] = ww[lane];
}
template <typename T, int PAT>
float run(int blocks, int iters, const int *tab)
{
    T *o;
    hipMalloc(&o, sizeof(T) * blocks * 256);
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipLaunchKernelGGL((k<T, PAT>), dim3(blocks), dim3(256), 0, 0, o, iters, tab);
    hipEventRecord(a);
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL((k<T, PAT>), dim3(blocks), dim3(256), 0, 0, o, iters, tab);
    hipEventRecord(b);
    hipEventSynchronize(b);
    float ms;
    hipEventElapsedTime(&ms, a, b);
    hipFree(o);
    return ms / 5;
}
int main()
{
    std::vector<int> h(64 * 64);
    unsigned s = 12345;
    for (auto &x : h) { s = s * 1664525u + 1013904223u; x = (s >> 8) & 2047; }
    int *tab;
    hipMalloc(&tab, h.size() * 4);
    hipMemcpy(tab, h.data(), h.size() * 4, hipMemcpyHostToDevice);
    const int blocks = 256 * 4, iters = 4096;
    const double ops = (double)blocks * 4 * iters;  // wave-instructions
    const char *nm[] = {"consecutive", "stride2", "stride32", "same-addr", "win6/48", "random"};
#define R(P) { float f = run<float, P>(blocks, iters, tab), d = run<double, P>(blocks, iters, tab); \
    printf("%-12s f32 %8.3f ms (%6.2f cyc/wave-op/CU)  f64 %8.3f ms (%6.2f)\n", nm[P], f, f * 1e-3 * 2.4e9 * 256 / ops, d, d * 1e-3 * 2.4e9 * 256 / ops); }
    R(0) R(1) R(2) R(3) R(4) R(5)
    return 0;
}
