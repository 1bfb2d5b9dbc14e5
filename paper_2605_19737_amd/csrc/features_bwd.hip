// Feature-pass adjoint for gfx950: dL/dI of the gradient (Sec. 2.3 Eq. 2), the first-scale
// curvature (Sec. 2.3 Eq. 3), the multi-scale Frangi vesselness (Sec. 1) and |g|_max (the Eq. 4
// normalizer), given dL/d(g, k, V) per voxel and dL/d|g|_max (what the render adjoint with
// feature gradients produces).
//
// Every linear step of the forward is a per-axis banded matrix: the clamped central difference of
// the gradient, and per scale and axis the three combined smoothing-and-difference operators
// (G, D1 G, D2 G) with their one-sided first and last rows.  The adjoint applies the transposes.
// First the six Hessian entries of every scale are computed with the forward's own kernels
// (Hessian-output mode) and kept, and the winning scale of each voxel is found (k_fb_win: FP64
// eigenvalues and V per scale, the first scale whose V exceeds every earlier one and 0).  Then per
// scale:
//   1. k_fb_local (FP64, one lane per voxel) forms dL/dH: the curvature term g g^T / g^T g at the
//      first scale, and at the voxel's winning scale dL/dV sigma^2 sum_i dV/dlambda_i e_i e_i^T from
//      a Jacobi eigen-decomposition (those voxels listed over the workgroup's 1024 and solved one per
//      lane); at the first scale it also writes dL/dg + dL/dk dk/dg and the arg-max key of |g|;
//   2. the x, y and z transposes apply the transposed operators (the forward's z-then-y-then-x order
//      reversed: six fields after x, three after y, one accumulated into dL/dI after z): for radii
//      2..10 k_tx_lds_r, k_ty_run_r, k_tz_run_r, else k_tx_lds (k_tx), k_ty_run, k_tz_run.
// Last, dL/d|g|_max goes to the arg-max voxel's gradient (k_fb_gmax) and the transposed central
// difference of the gradient is added (k_fb_gradT).
//
// The band tables are built on the device from the forward's FP32 taps (k_band), so the transpose
// is that of the operator the forward applies.
#include <math.h>

#include "common.hpp"
#include "features_dev.hpp"

namespace dvr {

// B[f][d + R][i]: weight of input i + d in output i of operator f (0: G, 1: D1 G, 2: D2 G) along an
// axis of n voxels; clamped taps fold onto the end voxels, the first and last rows are one-sided.
// Stored d-major so that lanes on consecutive outputs of a transposed filter read consecutive
// entries.  One lane per entry (f, d, i), summing the taps m that land on column i + d;
// blockIdx.y = axis.
struct BandJob {
    AxisTaps t[3];
    int n[3];
    float *B[3];
};

__global__ __launch_bounds__(256) void k_band(BandJob j)
{
    const int a = (int)blockIdx.y;
    const AxisTaps &t = j.t[a];
    const int n = j.n[a], R = t.R, W = 2 * R + 1;
    const int id = (int)(blockIdx.x * 256u + threadIdx.x);
    if (id >= 3 * n * W) return;
    const int f = id / (n * W), rem = id - f * n * W, d = rem / n, i = rem - d * n;
    const int cls = (i == 0) ? 1 : (i == n - 1 ? 2 : 0);
    float acc = 0.f;
    for (int m = -R; m <= R; ++m) {
        if (clampi(i + m, 0, n - 1) - i + R != d) continue;
        const int am = m < 0 ? -m : m;
        float c;
        if (f == 0) c = t.G[am];
        else if (cls == 0) c = (f == 1) ? (m > 0 ? t.D1[am] : (m < 0 ? -t.D1[am] : 0.f)) : t.D2[am];
        else if (cls == 1) c = (f == 1) ? t.E1[m + R] : t.E2[m + R];
        else c = (f == 1) ? t.E1[m + 1 + R] : -t.E2[m + 1 + R];
        acc += c;
    }
    j.B[a][id] = acc;
}

template <int DT>
__device__ __forceinline__ double ldd(const void *p, size_t i)
{
    if constexpr (DT == DVR_F32) return (double)reinterpret_cast<const float *>(p)[i];
    else return (double)__half2float(reinterpret_cast<const __half *>(p)[i]);
}

// (|l|, l) ascending, as the forward sorts the eigenvalues
__device__ __forceinline__ bool key_less(double u, double v) { return fabs(u) < fabs(v) || (fabs(u) == fabs(v) && u < v); }

// Frangi bright-tube vesselness of magnitude-sorted eigenvalues (FP64)
__device__ __forceinline__ double frangi64(double l1, double l2, double l3, double ia, double ib, double ic)
{
    if (l2 >= 0.0 || l3 >= 0.0) return 0.0;
    const double Ra2 = (l2 * l2) / (l3 * l3);
    const double Rb2 = (l1 * l1) / fabs(l2 * l3);
    const double S2 = l1 * l1 + l2 * l2 + l3 * l3;
    return -expm1(-Ra2 * ia) * exp(-Rb2 * ib) * -expm1(-S2 * ic);
}

// Whether V can be non-zero at A (FP64): V != 0 exactly when A - tr(A) I is positive definite (its
// eigenvalues are minus the pair sums of A's), so a leading principal minor of it below minus a
// margin proves V = 0 (Sylvester's criterion).  Margins of 1e-5 s^k (s the largest |m_ij|) put the
// pair sum at >= 1e-6 s, far above the error of the FP64 closed-form eigenvalues.
__device__ __forceinline__ bool maybe_vessel64(const double A[6])
{
    const double t = A[0] + A[1] + A[2];
    if (!(t < 0.0)) return false;
    const double m00 = A[0] - t, m11 = A[1] - t, m22 = A[2] - t, m01 = A[3], m02 = A[4], m12 = A[5];
    const double sc = fmax(fmax(fmax(fabs(m00), fabs(m11)), fmax(fabs(m22), fabs(m01))), fmax(fabs(m02), fabs(m12)));
    const double e = 1e-5 * sc, e2 = e * sc, e3 = e2 * sc;
    const double d2 = m00 * m11 - m01 * m01;
    const double d3 = m00 * (m11 * m22 - m12 * m12) - m01 * (m01 * m22 - m12 * m02) + m02 * (m01 * m12 - m11 * m02);
    return !(m00 < -e || d2 < -e2 || d3 < -e3);
}

// Workgroup list of voxel indices: the lanes with need set append v (one LDS atomic per wave).
// Every lane of the wave must call it.
__device__ __forceinline__ void wg_append(bool need, uint32_t v, uint32_t *list, int *count)
{
    const uint64_t bal = __ballot(need);
    if (bal == 0ull) return;
    const int lead = __ffsll((unsigned long long)bal) - 1;
    int base = 0;
    if ((int)(threadIdx.x & 63) == lead) base = atomicAdd(count, __popcll(bal));
    base = __shfl(base, lead, 64);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (need) list[base + rank] = v;
}

// Voxels per workgroup of the local-step kernel (kFbSub runs of 256): the few voxels that need the
// FP64 eigen work are listed over all of them and solved densely, so the lanes of a wave are busy
// instead of a wave running the solve for its few such lanes.
constexpr int kFbSub = 4;

// winning scale: V_s in FP64 (closed-form eigenvalues), the first scale above every earlier one and 0,
// one lane per voxel (its time is bound by reading the Hessians: listing the few voxels that take the
// eigenvalues, as the local step does, made it slower)
__global__ __launch_bounds__(256) void k_fb_win(const float *__restrict__ H, double *__restrict__ best,
                                                uint8_t *__restrict__ win, int s, double sigma2, double ia, double ib,
                                                double ic, uint32_t N)
{
    const uint32_t v = blockIdx.x * 256u + threadIdx.x;
    if (v >= N) return;
    double A[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) A[e] = sigma2 * (double)H[(size_t)e * N + v];
    double V = 0.0;
    if (maybe_vessel64(A)) {
        double lo, mi, hi;
        eig_trig<double>(A[0], A[1], A[2], A[3], A[4], A[5], lo, mi, hi);
        double a = lo, b = mi, c = hi, t;
        if (key_less(b, a)) { t = a; a = b; b = t; }
        if (key_less(c, b)) { t = b; b = c; c = t; }
        if (key_less(b, a)) { t = a; a = b; b = t; }
        V = frangi64(a, b, c, ia, ib, ic);
    }
    const double prev = s == 0 ? 0.0 : best[v];
    if (s == 0) win[v] = 255;
    if (V > prev) {
        best[v] = V;
        win[v] = (uint8_t)s;
    } else if (s == 0) {
        best[v] = 0.0;
    }
}

// one Jacobi rotation annihilating a_pq (r the third index); v accumulates the rotations
#define DVR_JROT(p, q, r)                                                                        \
    if (a[p][q] != 0.0) {                                                                        \
        if (fabs(a[p][q]) <= 1e-300 || fabs(a[p][q]) <= 1e-19 * (fabs(a[p][p]) + fabs(a[q][q]))) { \
            a[p][q] = a[q][p] = 0.0;                                                             \
        } else {                                                                                 \
            const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);                             \
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));       \
            const double cc = 1.0 / sqrt(tt * tt + 1.0), ss = tt * cc;                            \
            const double apq = a[p][q];                                                          \
            a[p][p] -= tt * apq;                                                                 \
            a[q][q] += tt * apq;                                                                 \
            a[p][q] = a[q][p] = 0.0;                                                             \
            const double arp = a[r][p], arq = a[r][q];                                           \
            a[r][p] = a[p][r] = cc * arp - ss * arq;                                             \
            a[r][q] = a[q][r] = ss * arp + cc * arq;                                             \
            for (int k = 0; k < 3; ++k) {                                                        \
                const double vp = V[k][p], vq = V[k][q];                                         \
                V[k][p] = cc * vp - ss * vq;                                                     \
                V[k][q] = ss * vp + cc * vq;                                                     \
            }                                                                                    \
        }                                                                                        \
    }

// eigenvalues lam[i] and unit eigenvectors V[.][i] of a symmetric 3x3 (cyclic Jacobi, FP64)
__device__ __forceinline__ void jacobi3v(const double A6[6], double lam[3], double V[3][3])
{
    double a[3][3] = {{A6[0], A6[3], A6[4]}, {A6[3], A6[1], A6[5]}, {A6[4], A6[5], A6[2]}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 16; ++sweep) {
        if (a[0][1] == 0.0 && a[0][2] == 0.0 && a[1][2] == 0.0) break;
        DVR_JROT(0, 1, 2)
        DVR_JROT(0, 2, 1)
        DVR_JROT(1, 2, 0)
    }
    lam[0] = a[0][0];
    lam[1] = a[1][1];
    lam[2] = a[2][2];
}
#undef DVR_JROT

// dV/dlambda for magnitude-sorted eigenvalues (0 where V = 0 by the sign rule)
__device__ __forceinline__ void frangi64_grad(const double l[3], double ia, double ib, double ic, double f[3])
{
    f[0] = f[1] = f[2] = 0.0;
    const double l1 = l[0], l2 = l[1], l3 = l[2];
    if (l2 >= 0.0 || l3 >= 0.0) return;
    const double p = l2 * l3;
    const double Ra2 = l2 * l2 / (l3 * l3), Rb2 = l1 * l1 / p, S2 = l1 * l1 + l2 * l2 + l3 * l3;
    const double ea = exp(-Ra2 * ia), Fa = 1.0 - ea;
    const double Fb = exp(-Rb2 * ib);
    const double ec = exp(-S2 * ic), Fc = 1.0 - ec;
    const double ga = Fb * Fc * ea * ia;       // dV/dRa2
    const double gb = -Fa * Fc * Fb * ib;      // dV/dRb2
    const double gc = Fa * Fb * ec * ic;       // dV/dS2
    f[0] = gb * (2.0 * l1 / p) + gc * 2.0 * l1;
    f[1] = ga * (2.0 * l2 / (l3 * l3)) + gb * (-l1 * l1 / (l2 * l2 * l3)) + gc * 2.0 * l2;
    f[2] = ga * (-2.0 * l2 * l2 / (l3 * l3 * l3)) + gb * (-l1 * l1 / (l2 * l3 * l3)) + gc * 2.0 * l3;
}

// order-preserving 64-bit key of (|g| rounded to FP32, lowest voxel index on a tie)
__device__ __forceinline__ unsigned long long gkey(float gn, uint32_t v)
{
    return ((unsigned long long)__float_as_uint(gn) << 32) | (unsigned long long)(0xffffffffu - v);
}

// The curvature part of the local step at one voxel of the first scale (x, y, z; v its index): adds
// dL/dk dk/dH to hb, writes dL/dg + dL/dk dk/dg of the voxel to dgt when wr is set, and returns the
// arg-max key of |g|
template <int DT>
__device__ __forceinline__ unsigned long long local_k(const void *__restrict__ vol, const float *__restrict__ H,
                                                      const float *__restrict__ dfeat, float *__restrict__ dgt,
                                                      uint32_t v, int x, int y, int z, int nx, int ny, int nz,
                                                      size_t N, double ih0, double ih1, double ih2, bool wr,
                                                      double hb[6])
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    double Hd[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) Hd[k] = (double)H[(size_t)k * N + v];
    const size_t row = (size_t)z * plane + (size_t)y * nx;
    const double ixp = ldd<DT>(vol, row + clampi(x + 1, 0, nx - 1)), ixm = ldd<DT>(vol, row + clampi(x - 1, 0, nx - 1));
    const double iyp = ldd<DT>(vol, (size_t)z * plane + (size_t)clampi(y + 1, 0, ny - 1) * nx + x);
    const double iym = ldd<DT>(vol, (size_t)z * plane + (size_t)clampi(y - 1, 0, ny - 1) * nx + x);
    const double izp = ldd<DT>(vol, (size_t)clampi(z + 1, 0, nz - 1) * plane + (size_t)y * nx + x);
    const double izm = ldd<DT>(vol, (size_t)clampi(z - 1, 0, nz - 1) * plane + (size_t)y * nx + x);
    const double g0 = (ixp - ixm) * ih0, g1 = (iyp - iym) * ih1, g2 = (izp - izm) * ih2;
    const double gg = g0 * g0 + g1 * g1 + g2 * g2;
    // the arg-max key takes |g| exactly as the feature pass rounds it: FP32 differences times the
    // FP32 1/(2h), then grad_norm (the values |g|_max is the maximum of)
    const float gn32 = grad_norm(((float)ixp - (float)ixm) * (float)ih0, ((float)iyp - (float)iym) * (float)ih1,
                                 ((float)izp - (float)izm) * (float)ih2);
    double d0 = dfeat[v], d1 = dfeat[N + v], d2 = dfeat[2 * N + v];
    const double dk = dfeat[3 * N + v];
    if (gg > 0.0 && dk != 0.0) {
        // k = g^T H g / g^T g: dk/dg = 2 (H g - k g) / g^T g, dk/dH_ab = g_a g_b / g^T g (x2 off-diagonal)
        const double Hg0 = Hd[0] * g0 + Hd[3] * g1 + Hd[4] * g2;
        const double Hg1 = Hd[3] * g0 + Hd[1] * g1 + Hd[5] * g2;
        const double Hg2 = Hd[4] * g0 + Hd[5] * g1 + Hd[2] * g2;
        const double ig = 1.0 / gg;
        const double k = (g0 * Hg0 + g1 * Hg1 + g2 * Hg2) * ig;
        const double c2 = 2.0 * dk * ig;
        d0 += c2 * (Hg0 - k * g0);
        d1 += c2 * (Hg1 - k * g1);
        d2 += c2 * (Hg2 - k * g2);
        const double c1 = dk * ig;
        hb[0] += c1 * g0 * g0;
        hb[1] += c1 * g1 * g1;
        hb[2] += c1 * g2 * g2;
        hb[3] += 2.0 * c1 * g0 * g1;
        hb[4] += 2.0 * c1 * g0 * g2;
        hb[5] += 2.0 * c1 * g1 * g2;
    }
    if (wr) {
        dgt[v] = (float)d0;
        dgt[N + v] = (float)d1;
        dgt[2 * N + v] = (float)d2;
    }
    return gkey(gn32, v);
}

// The vesselness part of the local step at a voxel whose winning scale is this one: dL/dH =
// dL/dV sigma^2 sum_i dV/dlambda_i e_i e_i^T (off-diagonal entries counted twice), from a Jacobi
// eigen-decomposition of sigma^2 H
__device__ __forceinline__ void local_v(const float *__restrict__ H, const float *__restrict__ dfeat, uint32_t v,
                                        size_t N, double sigma2, double ia, double ib, double ic, double add[6])
{
    double A[6], lam[3], Q[3][3];
#pragma unroll
    for (int k = 0; k < 6; ++k) A[k] = sigma2 * (double)H[(size_t)k * N + v];
    const double dV = dfeat[4 * N + v];
    jacobi3v(A, lam, Q);
    int o[3] = {0, 1, 2}, t;
    if (key_less(lam[o[1]], lam[o[0]])) { t = o[0]; o[0] = o[1]; o[1] = t; }
    if (key_less(lam[o[2]], lam[o[1]])) { t = o[1]; o[1] = o[2]; o[2] = t; }
    if (key_less(lam[o[1]], lam[o[0]])) { t = o[0]; o[0] = o[1]; o[1] = t; }
    const double ls[3] = {lam[o[0]], lam[o[1]], lam[o[2]]};
    double f[3];
    frangi64_grad(ls, ia, ib, ic, f);
    double P[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double x0 = Q[0][o[i]], x1 = Q[1][o[i]], x2 = Q[2][o[i]];
        P[0] += f[i] * x0 * x0;
        P[1] += f[i] * x1 * x1;
        P[2] += f[i] * x2 * x2;
        P[3] += f[i] * x0 * x1;
        P[4] += f[i] * x0 * x2;
        P[5] += f[i] * x1 * x2;
    }
    const double w = dV * sigma2;
#pragma unroll
    for (int k = 0; k < 6; ++k) add[k] = (k < 3 ? 1.0 : 2.0) * w * P[k];
}

// workgroup maximum of the arg-max keys, then one atomic when it beats the current maximum: atomics on
// one address serialize in the L2, and one per wave cost about a millisecond on the head (a stale
// read of the key is never above the true maximum, so skipping stays exact).  Every thread of the
// 256-lane workgroup must be here.
__device__ __forceinline__ void key_max(unsigned long long kv, unsigned long long *__restrict__ key)
{
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(kv, o, 64);
        kv = w > kv ? w : kv;
    }
    __shared__ unsigned long long wkey[4];
    if ((threadIdx.x & 63) == 0) wkey[threadIdx.x >> 6] = kv;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 1; k < 4; ++k) kv = wkey[k] > kv ? wkey[k] : kv;
        if (kv != 0ull && kv > __hip_atomic_load(key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(key, kv);
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_fb_local(const void *__restrict__ vol, const float *__restrict__ H,
                                                  const float *__restrict__ dfeat, const uint8_t *__restrict__ win,
                                                  float *__restrict__ Hb, float *__restrict__ dgt,
                                                  unsigned long long *__restrict__ key, int s, double sigma2, double ia,
                                                  double ib, double ic, int nx, int ny, int nz, double ih0, double ih1,
                                                  double ih2)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const int z = (int)blockIdx.y;
    const size_t N = (size_t)plane * (size_t)nz;
    // the vesselness term (voxels whose winning scale is s and whose dL/dV is not 0, a few per cent)
    // is listed over the workgroup's kFbSub runs of 256 voxels and solved densely after them
    __shared__ uint32_t vl[kFbSub * 256];
    __shared__ int vcount;
    if (threadIdx.x == 0) vcount = 0;
    __syncthreads();
    unsigned long long kv = 0ull;
    for (int j = 0; j < kFbSub; ++j) {
        const uint32_t e = (blockIdx.x * kFbSub + j) * 256u + threadIdx.x;
        const bool live = e < plane;
        const uint32_t v = (uint32_t)z * plane + (live ? e : 0u);
        double hb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (s == 0 && live) {
            const int y = (int)(e / (uint32_t)nx), x = (int)(e - (uint32_t)y * nx);
            const unsigned long long kk = local_k<DT>(vol, H, dfeat, dgt, v, x, y, z, nx, ny, nz, N, ih0, ih1, ih2, true, hb);
            kv = kk > kv ? kk : kv;
        }
        if (live) {
#pragma unroll
            for (int k = 0; k < 6; ++k) Hb[(size_t)k * N + v] = (float)hb[k];
        }
        wg_append(live && win[v] == (uint8_t)s && dfeat[4 * N + v] != 0.f, v, vl, &vcount);
    }
    __syncthreads();  // the list, and this workgroup's Hb stores, are complete
    const int count = vcount;
    for (int q = threadIdx.x; q < count; q += 256) {
        const uint32_t v = vl[q];
        double add[6];
        local_v(H, dfeat, v, N, sigma2, ia, ib, ic, add);
        // added to the k term this workgroup stored for the voxel above
#pragma unroll
        for (int k = 0; k < 6; ++k) Hb[(size_t)k * N + v] = (float)((double)Hb[(size_t)k * N + v] + add[k]);
    }
    if (s == 0) key_max(kv, key);
}

// x: six fields X_e = (operator of entry e along x)^T Hb_e; xx uses D2 G, xy and xz D1 G, the rest G
__global__ __launch_bounds__(256) void k_tx(const float *__restrict__ Hb, float *__restrict__ X,
                                            const float *__restrict__ B, int nx, int ny, int nz, int R)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= plane) return;
    const int z = (int)blockIdx.y;
    const int y = (int)(e / (uint32_t)nx), x = (int)(e - (uint32_t)y * nx);
    const size_t N = (size_t)plane * (size_t)nz;
    const size_t row = (size_t)z * plane + (size_t)y * nx;
    const int W = 2 * R + 1;
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int i0 = max(0, x - R), i1 = min(nx - 1, x + R);
    for (int i = i0; i <= i1; ++i) {
        const int d = x - i + R;
        const float b0 = B[(size_t)d * nx + i], b1 = B[(size_t)(W + d) * nx + i], b2 = B[(size_t)(2 * W + d) * nx + i];
        const size_t sidx = row + i;
        acc[0] = fmaf(b2, Hb[sidx], acc[0]);
        acc[1] = fmaf(b0, Hb[N + sidx], acc[1]);
        acc[2] = fmaf(b0, Hb[2 * N + sidx], acc[2]);
        acc[3] = fmaf(b1, Hb[3 * N + sidx], acc[3]);
        acc[4] = fmaf(b1, Hb[4 * N + sidx], acc[4]);
        acc[5] = fmaf(b0, Hb[5 * N + sidx], acc[5]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) X[(size_t)k * N + row + x] = acc[k];
}

// The same x transpose for one chunk of up to 256 outputs of one row per workgroup (blockIdx.x =
// y + ny z, blockIdx.y = chunk): the six fields of the chunk and its R-voxel halo are staged in LDS
// once, instead of 6 (2R + 1) global loads per output.  An output whose contributing forward rows
// i in [x - R, x + R] all lie in [R, nx - 1 - R] (no clamped or one-sided taps) takes the weights from
// the taps themselves, which is what the band table holds there (a single tap per entry); the
// others read the band table.  Same products in the same order as k_tx: the same bits.
constexpr int kTxChunk = 256;
__global__ __launch_bounds__(256) void k_tx_lds(const float *__restrict__ Hb, float *__restrict__ X,
                                                const float *__restrict__ B, AxisTaps t, int nx, int ny, int nz)
{
    __shared__ float s[6][kTxChunk + 2 * (DVR_MAX_RADIUS + 1)];
    __shared__ float tg[DVR_MAX_RADIUS + 2], td1[DVR_MAX_RADIUS + 2], td2[DVR_MAX_RADIUS + 2];
    const int R = t.R, W = 2 * R + 1;
    const size_t N = (size_t)nx * (size_t)ny * (size_t)nz;
    const size_t rbase = (size_t)blockIdx.x * (size_t)nx;
    const int x0 = (int)blockIdx.y * kTxChunk;
    const int lo = max(0, x0 - R), hi = min(nx, x0 + kTxChunk + R);
    for (int p = (int)threadIdx.x; p < hi - lo; p += 256) {
#pragma unroll
        for (int f = 0; f < 6; ++f) s[f][p] = Hb[(size_t)f * N + rbase + (size_t)(lo + p)];
    }
    if (threadIdx.x <= (unsigned)R) {
        tg[threadIdx.x] = t.G[threadIdx.x];
        td1[threadIdx.x] = t.D1[threadIdx.x];
        td2[threadIdx.x] = t.D2[threadIdx.x];
    }
    __syncthreads();
    const int x = x0 + (int)threadIdx.x;
    if (x >= nx) return;
    const bool interior = x - 2 * R >= 0 && x + 2 * R <= nx - 1;
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int i0 = max(0, x - R), i1 = min(nx - 1, x + R);
    for (int i = i0; i <= i1; ++i) {
        const int d = x - i + R;
        float b0, b1, b2;
        if (interior) {
            const int m = x - i, am = m < 0 ? -m : m;
            b0 = tg[am];
            b1 = m > 0 ? td1[am] : (m < 0 ? -td1[am] : 0.f);
            b2 = td2[am];
        } else {
            b0 = B[(size_t)d * nx + i];
            b1 = B[(size_t)(W + d) * nx + i];
            b2 = B[(size_t)(2 * W + d) * nx + i];
        }
        const int li = i - lo;
        acc[0] = fmaf(b2, s[0][li], acc[0]);
        acc[1] = fmaf(b0, s[1][li], acc[1]);
        acc[2] = fmaf(b0, s[2][li], acc[2]);
        acc[3] = fmaf(b1, s[3][li], acc[3]);
        acc[4] = fmaf(b1, s[4][li], acc[4]);
        acc[5] = fmaf(b0, s[5][li], acc[5]);
    }
    const size_t o = rbase + (size_t)x;
#pragma unroll
    for (int k = 0; k < 6; ++k) X[(size_t)k * N + o] = acc[k];
}

// Fixed-radius form of k_tx_lds for the radii of the forward's fixed-radius kernels: an interior
// output unrolls its 2R + 1 taps (offset m = x - i from R down to -R: the rows in ascending order),
// so its weights are compile-time-indexed kernel arguments held in scalar registers and its LDS
// reads take immediate offsets; the others loop over the band table as k_tx_lds does.  The same
// products in the same order: the same bits.
template <int R>
__global__ __launch_bounds__(256) void k_tx_lds_r(const float *__restrict__ Hb, float *__restrict__ X,
                                                  const float *__restrict__ B, AxisTaps t, int nx, int ny, int nz)
{
    __shared__ float s[6][kTxChunk + 2 * (R + 1)];
    constexpr int W = 2 * R + 1;
    const size_t N = (size_t)nx * (size_t)ny * (size_t)nz;
    const size_t rbase = (size_t)blockIdx.x * (size_t)nx;
    const int x0 = (int)blockIdx.y * kTxChunk;
    const int lo = max(0, x0 - R), hi = min(nx, x0 + kTxChunk + R);
    for (int p = (int)threadIdx.x; p < hi - lo; p += 256) {
#pragma unroll
        for (int f = 0; f < 6; ++f) s[f][p] = Hb[(size_t)f * N + rbase + (size_t)(lo + p)];
    }
    __syncthreads();
    const int x = x0 + (int)threadIdx.x;
    if (x >= nx) return;
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (x - 2 * R >= 0 && x + 2 * R <= nx - 1) {
        const int lx = x - lo;
#pragma unroll
        for (int m = R; m >= -R; --m) {
            const int am = m < 0 ? -m : m;
            const float b0 = t.G[am], b1 = m > 0 ? t.D1[am] : (m < 0 ? -t.D1[am] : 0.f), b2 = t.D2[am];
            const int li = lx - m;
            acc[0] = fmaf(b2, s[0][li], acc[0]);
            acc[1] = fmaf(b0, s[1][li], acc[1]);
            acc[2] = fmaf(b0, s[2][li], acc[2]);
            acc[3] = fmaf(b1, s[3][li], acc[3]);
            acc[4] = fmaf(b1, s[4][li], acc[4]);
            acc[5] = fmaf(b0, s[5][li], acc[5]);
        }
    } else {
        const int i0 = max(0, x - R), i1 = min(nx - 1, x + R);
        for (int i = i0; i <= i1; ++i) {
            const int d = x - i + R;
            const float b0 = B[(size_t)d * nx + i], b1 = B[(size_t)(W + d) * nx + i];
            const float b2 = B[(size_t)(2 * W + d) * nx + i];
            const int li = i - lo;
            acc[0] = fmaf(b2, s[0][li], acc[0]);
            acc[1] = fmaf(b0, s[1][li], acc[1]);
            acc[2] = fmaf(b0, s[2][li], acc[2]);
            acc[3] = fmaf(b1, s[3][li], acc[3]);
            acc[4] = fmaf(b1, s[4][li], acc[4]);
            acc[5] = fmaf(b0, s[5][li], acc[5]);
        }
    }
    const size_t o = rbase + (size_t)x;
#pragma unroll
    for (int k = 0; k < 6; ++k) X[(size_t)k * N + o] = acc[k];
}

// the fixed-radius x transpose for radii 2..10, else the generic one
template <int R>
static void launch_tx_lds(const float *Hb, float *X, const float *B, const AxisTaps &t, const dvr_grid &g,
                          unsigned xchunks, hipStream_t st)
{
    if constexpr (R > 10) {
        hipLaunchKernelGGL(k_tx_lds, dim3((unsigned)g.ny * (unsigned)g.nz, xchunks), dim3(256), 0, st, Hb, X, B, t,
                           g.nx, g.ny, g.nz);
    } else {
        if (t.R != R) return launch_tx_lds<R + 1>(Hb, X, B, t, g, xchunks, st);
        hipLaunchKernelGGL(k_tx_lds_r<R>, dim3((unsigned)g.ny * (unsigned)g.nz, xchunks), dim3(256), 0, st, Hb, X, B,
                           t, g.nx, g.ny, g.nz);
    }
}

// y and z: each lane walks a run of kTRun consecutive outputs along the axis at one position of the
// other two (k_ty_run: blockIdx.y = run, blockIdx.z = z; k_tz_run: blockIdx.y = run), so every input
// row along the axis is loaded once per run rather than once per output it reaches (2R + 1 times:
// those re-reads through the caches bound a one-output-per-lane form).  Each output sums the rows i
// of its band in ascending order.  The band-table reads are uniform over the workgroup.
//
// y: the three z-groups: Y0 = G^T X_xx + (D2 G)^T X_yy + (D1 G)^T X_xy (z operator G),
// Y1 = G^T X_xz + (D1 G)^T X_yz (z operator D1 G), Y2 = G^T X_zz (z operator D2 G)
constexpr int kTyRun = 8, kTzRun = 4;
// waves per workgroup of the fixed-radius y and z transposes (y: one z-slice each; z: consecutive
// stretches of 64 plane positions): one-wave workgroups are limited by the workgroup slots of a CU
constexpr int kTWaves = 4;
template <int kTRun>
__global__ __launch_bounds__(64) void k_ty_run(const float *__restrict__ X, float *__restrict__ Y,
                                               const float *__restrict__ B, int nx, int ny, int nz, int R)
{
    const int x = (int)(blockIdx.x * 64u + threadIdx.x);
    if (x >= nx) return;
    const int yb = (int)blockIdx.y * kTRun, z = (int)blockIdx.z;
    const int nq = min(kTRun, ny - yb);
    const size_t plane = (size_t)nx * (size_t)ny, N = plane * (size_t)nz;
    const size_t col = (size_t)z * plane + (size_t)x;
    const int W = 2 * R + 1;
    float y0[kTRun], y1[kTRun], y2[kTRun];
#pragma unroll
    for (int q = 0; q < kTRun; ++q) y0[q] = y1[q] = y2[q] = 0.f;
    const int i0 = max(0, yb - R), i1 = min(ny - 1, yb + nq - 1 + R);
#pragma unroll 2
    for (int i = i0; i <= i1; ++i) {
        const size_t sidx = col + (size_t)i * nx;
        const float x0 = X[sidx], x1 = X[N + sidx], x2 = X[2 * N + sidx];
        const float x3 = X[3 * N + sidx], x4 = X[4 * N + sidx], x5 = X[5 * N + sidx];
#pragma unroll
        for (int q = 0; q < kTRun; ++q) {
            const int d = yb + q - i + R;
            if (q < nq && d >= 0 && d < W) {
                const float b0 = B[(size_t)d * ny + i], b1 = B[(size_t)(W + d) * ny + i];
                const float b2 = B[(size_t)(2 * W + d) * ny + i];
                y0[q] = fmaf(b0, x0, y0[q]);
                y0[q] = fmaf(b2, x1, y0[q]);
                y0[q] = fmaf(b1, x3, y0[q]);
                y1[q] = fmaf(b0, x4, y1[q]);
                y1[q] = fmaf(b1, x5, y1[q]);
                y2[q] = fmaf(b0, x2, y2[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kTRun; ++q) {
        if (q < nq) {
            const size_t o = col + (size_t)(yb + q) * nx;
            Y[o] = y0[q];
            Y[N + o] = y1[q];
            Y[2 * N + o] = y2[q];
        }
    }
}

// z: dL/dI += G^T Y0 + (D1 G)^T Y1 + (D2 G)^T Y2 along z
template <int kTRun>
__global__ __launch_bounds__(64) void k_tz_run(const float *__restrict__ Y, float *__restrict__ dvol,
                                               const float *__restrict__ B, int nx, int ny, int nz, int R)
{
    const size_t plane = (size_t)nx * (size_t)ny;
    const size_t e = (size_t)blockIdx.x * 64u + threadIdx.x;
    if (e >= plane) return;
    const int zb = (int)blockIdx.y * kTRun;
    const int nq = min(kTRun, nz - zb);
    const size_t N = plane * (size_t)nz;
    const int W = 2 * R + 1;
    float acc[kTRun];
#pragma unroll
    for (int q = 0; q < kTRun; ++q) acc[q] = 0.f;
    const int i0 = max(0, zb - R), i1 = min(nz - 1, zb + nq - 1 + R);
#pragma unroll 4
    for (int i = i0; i <= i1; ++i) {
        const size_t sidx = (size_t)i * plane + e;
        const float v0 = Y[sidx], v1 = Y[N + sidx], v2 = Y[2 * N + sidx];
#pragma unroll
        for (int q = 0; q < kTRun; ++q) {
            const int d = zb + q - i + R;
            if (q < nq && d >= 0 && d < W) {
                const float b0 = B[(size_t)d * nz + i], b1 = B[(size_t)(W + d) * nz + i];
                const float b2 = B[(size_t)(2 * W + d) * nz + i];
                acc[q] = fmaf(b0, v0, acc[q]);
                acc[q] = fmaf(b1, v1, acc[q]);
                acc[q] = fmaf(b2, v2, acc[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kTRun; ++q)
        if (q < nq) dvol[(size_t)(zb + q) * plane + e] += acc[q];
}

// Fixed-radius forms of k_ty_run and k_tz_run (R = 2..10): the walk over the K + 2R input rows of
// a run is unrolled, row j of the run (i = start - R + j) reaches outputs q with j - 2R <= q <= j at
// band offset d = q - j + 2R, both known at compile time, so only the axis ends and the run's
// ragged tail are tested at run time.  Same rows, products and order: the same bits.
template <int K, int R>
__global__ __launch_bounds__(64 * kTWaves) void k_ty_run_r(const float *__restrict__ X, float *__restrict__ Y,
                                                           const float *__restrict__ B, int nx, int ny, int nz)
{
    const int x = (int)(blockIdx.x * 64u + (threadIdx.x & 63u));
    const int z = (int)(blockIdx.z * kTWaves + (threadIdx.x >> 6));
    if (x >= nx || z >= nz) return;
    const int yb = (int)blockIdx.y * K;
    const int nq = min(K, ny - yb);
    const size_t plane = (size_t)nx * (size_t)ny, N = plane * (size_t)nz;
    const size_t col = (size_t)z * plane + (size_t)x;
    constexpr int W = 2 * R + 1;
    float y0[K], y1[K], y2[K];
#pragma unroll
    for (int q = 0; q < K; ++q) y0[q] = y1[q] = y2[q] = 0.f;
#pragma unroll
    for (int j = 0; j < K + 2 * R; ++j) {
        const int i = yb - R + j;
        if (i < 0 || i > ny - 1) continue;
        const size_t sidx = col + (size_t)i * nx;
        const float x0 = X[sidx], x1 = X[N + sidx], x2 = X[2 * N + sidx];
        const float x3 = X[3 * N + sidx], x4 = X[4 * N + sidx], x5 = X[5 * N + sidx];
#pragma unroll
        for (int q = (j - 2 * R > 0 ? j - 2 * R : 0); q <= (j < K - 1 ? j : K - 1); ++q) {
            if (q >= nq) break;
            const int d = q - j + 2 * R;
            const float b0 = B[(size_t)d * ny + i], b1 = B[(size_t)(W + d) * ny + i];
            const float b2 = B[(size_t)(2 * W + d) * ny + i];
            y0[q] = fmaf(b0, x0, y0[q]);
            y0[q] = fmaf(b2, x1, y0[q]);
            y0[q] = fmaf(b1, x3, y0[q]);
            y1[q] = fmaf(b0, x4, y1[q]);
            y1[q] = fmaf(b1, x5, y1[q]);
            y2[q] = fmaf(b0, x2, y2[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < K; ++q) {
        if (q < nq) {
            const size_t o = col + (size_t)(yb + q) * nx;
            Y[o] = y0[q];
            Y[N + o] = y1[q];
            Y[2 * N + o] = y2[q];
        }
    }
}

template <int K, int R>
__global__ __launch_bounds__(64 * kTWaves) void k_tz_run_r(const float *__restrict__ Y, float *__restrict__ dvol,
                                                           const float *__restrict__ B, int nx, int ny, int nz)
{
    const size_t plane = (size_t)nx * (size_t)ny;
    const size_t e = (size_t)blockIdx.x * (64u * kTWaves) + threadIdx.x;
    if (e >= plane) return;
    const int zb = (int)blockIdx.y * K;
    const int nq = min(K, nz - zb);
    const size_t N = plane * (size_t)nz;
    constexpr int W = 2 * R + 1;
    float acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.f;
#pragma unroll
    for (int j = 0; j < K + 2 * R; ++j) {
        const int i = zb - R + j;
        if (i < 0 || i > nz - 1) continue;
        const size_t sidx = (size_t)i * plane + e;
        const float v0 = Y[sidx], v1 = Y[N + sidx], v2 = Y[2 * N + sidx];
#pragma unroll
        for (int q = (j - 2 * R > 0 ? j - 2 * R : 0); q <= (j < K - 1 ? j : K - 1); ++q) {
            if (q >= nq) break;
            const int d = q - j + 2 * R;
            const float b0 = B[(size_t)d * nz + i], b1 = B[(size_t)(W + d) * nz + i];
            const float b2 = B[(size_t)(2 * W + d) * nz + i];
            acc[q] = fmaf(b0, v0, acc[q]);
            acc[q] = fmaf(b1, v1, acc[q]);
            acc[q] = fmaf(b2, v2, acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < K; ++q)
        if (q < nq) dvol[(size_t)(zb + q) * plane + e] += acc[q];
}

// the fixed-radius y and z transposes for radii 2..10 (runs of kTyRunR, kTzRunR), else the generic
// ones (runs of kTyRun, kTzRun)
constexpr int kTyRunR = 8, kTzRunR = 8;
static dim3 ty_grid(const dvr_grid &g, int K, int nw = 1)
{
    return dim3((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + K - 1) / K), (unsigned)((g.nz + nw - 1) / nw));
}
static dim3 tz_grid(const dvr_grid &g, int K, int nw = 1)
{
    const size_t plane = (size_t)g.nx * (size_t)g.ny;
    return dim3((unsigned)((plane + 64 * nw - 1) / (64 * nw)), (unsigned)((g.nz + K - 1) / K));
}

template <int R>
static void launch_ty(const float *X, float *Y, const float *B, int Ry, const dvr_grid &g, hipStream_t st)
{
    if constexpr (R > 10) {
        hipLaunchKernelGGL(k_ty_run<kTyRun>, ty_grid(g, kTyRun), dim3(64), 0, st, X, Y, B, g.nx, g.ny, g.nz, Ry);
    } else {
        if (Ry != R) return launch_ty<R + 1>(X, Y, B, Ry, g, st);
        hipLaunchKernelGGL((k_ty_run_r<kTyRunR, R>), ty_grid(g, kTyRunR, kTWaves), dim3(64 * kTWaves), 0, st, X, Y, B,
                           g.nx, g.ny, g.nz);
    }
}

template <int R>
static void launch_tz(const float *Y, float *dvol, const float *B, int Rz, const dvr_grid &g, hipStream_t st)
{
    if constexpr (R > 10) {
        hipLaunchKernelGGL(k_tz_run<kTzRun>, tz_grid(g, kTzRun), dim3(64), 0, st, Y, dvol, B, g.nx, g.ny, g.nz, Rz);
    } else {
        if (Rz != R) return launch_tz<R + 1>(Y, dvol, B, Rz, g, st);
        hipLaunchKernelGGL((k_tz_run_r<kTzRunR, R>), tz_grid(g, kTzRunR, kTWaves), dim3(64 * kTWaves), 0, st, Y, dvol,
                           B, g.nx, g.ny, g.nz);
    }
}

// dL/d|g|_max to the arg-max voxel's gradient: d|g|/dg = g / |g|
template <int DT>
__global__ void k_fb_gmax(const void *__restrict__ vol, const unsigned long long *__restrict__ key,
                          const float *__restrict__ dgmax, float *__restrict__ dgt, int nx, int ny, int nz, double ih0,
                          double ih1, double ih2)
{
    if (threadIdx.x != 0) return;
    const unsigned long long k = *key;
    const float dm = *dgmax;
    if (k == 0ull || dm == 0.f) return;
    const uint32_t v = 0xffffffffu - (uint32_t)(k & 0xffffffffull);
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const size_t N = (size_t)plane * (size_t)nz;
    const int z = (int)(v / plane), r = (int)(v - (uint32_t)z * plane);
    const int y = r / nx, x = r - y * nx;
    const size_t row = (size_t)z * plane + (size_t)y * nx;
    const double g0 = (ldd<DT>(vol, row + clampi(x + 1, 0, nx - 1)) - ldd<DT>(vol, row + clampi(x - 1, 0, nx - 1))) * ih0;
    const double g1 = (ldd<DT>(vol, (size_t)z * plane + (size_t)clampi(y + 1, 0, ny - 1) * nx + x) -
                       ldd<DT>(vol, (size_t)z * plane + (size_t)clampi(y - 1, 0, ny - 1) * nx + x)) * ih1;
    const double g2 = (ldd<DT>(vol, (size_t)clampi(z + 1, 0, nz - 1) * plane + (size_t)y * nx + x) -
                       ldd<DT>(vol, (size_t)clampi(z - 1, 0, nz - 1) * plane + (size_t)y * nx + x)) * ih2;
    const double gn = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
    if (!(gn > 0.0)) return;
    const double c = (double)dm / gn;
    dgt[v] = (float)((double)dgt[v] + c * g0);
    dgt[N + v] = (float)((double)dgt[N + v] + c * g1);
    dgt[2 * N + v] = (float)((double)dgt[2 * N + v] + c * g2);
}

// transposed clamped central difference along one axis at position c of n (stride st), times 1/(2h)
__device__ __forceinline__ float d1t(const float *__restrict__ a, size_t j, int c, int n, size_t st)
{
    float s = 0.f;
    if (c >= 1) s += a[j - st];
    if (c == n - 1) s += a[j];
    if (c + 1 <= n - 1) s -= a[j + st];
    if (c == 0) s -= a[j];
    return s;
}

__global__ __launch_bounds__(256) void k_fb_gradT(const float *__restrict__ dgt, float *__restrict__ dvol, int nx,
                                                  int ny, int nz, float ih0, float ih1, float ih2)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= plane) return;
    const int z = (int)blockIdx.y;
    const int y = (int)(e / (uint32_t)nx), x = (int)(e - (uint32_t)y * nx);
    const size_t N = (size_t)plane * (size_t)nz;
    const size_t j = (size_t)z * plane + e;
    float acc = ih0 * d1t(dgt, j, x, nx, 1);
    acc = fmaf(ih1, d1t(dgt + N, j, y, ny, (size_t)nx), acc);
    acc = fmaf(ih2, d1t(dgt + 2 * N, j, z, nz, (size_t)plane), acc);
    dvol[j] += acc;
}

__global__ void k_zero_u64(unsigned long long *p)
{
    if (threadIdx.x == 0) *p = 0ull;
}

// ------------------------------------------------------------------------------------------------
static size_t al256(size_t b) { return (b + 255u) & ~(size_t)255u; }

struct BwdWs {
    unsigned long long *key;
    float *zws;   // 3N: z-filtered fields of the Hessian recomputation; then Y (3N)
    float *H;     // 6N per scale: H of every scale; a scale's block then holds X (6N)
    float *Hb;    // 6N: dL/dH of the current scale
    float *dgt;   // 3N: dL/dg total
    double *best; // N
    uint8_t *win; // N
    float *band;  // per scale and axis: [3][n_a][2 R_a + 1]
};

static size_t band_floats(const dvr_grid &g, const FeatBwdPlan &p)
{
    const int n[3] = {g.nx, g.ny, g.nz};
    size_t t = 0;
    for (int s = 0; s < p.nsigma; ++s)
        for (int a = 0; a < 3; ++a) t += (size_t)3 * n[a] * (2 * p.taps[s].ax[a].R + 1);
    return t;
}

static BwdWs carve(void *ws, const dvr_grid &g, const FeatBwdPlan &p, size_t *total)
{
    const size_t N = (size_t)g.nx * g.ny * g.nz;
    char *b = (char *)ws;
    size_t o = 0;
    BwdWs w;
    w.key = (unsigned long long *)(b + o);
    o += 256;
    w.zws = (float *)(b + o);
    o += al256(12 * N);
    w.H = (float *)(b + o);
    o += al256(24 * N * (size_t)p.nsigma);
    w.Hb = (float *)(b + o);
    o += al256(24 * N);
    w.dgt = (float *)(b + o);
    o += al256(12 * N);
    w.best = (double *)(b + o);
    o += al256(8 * N);
    w.win = (uint8_t *)(b + o);
    o += al256(N);
    w.band = (float *)(b + o);
    o += al256(4 * band_floats(g, p));
    if (total) *total = o;
    return w;
}

size_t features_bwd_ws_bytes(const dvr_grid &g, const FeatBwdPlan &p)
{
    size_t t = 0;
    carve(nullptr, g, p, &t);
    return t;
}

hipError_t launch_features_backward(const void *vol, int vol_dt, const dvr_grid &g, const FeatBwdPlan &p,
                                    const float *dfeat, const float *dgmax, float *dvol, void *ws, hipStream_t st)
{
    const BwdWs w = carve(ws, g, p, nullptr);
    const int n[3] = {g.nx, g.ny, g.nz};
    const uint32_t plane = (uint32_t)g.nx * (uint32_t)g.ny;
    const uint32_t N = plane * (uint32_t)g.nz;
    const dim3 pgrid((plane + 255) / 256, g.nz);
    const dim3 lgrid((plane + 256 * kFbSub - 1) / (256 * kFbSub), g.nz);  // k_fb_local: kFbSub runs per workgroup
    const dim3 vgrid((N + 255) / 256);
    hipError_t e;
    // band tables of every scale and axis (one launch per scale)
    float *bt[DVR_MAX_SIGMA][3];
    {
        float *b = w.band;
        for (int s = 0; s < p.nsigma; ++s) {
            BandJob j;
            int most = 0;
            for (int a = 0; a < 3; ++a) {
                bt[s][a] = b;
                j.t[a] = p.taps[s].ax[a];
                j.n[a] = n[a];
                j.B[a] = b;
                const int cnt = 3 * n[a] * (2 * p.taps[s].ax[a].R + 1);
                most = cnt > most ? cnt : most;
                b += cnt;
            }
            hipLaunchKernelGGL(k_band, dim3((most + 255) / 256, 3), dim3(256), 0, st, j);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, w.key);
    // every scale's Hessian, and the winning scale of each voxel
    for (int s = 0; s < p.nsigma; ++s) {
        float *Hs = w.H + (size_t)6 * N * s;
        if ((e = launch_hessian(vol, vol_dt, g, p.taps[s], w.zws, Hs, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_fb_win, vgrid, dim3(256), 0, st, Hs, w.best, w.win, s, p.sigma2[s], p.inv2a2, p.inv2b2,
                           p.inv2c2, N);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int s = 0; s < p.nsigma; ++s) {
        float *Hs = w.H + (size_t)6 * N * s;
        if (vol_dt == DVR_F32)
            hipLaunchKernelGGL(k_fb_local<DVR_F32>, lgrid, dim3(256), 0, st, vol, Hs, dfeat, w.win, w.Hb, w.dgt, w.key,
                               s, p.sigma2[s], p.inv2a2, p.inv2b2, p.inv2c2, g.nx, g.ny, g.nz, p.inv2h[0], p.inv2h[1],
                               p.inv2h[2]);
        else
            hipLaunchKernelGGL(k_fb_local<DVR_F16>, lgrid, dim3(256), 0, st, vol, Hs, dfeat, w.win, w.Hb, w.dgt, w.key,
                               s, p.sigma2[s], p.inv2a2, p.inv2b2, p.inv2c2, g.nx, g.ny, g.nz, p.inv2h[0], p.inv2h[1],
                               p.inv2h[2]);
        float *X = Hs, *Y = w.zws;  // this scale's H is no longer needed
        const unsigned xchunks = (unsigned)((g.nx + kTxChunk - 1) / kTxChunk);
        if (xchunks <= 65535u)
            launch_tx_lds<2>(w.Hb, X, bt[s][0], p.taps[s].ax[0], g, xchunks, st);
        else
            hipLaunchKernelGGL(k_tx, pgrid, dim3(256), 0, st, w.Hb, X, bt[s][0], g.nx, g.ny, g.nz, p.taps[s].ax[0].R);
        launch_ty<2>(X, Y, bt[s][1], p.taps[s].ax[1].R, g, st);
        launch_tz<2>(Y, dvol, bt[s][2], p.taps[s].ax[2].R, g, st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (vol_dt == DVR_F32)
        hipLaunchKernelGGL(k_fb_gmax<DVR_F32>, dim3(1), dim3(64), 0, st, vol, w.key, dgmax, w.dgt, g.nx, g.ny, g.nz,
                           p.inv2h[0], p.inv2h[1], p.inv2h[2]);
    else
        hipLaunchKernelGGL(k_fb_gmax<DVR_F16>, dim3(1), dim3(64), 0, st, vol, w.key, dgmax, w.dgt, g.nx, g.ny, g.nz,
                           p.inv2h[0], p.inv2h[1], p.inv2h[2]);
    hipLaunchKernelGGL(k_fb_gradT, pgrid, dim3(256), 0, st, w.dgt, dvol, g.nx, g.ny, g.nz, (float)p.inv2h[0],
                       (float)p.inv2h[1], (float)p.inv2h[2]);
    return hipGetLastError();
}

}  // namespace dvr
