// C ABI of libdvr: argument validation, workspace sizing, tap tables, dispatch to the launchers.
// Nothing is enqueued unless every argument checks out; errors are reported by status code and a
// thread-local message.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "common.hpp"
#include "render_args.hpp"

#include "host.hpp"

namespace dvr {
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t st);
}

namespace dvr::host {

thread_local std::string g_err;

dvr_status fail(dvr_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

dvr_status dev_fail(hipError_t e, const char *what)
{
    return fail(DVR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
bool finite_pos(float v) { return isfinite(v) && v > 0.f; }

dvr_status check_grid(const dvr_grid *g)
{
    if (!g) return fail(DVR_E_NULL, "grid is NULL");
    if (g->nx < 2 || g->ny < 2 || g->nz < 2)
        return fail(DVR_E_INVALID_ARG, "grid dims must be >= 2 (got %d x %d x %d)", g->nx, g->ny, g->nz);
    if (!finite_pos(g->hx) || !finite_pos(g->hy) || !finite_pos(g->hz))
        return fail(DVR_E_INVALID_ARG, "spacing must be finite and > 0");
    const double N = (double)g->nx * g->ny * g->nz;
    if (N * 32.0 > 4294967295.0)
        return fail(DVR_E_INVALID_ARG, "volume of %.0f voxels exceeds the 32-bit addressing limit (2^27 voxels)", N);
    return DVR_OK;
}

int64_t nvox(const dvr_grid *g) { return (int64_t)g->nx * g->ny * g->nz; }

int gauss_radius(double sigma_vox)
{
    const int r = (int)floor(3.0 * sigma_vox + 0.5);
    return r < 1 ? 1 : r;
}

dvr_status check_fparams(const dvr_grid *g, const dvr_feature_params *fp)
{
    if (!fp) return fail(DVR_E_NULL, "feature params are NULL");
    if (fp->nsigma < 1 || fp->nsigma > DVR_MAX_SIGMA)
        return fail(DVR_E_INVALID_ARG, "nsigma must be in [1, %d]", DVR_MAX_SIGMA);
    const double h[3] = {g->hx, g->hy, g->hz};
    for (int s = 0; s < fp->nsigma; ++s) {
        if (!finite_pos(fp->sigma_mm[s])) return fail(DVR_E_INVALID_ARG, "sigma_mm[%d] must be finite and > 0", s);
        for (int a = 0; a < 3; ++a)
            if (gauss_radius((double)fp->sigma_mm[s] / h[a]) > DVR_MAX_RADIUS)
                return fail(DVR_E_INVALID_ARG, "Gaussian radius of sigma_mm[%d] on axis %d exceeds %d", s, a,
                            DVR_MAX_RADIUS);
    }
    if (!finite_pos(fp->alpha) || !finite_pos(fp->beta)) return fail(DVR_E_INVALID_ARG, "alpha and beta must be > 0");
    if (!isfinite(fp->c)) return fail(DVR_E_INVALID_ARG, "c must be finite");
    if (!isfinite(fp->eig_gap_fp64) || fp->eig_gap_fp64 < 0.f)
        return fail(DVR_E_INVALID_ARG, "eig_gap_fp64 must be finite and >= 0");
    return DVR_OK;
}

dvr_status check_feat_buf(const dvr_features_buf *f, bool need_writable)
{
    (void)need_writable;
    if (!f) return fail(DVR_E_NULL, "features buffer is NULL");
    if (f->dtype != DVR_F32 && f->dtype != DVR_F16) return fail(DVR_E_UNSUPPORTED, "feature dtype must be F32 or F16");
    if (f->layout != DVR_PLANAR && f->layout != DVR_INTERLEAVED && f->layout != DVR_SPLIT && f->layout != DVR_QUAD)
        return fail(DVR_E_UNSUPPORTED, "feature layout must be PLANAR, INTERLEAVED, SPLIT or QUAD");
    if (!f->grad || !f->gmax) return fail(DVR_E_NULL, "features grad/gmax is NULL");
    if (!aligned16(f->grad)) return fail(DVR_E_ALIGN, "features grad is not 16-byte aligned");
    if (((uintptr_t)f->gmax & 3u) != 0) return fail(DVR_E_ALIGN, "gmax is not 4-byte aligned");
    if (f->layout == DVR_PLANAR) {
        if (!f->kappa || !f->ves) return fail(DVR_E_NULL, "planar features need kappa and ves");
        if (!aligned16(f->kappa) || !aligned16(f->ves)) return fail(DVR_E_ALIGN, "kappa/ves not 16-byte aligned");
    }
    if (f->layout == DVR_SPLIT || f->layout == DVR_QUAD) {
        if (!f->ves) return fail(DVR_E_NULL, "split and quad features need ves");
        if (!aligned16(f->ves)) return fail(DVR_E_ALIGN, "ves not 16-byte aligned");
    }
    if (f->layout == DVR_QUAD) {
        if (!f->iquad) return fail(DVR_E_NULL, "quad features need iquad");
        if (!aligned16(f->iquad)) return fail(DVR_E_ALIGN, "iquad not 16-byte aligned");
    }
    if (((uintptr_t)f->bricks & 7u) != 0) return fail(DVR_E_ALIGN, "bricks is not 8-byte aligned");
    return DVR_OK;
}

int nbricks(int n) { return (n - 1 + DVR_BRICK - 1) / DVR_BRICK; }

// every feature array is addressed with 32-bit byte offsets
dvr_status check_feat_size(const dvr_grid *g, const dvr_features_buf *f)
{
    const uint64_t es = f->dtype == DVR_F32 ? 4u : 2u;
    const uint64_t per = f->layout == DVR_INTERLEAVED ? 8u * es : (f->layout == DVR_PLANAR ? es : 4u * es);
    if ((uint64_t)g->nx * (uint64_t)g->ny * (uint64_t)g->nz * per >= ((uint64_t)1 << 32))
        return fail(DVR_E_INVALID_ARG, "feature arrays of this grid exceed 4 GiB (32-bit offsets)");
    return DVR_OK;
}

void axis_taps(double sigma_vox, double h, dvr::AxisTaps &t)
{
    const int r = gauss_radius(sigma_vox);
    const int R = r + 1;
    double w[2 * DVR_MAX_RADIUS + 1];
    double sum = 0.0;
    for (int j = -r; j <= r; ++j) {
        w[j + r] = exp(-(double)j * j / (2.0 * sigma_vox * sigma_vox));
        sum += w[j + r];
    }
    for (int j = 0; j <= 2 * r; ++j) w[j] /= sum;
    auto W = [&](int j) -> double { return (j < -r || j > r) ? 0.0 : w[j + r]; };
    memset(&t, 0, sizeof t);
    t.R = R;
    for (int j = 0; j <= R; ++j) {
        t.G[j] = (float)W(j);
        t.D2[j] = (float)((W(j - 1) - 2.0 * W(j) + W(j + 1)) / (h * h));
        if (j >= 1) t.D1[j] = (float)((W(j - 1) - W(j + 1)) / (2.0 * h));
    }
    for (int m = -R; m <= R + 1; ++m) {
        const double e = W(m - 1) - W(m);
        t.E1[m + R] = (float)(e / (2.0 * h));
        t.E2[m + R] = (float)(e / (h * h));
    }
}

size_t features_ws_bytes(const dvr_grid *g) { return 256 + (size_t)12 * (size_t)nvox(g); }

}  // namespace dvr::host

using namespace dvr::host;

extern "C" {

int32_t dvr_version(void) { return 1; }

const char *dvr_last_error(void) { return g_err.c_str(); }

dvr_status dvr_normalize_workspace(int64_t n, size_t *bytes)
{
    if (!bytes) return fail(DVR_E_NULL, "bytes is NULL");
    if (n <= 0) return fail(DVR_E_INVALID_ARG, "n must be > 0");
    *bytes = 256;
    return DVR_OK;
}

dvr_status dvr_normalize(const void *raw, int32_t raw_dtype, void *out, int32_t out_dtype, int64_t n, void *ws,
                         size_t ws_bytes, hipStream_t stream)
{
    if (!raw || !out || !ws) return fail(DVR_E_NULL, "raw, out and ws must be non-NULL");
    if (!aligned16(raw) || !aligned16(out) || !aligned16(ws)) return fail(DVR_E_ALIGN, "pointers must be 16-byte aligned");
    if (n <= 0) return fail(DVR_E_INVALID_ARG, "n must be > 0");
    if (raw_dtype != DVR_U16 && raw_dtype != DVR_F32 && raw_dtype != DVR_F16)
        return fail(DVR_E_UNSUPPORTED, "raw dtype must be U16, F32 or F16");
    if (out_dtype != DVR_F16 && out_dtype != DVR_F32) return fail(DVR_E_UNSUPPORTED, "out dtype must be F16 or F32");
    if (ws_bytes < 256) return fail(DVR_E_WORKSPACE, "workspace must hold 256 bytes");
    hipError_t e = dvr::launch_normalize(raw, raw_dtype, out, out_dtype, n, (uint32_t *)ws, stream);
    return e == hipSuccess ? DVR_OK : dev_fail(e, "normalize launch");
}

dvr_status dvr_normalize_noalloc(const void *raw, int32_t raw_dtype, void *out, int32_t out_dtype, int64_t n,
                                 hipStream_t stream)
{
    if (!raw || !out) return fail(DVR_E_NULL, "raw and out must be non-NULL");
    if (!aligned16(raw) || !aligned16(out)) return fail(DVR_E_ALIGN, "raw and out must be 16-byte aligned");
    if (n <= 0) return fail(DVR_E_INVALID_ARG, "n must be > 0");
    if (raw_dtype != DVR_U16 && raw_dtype != DVR_F32 && raw_dtype != DVR_F16)
        return fail(DVR_E_UNSUPPORTED, "raw dtype must be U16, F32 or F16");
    if (out_dtype != DVR_F16 && out_dtype != DVR_F32) return fail(DVR_E_UNSUPPORTED, "out dtype must be F16 or F32");
    // the reduction needs the two words of dvr_normalize's workspace whatever n is; refuse anything
    // that would need more than the static scratch holds
    size_t need = 0;
    dvr_status s = dvr_normalize_workspace(n, &need);
    if (s) return s;
    if (need > dvr::normalize_scratch_bytes())
        return fail(DVR_E_WORKSPACE, "normalize needs %zu bytes of scratch; the static scratch holds %zu", need,
                    dvr::normalize_scratch_bytes());
    void *scratch = nullptr;
    hipError_t e = dvr::normalize_scratch(&scratch);
    if (e != hipSuccess) return dev_fail(e, "static scratch lookup");
    e = dvr::launch_normalize(raw, raw_dtype, out, out_dtype, n, (uint32_t *)scratch, stream);
    return e == hipSuccess ? DVR_OK : dev_fail(e, "normalize launch");
}

dvr_status dvr_denoise_workspace(const dvr_grid *grid, int32_t mode, size_t *bytes)
{
    dvr_status s = check_grid(grid);
    if (s) return s;
    if (!bytes) return fail(DVR_E_NULL, "bytes is NULL");
    if (mode != DVR_DENOISE_GAUSS && mode != DVR_DENOISE_MEDIAN3) return fail(DVR_E_INVALID_ARG, "unknown denoise mode");
    *bytes = mode == DVR_DENOISE_GAUSS ? (size_t)8 * (size_t)nvox(grid) : 0;
    return DVR_OK;
}

dvr_status dvr_denoise(const void *vol, int32_t dtype, const dvr_grid *grid, int32_t mode, float sigma_mm, void *out,
                       void *ws, size_t ws_bytes, hipStream_t stream)
{
    dvr_status s = check_grid(grid);
    if (s) return s;
    if (mode != DVR_DENOISE_GAUSS && mode != DVR_DENOISE_MEDIAN3) return fail(DVR_E_INVALID_ARG, "unknown denoise mode");
    if (!vol || !out) return fail(DVR_E_NULL, "vol and out must be non-NULL");
    if (vol == out) return fail(DVR_E_INVALID_ARG, "out must not alias vol");
    if (!aligned16(vol) || !aligned16(out)) return fail(DVR_E_ALIGN, "vol and out must be 16-byte aligned");
    if (dtype != DVR_F32 && dtype != DVR_F16) return fail(DVR_E_UNSUPPORTED, "dtype must be F32 or F16");
    int r[3] = {0, 0, 0};
    float w[3][DVR_MAX_RADIUS + 1] = {};
    if (mode == DVR_DENOISE_GAUSS) {
        if (!finite_pos(sigma_mm)) return fail(DVR_E_INVALID_ARG, "sigma_mm must be > 0");
        const double h[3] = {grid->hx, grid->hy, grid->hz};
        for (int a = 0; a < 3; ++a) {
            const double sv = sigma_mm / h[a];
            if (gauss_radius(sv) > DVR_MAX_RADIUS) return fail(DVR_E_INVALID_ARG, "Gaussian radius beyond DVR_MAX_RADIUS");
            dvr::AxisTaps t;
            axis_taps(sv, h[a], t);
            r[a] = t.R - 1;
            for (int j = 0; j <= r[a]; ++j) w[a][j] = t.G[j];
        }
        if (!ws) return fail(DVR_E_WORKSPACE, "workspace is NULL");
        if (!aligned16(ws)) return fail(DVR_E_ALIGN, "workspace is not 16-byte aligned");
        if (ws_bytes < (size_t)8 * (size_t)nvox(grid)) return fail(DVR_E_WORKSPACE, "workspace too small");
    }
    hipError_t e = dvr::launch_denoise(vol, dtype, *grid, mode, r, w, out, (float *)ws, stream);
    return e == hipSuccess ? DVR_OK : dev_fail(e, "denoise launch");
}

dvr_status dvr_histogram(const void *vol, int32_t dtype, int64_t n, float floor_, uint32_t *hist, uint32_t *used,
                         hipStream_t stream)
{
    if (!vol || !hist) return fail(DVR_E_NULL, "vol and hist must be non-NULL");
    if (!aligned16(vol) || ((uintptr_t)hist & 3u) || ((uintptr_t)used & 3u))
        return fail(DVR_E_ALIGN, "vol must be 16-byte aligned, hist and used 4-byte aligned");
    if (dtype != DVR_F32 && dtype != DVR_F16) return fail(DVR_E_UNSUPPORTED, "dtype must be F32 or F16");
    if (n <= 0 || n >= ((int64_t)1 << 32)) return fail(DVR_E_INVALID_ARG, "n must be in [1, 2^32)");
    if (!isfinite(floor_)) return fail(DVR_E_INVALID_ARG, "floor must be finite");
    hipError_t e = dvr::launch_histogram(vol, dtype, n, floor_, hist, used, stream);
    return e == hipSuccess ? DVR_OK : dev_fail(e, "histogram launch");
}

dvr_status dvr_tissue_peaks(const uint32_t *hist, int32_t min_sep, dvr_peaks *out, hipStream_t stream)
{
    if (!hist || !out) return fail(DVR_E_NULL, "hist and out must be non-NULL");
    if (((uintptr_t)hist & 3u) || ((uintptr_t)out & 3u)) return fail(DVR_E_ALIGN, "hist and out must be 4-byte aligned");
    if (min_sep < 1 || min_sep > 255) return fail(DVR_E_INVALID_ARG, "min_sep must be in [1, 255]");
    hipError_t e = dvr::launch_peaks(hist, min_sep, out, stream);
    return e == hipSuccess ? DVR_OK : dev_fail(e, "peaks launch");
}

dvr_status dvr_tissue_tf(const dvr_peaks *peaks, const dvr_tissue_tf_params *params, float *knots, float *rgba,
                         hipStream_t stream)
{
    if (!peaks || !params || !knots || !rgba) return fail(DVR_E_NULL, "peaks, params, knots and rgba must be non-NULL");
    if (((uintptr_t)peaks & 3u) || ((uintptr_t)knots & 3u) || !aligned16(rgba))
        return fail(DVR_E_ALIGN, "peaks and knots 4-byte, rgba 16-byte aligned");
    for (int c = 0; c < 3; ++c) {
        if (!(params->tau[c] >= 0.f) || !isfinite(params->tau[c])) return fail(DVR_E_INVALID_ARG, "tau must be >= 0");
        for (int k = 0; k < 3; ++k)
            if (!(params->rgb[c][k] >= 0.f && params->rgb[c][k] <= 1.f) || !(params->rgb_hi[k] >= 0.f && params->rgb_hi[k] <= 1.f))
                return fail(DVR_E_INVALID_ARG, "colours must be in [0, 1]");
    }
    if (!(params->tau_hi >= 0.f) || !isfinite(params->tau_hi)) return fail(DVR_E_INVALID_ARG, "tau_hi must be >= 0");
    hipError_t e = dvr::launch_tissue_tf(peaks, *params, knots, rgba, stream);
    return e == hipSuccess ? DVR_OK : dev_fail(e, "tissue TF launch");
}

dvr_status dvr_features_workspace(const dvr_grid *grid, const dvr_feature_params *fp, size_t *bytes)
{
    dvr_status s = check_grid(grid);
    if (s) return s;
    if ((s = check_fparams(grid, fp))) return s;
    if (!bytes) return fail(DVR_E_NULL, "bytes is NULL");
    *bytes = features_ws_bytes(grid);
    return DVR_OK;
}

dvr_status dvr_bricks_count(const dvr_grid *grid, int64_t *count)
{
    dvr_status s = check_grid(grid);
    if (s) return s;
    if (!count) return fail(DVR_E_NULL, "count is NULL");
    *count = (int64_t)nbricks(grid->nx) * nbricks(grid->ny) * nbricks(grid->nz);
    return DVR_OK;
}

dvr_status dvr_bricks_bytes(const dvr_grid *grid, size_t *bytes)
{
    int64_t nb = 0;
    dvr_status s = dvr_bricks_count(grid, &nb);
    if (s) return s;
    if (!bytes) return fail(DVR_E_NULL, "bytes is NULL");
    *bytes = (size_t)nb * 8u + (size_t)((nb + 31) / 32) * 4u;
    return DVR_OK;
}

dvr_status dvr_features(const void *vol, int32_t vol_dtype, const dvr_grid *grid, const dvr_feature_params *fp,
                        const dvr_features_buf *out, void *ws, size_t ws_bytes, hipStream_t stream)
{
    dvr_status s = check_grid(grid);
    if (s) return s;
    if ((s = check_fparams(grid, fp))) return s;
    if ((s = check_feat_buf(out, true))) return s;
    if ((s = check_feat_size(grid, out))) return s;
    if (!vol) return fail(DVR_E_NULL, "vol is NULL");
    if (!aligned16(vol)) return fail(DVR_E_ALIGN, "vol is not 16-byte aligned");
    if (vol_dtype != DVR_F32 && vol_dtype != DVR_F16) return fail(DVR_E_UNSUPPORTED, "vol dtype must be F32 or F16");
    if (!ws) return fail(DVR_E_WORKSPACE, "workspace is NULL");
    if (!aligned16(ws)) return fail(DVR_E_ALIGN, "workspace is not 16-byte aligned");
    if (ws_bytes < features_ws_bytes(grid))
        return fail(DVR_E_WORKSPACE, "workspace of %zu bytes is smaller than the required %zu", ws_bytes,
                    features_ws_bytes(grid));
    // QUAD runs the SPLIT pass with V written plainly into the iquad array, then builds both quads
    dvr_features_buf run = *out;
    if (out->layout == DVR_QUAD) {
        if (vol_dtype != out->dtype) return fail(DVR_E_UNSUPPORTED, "QUAD features need the volume in the feature dtype");
        run.layout = DVR_SPLIT;
        run.ves = out->iquad;
    }
    float *scalars = (float *)ws;
    float *fields = (float *)((char *)ws + 256);
    hipError_t e = dvr::launch_init_scalars(out->gmax, scalars, stream);
    if (e != hipSuccess) return dev_fail(e, "features init");
    const double h[3] = {grid->hx, grid->hy, grid->hz};
    for (int pass = (fp->c > 0.f ? 1 : 0); pass < 2; ++pass) {
        for (int sc = 0; sc < fp->nsigma; ++sc) {
            dvr::ScaleTaps taps;
            const double sg = fp->sigma_mm[sc];
            for (int a = 0; a < 3; ++a) axis_taps(sg / h[a], h[a], taps.ax[a]);
            taps.sigma2 = (float)(sg * sg);
            e = dvr::launch_features_scale(vol, vol_dtype, *grid, taps, sc, sc == fp->nsigma - 1, *fp, run, fields,
                                           scalars, pass == 0, stream);
            if (e != hipSuccess) return dev_fail(e, "features launch");
        }
    }
    if (out->bricks) {
        e = dvr::launch_bricks(vol, vol_dtype, *grid, *out, stream);
        if (e != hipSuccess) return dev_fail(e, "brick table launch");
    }
    if (out->layout == DVR_QUAD) {
        // V quads from the plain V first, then the intensity quads over it
        e = dvr::launch_quads(out->iquad, out->ves, *grid, out->dtype, stream);
        if (e == hipSuccess) e = dvr::launch_quads(vol, out->iquad, *grid, out->dtype, stream);
        if (e != hipSuccess) return dev_fail(e, "quad launch");
    }
    return DVR_OK;
}

static dvr_status feat_bwd_plan(const dvr_grid *grid, const dvr_feature_params *fp, dvr::FeatBwdPlan &p)
{
    dvr_status s = check_grid(grid);
    if (s) return s;
    if ((s = check_fparams(grid, fp))) return s;
    if (!(fp->c > 0.f)) return fail(DVR_E_INVALID_ARG, "the feature adjoint needs Frangi's c > 0 (got %g)", (double)fp->c);
    const double h[3] = {grid->hx, grid->hy, grid->hz};
    memset(&p, 0, sizeof p);
    p.nsigma = fp->nsigma;
    for (int sc = 0; sc < fp->nsigma; ++sc) {
        const double sg = fp->sigma_mm[sc];
        for (int a = 0; a < 3; ++a) axis_taps(sg / h[a], h[a], p.taps[sc].ax[a]);
        p.taps[sc].sigma2 = (float)(sg * sg);
        p.sigma2[sc] = sg * sg;
    }
    const double al = fp->alpha, be = fp->beta, c = fp->c;
    p.inv2a2 = 1.0 / (2.0 * al * al);
    p.inv2b2 = 1.0 / (2.0 * be * be);
    p.inv2c2 = 1.0 / (2.0 * c * c);
    for (int a = 0; a < 3; ++a) p.inv2h[a] = 1.0 / (2.0 * h[a]);
    return DVR_OK;
}

dvr_status dvr_features_backward_workspace(const dvr_grid *grid, const dvr_feature_params *fp, size_t *bytes)
{
    dvr::FeatBwdPlan p;
    dvr_status s = feat_bwd_plan(grid, fp, p);
    if (s) return s;
    if (!bytes) return fail(DVR_E_NULL, "bytes is NULL");
    *bytes = dvr::features_bwd_ws_bytes(*grid, p);
    return DVR_OK;
}

dvr_status dvr_features_backward(const void *vol, int32_t vol_dtype, const dvr_grid *grid,
                                 const dvr_feature_params *fp, const dvr_feature_grads *fg, float *dL_dvol, void *ws,
                                 size_t ws_bytes, hipStream_t stream)
{
    dvr::FeatBwdPlan p;
    dvr_status s = feat_bwd_plan(grid, fp, p);
    if (s) return s;
    if (!vol) return fail(DVR_E_NULL, "vol is NULL");
    if (!aligned16(vol)) return fail(DVR_E_ALIGN, "vol is not 16-byte aligned");
    if (vol_dtype != DVR_F32 && vol_dtype != DVR_F16) return fail(DVR_E_UNSUPPORTED, "vol dtype must be F32 or F16");
    if (!fg || !fg->dfeat || !fg->dgmax) return fail(DVR_E_NULL, "feature gradients are required");
    if (((uintptr_t)fg->dfeat & 3u) || ((uintptr_t)fg->dgmax & 3u))
        return fail(DVR_E_ALIGN, "feature gradient buffers misaligned");
    if (!dL_dvol) return fail(DVR_E_NULL, "dL_dvol is NULL");
    if ((uintptr_t)dL_dvol & 3u) return fail(DVR_E_ALIGN, "dL_dvol is not 4-byte aligned");
    const size_t need = dvr::features_bwd_ws_bytes(*grid, p);
    if (!ws) return fail(DVR_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255u)) return fail(DVR_E_ALIGN, "workspace is not 256-byte aligned");
    if (ws_bytes < need)
        return fail(DVR_E_WORKSPACE, "workspace of %zu bytes is smaller than the required %zu", ws_bytes, need);
    hipError_t e = dvr::launch_features_backward(vol, vol_dtype, *grid, p, fg->dfeat, fg->dgmax, dL_dvol, ws, stream);
    return e == hipSuccess ? DVR_OK : dev_fail(e, "feature adjoint launch");
}

}  // extern "C"

dvr_status dvr::host::build_render_args(const void *vol, int32_t vol_dtype, const dvr_grid *grid,
                                    const dvr_features_buf *feat, const dvr_tf *tf, const dvr_render_params *rp,
                                    const dvr_camera *cams, int32_t ncam, dvr::RenderArgs &a, dvr::KCam *kc)
{
    dvr_status s = check_grid(grid);
    if (s) return s;
    if ((s = check_feat_buf(feat, false))) return s;
    if ((s = check_feat_size(grid, feat))) return s;
    if (feat->layout != DVR_INTERLEAVED && feat->layout != DVR_QUAD) {
        if (!vol) return fail(DVR_E_NULL, "vol is NULL (planar and split features sample it)");
        if (!aligned16(vol)) return fail(DVR_E_ALIGN, "vol is not 16-byte aligned");
        if (vol_dtype != feat->dtype) return fail(DVR_E_UNSUPPORTED, "planar render needs vol dtype == feature dtype");
    }
    if (!tf) return fail(DVR_E_NULL, "tf is NULL");
    if (tf->K < 2 || tf->K > 64) return fail(DVR_E_INVALID_ARG, "tf K must be in [2, 64]");
    if (!tf->knots || !tf->rgba) return fail(DVR_E_NULL, "tf knots/rgba NULL");
    if (!aligned16(tf->rgba) || ((uintptr_t)tf->knots & 3u)) return fail(DVR_E_ALIGN, "tf rgba must be 16-byte aligned");
    if (!rp) return fail(DVR_E_NULL, "render params NULL");
    if (!(rp->lambda_g >= 0.f && rp->lambda_g <= 1.f) || !(rp->lambda_k >= 0.f && rp->lambda_k <= 1.f))
        return fail(DVR_E_INVALID_ARG, "lambda_g and lambda_k must be in [0, 1]");
    if (!finite_pos(rp->kappa0)) return fail(DVR_E_INVALID_ARG, "kappa0 must be > 0");
    if (!(rp->lambda_v >= 0.f) || !isfinite(rp->lambda_v)) return fail(DVR_E_INVALID_ARG, "lambda_v must be >= 0");
    if (!(rp->step_vox >= 1.0f / 64.0f) || !isfinite(rp->step_vox))
        return fail(DVR_E_INVALID_ARG, "step_vox must be >= 1/64 (got %g)", (double)rp->step_vox);
    if (!(rp->et_alpha < 1.f) || !isfinite(rp->et_alpha)) return fail(DVR_E_INVALID_ARG, "et_alpha must be < 1");
    if (!cams || ncam < 1) return fail(DVR_E_INVALID_ARG, "need at least one camera");
    const int W = cams[0].width, H = cams[0].height;
    if (W < 1 || H < 1) return fail(DVR_E_INVALID_ARG, "image size must be >= 1");
    // pixel centres i + 1/2 are exact FP32 numbers below 2^23 (the ray setup's double-float FP32)
    if (W > (1 << 23) || H > (1 << 23)) return fail(DVR_E_INVALID_ARG, "image width and height must not exceed 2^23");
    if ((double)W * H * ncam > 2147483647.0) return fail(DVR_E_INVALID_ARG, "too many pixels");
    for (int i = 0; i < ncam; ++i) {
        const dvr_camera &c = cams[i];
        if (c.width != W || c.height != H) return fail(DVR_E_INVALID_ARG, "all cameras must share width and height");
        if (c.persp != 0 && c.persp != 1) return fail(DVR_E_INVALID_ARG, "camera %d: persp must be 0 or 1", i);
        for (int k = 0; k < 3; ++k)
            if (!isfinite(c.o[k]) || !isfinite(c.d0[k]) || !isfinite(c.du[k]) || !isfinite(c.dv[k]))
                return fail(DVR_E_INVALID_ARG, "camera %d has a non-finite value", i);
        kc[i].persp = c.persp;
        for (int k = 0; k < 3; ++k) {
            kc[i].o[k] = c.o[k];
            kc[i].d0[k] = c.d0[k];
            kc[i].du[k] = c.du[k];
            kc[i].dv[k] = c.dv[k];
        }
    }
    memset(&a, 0, sizeof a);
    a.feat.vol = feat->layout == DVR_QUAD ? feat->iquad : vol;
    a.feat.grad = feat->grad;
    a.feat.kappa = feat->kappa;
    a.feat.ves = feat->ves;
    a.feat.gmax = feat->gmax;
    a.feat.dtype = feat->dtype;
    a.feat.layout = feat->layout;
    a.feat.bricks = feat->bricks;
    a.feat.nb[0] = nbricks(grid->nx);
    a.feat.nb[1] = nbricks(grid->ny);
    a.feat.nb[2] = nbricks(grid->nz);
    a.grid.n[0] = grid->nx;
    a.grid.n[1] = grid->ny;
    a.grid.n[2] = grid->nz;
    const float hg[3] = {grid->hx, grid->hy, grid->hz};
    dvr::set_grid_steps(a.grid, hg, rp->step_vox);
    a.tf.K = tf->K;
    a.tf.knots = tf->knots;
    a.tf.rgba = tf->rgba;
    a.rp.lg = rp->lambda_g;
    a.rp.omlg = (float)(1.0 - (double)rp->lambda_g);
    a.rp.lk = rp->lambda_k;
    a.rp.omlk = (float)(1.0 - (double)rp->lambda_k);
    a.rp.k0 = rp->kappa0;
    a.rp.lv = rp->lambda_v;
    a.rp.Tstop = rp->et_alpha > 0.f ? (float)(1.0 - (double)rp->et_alpha) : 5.9604644775390625e-08f;
    a.launch.W = W;
    a.launch.H = H;
    a.cams = kc;
    a.ncam = ncam;
    return DVR_OK;
}

extern "C" {

dvr_status dvr_render(const void *vol, int32_t vol_dtype, const dvr_grid *grid, const dvr_features_buf *feat,
                      const dvr_tf *tf, const dvr_render_params *rp, const dvr_camera *cams, int32_t ncam,
                      float *rgba, const dvr_ray_state *state, hipStream_t stream)
{
    if (ncam > 1 << 20) return fail(DVR_E_INVALID_ARG, "too many cameras");
    dvr::KCam *kc = ncam > 0 ? new (std::nothrow) dvr::KCam[ncam] : nullptr;
    if (ncam > 0 && !kc) return fail(DVR_E_NOMEM, "host allocation");
    dvr::RenderArgs a;
    dvr_status s = build_render_args(vol, vol_dtype, grid, feat, tf, rp, cams, ncam, a, kc);
    if (s == DVR_OK && (!rgba || !aligned16(rgba))) s = fail(rgba ? DVR_E_ALIGN : DVR_E_NULL, "rgba output missing or unaligned");
    if (s == DVR_OK && state && (!state->T_last || !state->k_last)) s = fail(DVR_E_NULL, "ray state arrays are NULL");
    if (s == DVR_OK && state && state->counters && ((uintptr_t)state->counters & 7u))
        s = fail(DVR_E_ALIGN, "counters must be 8-byte aligned");
    if (s != DVR_OK) {
        delete[] kc;
        return s;
    }
    a.launch.out = rgba;
    a.launch.T_last = state ? state->T_last : nullptr;
    a.launch.k_last = state ? state->k_last : nullptr;
    a.launch.counters = state ? (unsigned long long *)state->counters : nullptr;
    hipError_t e = hipSuccess;
    if (a.launch.counters) e = dvr::launch_fill_zero((float *)a.launch.counters, 4, stream);
    if (e == hipSuccess) e = dvr::launch_render(a, stream);
    delete[] kc;
    return e == hipSuccess ? DVR_OK : dev_fail(e, "render launch");
}

dvr_status dvr_render_gather(const void *vol, int32_t vol_dtype, const dvr_grid *grid, const dvr_features_buf *feat,
                             const dvr_tf *tf, const dvr_render_params *rp, const dvr_camera *cams, int32_t ncam,
                             const int32_t *k_last, float *sink, uint64_t *counters, hipStream_t stream)
{
    if (ncam > 1 << 20) return fail(DVR_E_INVALID_ARG, "too many cameras");
    dvr::KCam *kc = ncam > 0 ? new (std::nothrow) dvr::KCam[ncam] : nullptr;
    if (ncam > 0 && !kc) return fail(DVR_E_NOMEM, "host allocation");
    dvr::RenderArgs a;
    dvr_status s = build_render_args(vol, vol_dtype, grid, feat, tf, rp, cams, ncam, a, kc);
    if (s == DVR_OK && (!k_last || !sink)) s = fail(DVR_E_NULL, "k_last and sink are required");
    if (s == DVR_OK && (((uintptr_t)k_last & 3u) || ((uintptr_t)sink & 3u) || ((uintptr_t)counters & 7u)))
        s = fail(DVR_E_ALIGN, "k_last, sink or counters misaligned");
    if (s != DVR_OK) {
        delete[] kc;
        return s;
    }
    a.launch.out = sink;
    a.launch.k_last = const_cast<int32_t *>(k_last);
    a.launch.counters = (unsigned long long *)counters;
    hipError_t e = hipSuccess;
    if (counters) e = dvr::launch_fill_zero((float *)counters, 4, stream);
    if (e == hipSuccess) e = dvr::launch_render_gather(a, stream);
    delete[] kc;
    return e == hipSuccess ? DVR_OK : dev_fail(e, "render gather launch");
}

static dvr_status render_backward(const void *vol, int32_t vol_dtype, const dvr_grid *grid,
                                  const dvr_features_buf *feat, const dvr_tf *tf, const dvr_render_params *rp,
                                  const dvr_camera *cams, int32_t ncam, const dvr_ray_state *state,
                                  const float *dL_drgba, float *dL_dtf, float *dL_dvol, const dvr_feature_grads *fg,
                                  hipStream_t stream)
{
    if (ncam > 1 << 20) return fail(DVR_E_INVALID_ARG, "too many cameras");
    dvr::KCam *kc = ncam > 0 ? new (std::nothrow) dvr::KCam[ncam] : nullptr;
    if (ncam > 0 && !kc) return fail(DVR_E_NOMEM, "host allocation");
    dvr::RenderArgs a;
    dvr_status s = build_render_args(vol, vol_dtype, grid, feat, tf, rp, cams, ncam, a, kc);
    if (s == DVR_OK && (!state || !state->T_last || !state->k_last)) s = fail(DVR_E_NULL, "ray state is required");
    if (s == DVR_OK && (!dL_drgba || !dL_dtf)) s = fail(DVR_E_NULL, "dL_drgba and dL_dtf are required");
    if (s == DVR_OK && (!aligned16(dL_drgba) || ((uintptr_t)dL_dtf & 3u) || (dL_dvol && ((uintptr_t)dL_dvol & 3u))))
        s = fail(DVR_E_ALIGN, "gradient buffers misaligned");
    if (s == DVR_OK && fg && (!fg->dfeat || !fg->dgmax)) s = fail(DVR_E_NULL, "dfeat and dgmax are required");
    if (s == DVR_OK && fg && (((uintptr_t)fg->dfeat & 3u) || ((uintptr_t)fg->dgmax & 3u)))
        s = fail(DVR_E_ALIGN, "feature gradient buffers misaligned");
    if (s != DVR_OK) {
        delete[] kc;
        return s;
    }
    a.launch.T_last = state->T_last;
    a.launch.k_last = state->k_last;
    a.launch.dout = dL_drgba;
    a.launch.dtf = dL_dtf;
    a.launch.dvol = dL_dvol;
    a.launch.dfeat = fg ? fg->dfeat : nullptr;
    a.launch.dgmax = fg ? fg->dgmax : nullptr;
    hipError_t e = dvr::launch_fill_zero(dL_dtf, (int64_t)tf->K * 4, stream);
    if (e == hipSuccess && dL_dvol) e = dvr::launch_fill_zero(dL_dvol, nvox(grid), stream);
    if (e == hipSuccess && fg) e = dvr::launch_fill_zero(fg->dfeat, 5 * nvox(grid), stream);
    if (e == hipSuccess && fg) e = dvr::launch_fill_zero(fg->dgmax, 1, stream);
    if (e == hipSuccess) e = dvr::launch_render_backward(a, stream);
    delete[] kc;
    return e == hipSuccess ? DVR_OK : dev_fail(e, "render backward launch");
}

dvr_status dvr_render_backward(const void *vol, int32_t vol_dtype, const dvr_grid *grid,
                               const dvr_features_buf *feat, const dvr_tf *tf, const dvr_render_params *rp,
                               const dvr_camera *cams, int32_t ncam, const dvr_ray_state *state,
                               const float *dL_drgba, float *dL_dtf, float *dL_dvol, hipStream_t stream)
{
    return render_backward(vol, vol_dtype, grid, feat, tf, rp, cams, ncam, state, dL_drgba, dL_dtf, dL_dvol, nullptr,
                           stream);
}

dvr_status dvr_render_backward_features(const void *vol, int32_t vol_dtype, const dvr_grid *grid,
                                        const dvr_features_buf *feat, const dvr_tf *tf, const dvr_render_params *rp,
                                        const dvr_camera *cams, int32_t ncam, const dvr_ray_state *state,
                                        const float *dL_drgba, float *dL_dtf, float *dL_dvol,
                                        const dvr_feature_grads *fg, hipStream_t stream)
{
    if (!fg) return fail(DVR_E_NULL, "feature gradients are required");
    return render_backward(vol, vol_dtype, grid, feat, tf, rp, cams, ncam, state, dL_drgba, dL_dtf, dL_dvol, fg,
                           stream);
}

}  // extern "C"
