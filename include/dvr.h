/*
 * dvr.h -- C ABI of the MI355X (gfx950) direct-volume-rendering hot path.
 *
 * Method: Beckley, "Decentralized Direct Volume Rendering: A Browser-Native GPU Architecture
 * for MRI Digital Twins in Resource-Constrained Settings".  Two data-parallel passes:
 *   features  per-voxel morphology: central-difference gradient (Sec. 2.3 Eq. 2), Gaussian-scale
 *             Hessian and its eigenvalues, directional curvature k = g^T H g / g^T g (Sec. 2.3
 *             Eq. 3) and multi-scale vesselness (Sec. 1, Frangi et al. 1998);
 *   render    single-pass front-to-back raymarch: morphologically modulated opacity (Sec. 2.4
 *             Eq. 4) and emission-absorption compositing (Sec. 2.4 Eq. 5-6);
 * plus min-max normalization (Sec. 2.2 Eq. 1), the adjoint of the raymarch, and a batched
 * launch of many volumes and views.
 *
 * Conventions (every entry point):
 *   - Volumes are C order [nz][ny][nx] (x fastest); voxel (i,j,k) sits at (i hx, j hy, k hz) mm.
 *     Every axis has n >= 2 and spacing h > 0.
 *   - Pointers documented as "device" are device pointers, 16-byte aligned, owned by the caller;
 *     structs passed by pointer are host memory and are read before the call returns.
 *   - Calls are asynchronous and ordered on the given HIP stream (NULL = default stream).
 *     Nothing synchronizes the device.  Scalars produced on the device (|grad I|_max) stay there.
 *   - Arguments are validated before anything is enqueued: on a non-OK return nothing was
 *     enqueued and dvr_last_error() describes the problem.  No exception crosses the ABI.
 *   - Outputs are overwritten, except dL_dvol of dvr_features_backward, which is accumulated into
 *     (so that the gradient through the TF lookup can be added to it first).
 *   - The transfer function lives in device memory (the analogue of the paper's uniform buffers,
 *     Sec. 4): editing it needs no re-launch setup, and the batched plan picks up the change.
 */
#ifndef DVR_H
#define DVR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dvr_status {
    DVR_OK = 0,
    DVR_E_INVALID_ARG = -1, /* bad size, spacing, scale, parameter value */
    DVR_E_NULL = -2,        /* a required pointer is NULL */
    DVR_E_ALIGN = -3,       /* a device pointer is not 16-byte aligned */
    DVR_E_UNSUPPORTED = -4, /* valid but not implemented combination (dtype/layout) */
    DVR_E_NOMEM = -5,       /* host allocation failed (batched plans only) */
    DVR_E_DEVICE = -6,      /* a HIP runtime call failed */
    DVR_E_TIMEOUT = -8,     /* the batched launch's bounded dependency wait expired */
    DVR_E_WORKSPACE = -9    /* workspace missing or smaller than the queried size */
} dvr_status;

typedef enum dvr_dtype { DVR_F32 = 0, DVR_F16 = 1, DVR_U16 = 2 } dvr_dtype;

/* Feature storage layout.
 *   DVR_PLANAR:       grad = [3][nz][ny][nx] (gx, gy, gz planes), kappa = [nz][ny][nx],
 *                     ves = [nz][ny][nx], each of the buffer's dtype.
 *   DVR_INTERLEAVED:  grad = one record of 8 values per voxel, [nz][ny][nx][8] =
 *                     (I, gx, gy, gz, kappa, V, 0, 0) of the buffer's dtype (32 B in F32, 16 B in
 *                     F16); kappa and ves are unused.  The record carries the intensity so that the
 *                     raymarcher fetches one record per corner.
 *   DVR_SPLIT:        grad = one record of 4 values per voxel, [nz][ny][nx][4] = (gx, gy, gz, kappa)
 *                     (16 B in F32, 8 B in F16); ves = [nz][ny][nx]; kappa is unused; the intensity
 *                     is the volume, as in PLANAR.  A sample of zero extinction fetches only I; a
 *                     shaded one fetches I, one record and V per corner (the same 24 / 12 bytes per
 *                     voxel as PLANAR, in half the gathers).
 *   DVR_QUAD:         grad = the SPLIT records, [nz][ny][nx][4] = (gx, gy, gz, kappa); ves =
 *                     [nz][ny][nx][4] vesselness quads (V(x,y,z), V(x,y+1,z), V(x,y,z+1),
 *                     V(x,y+1,z+1)), 0 past the last row or slice; iquad = the same quads of the
 *                     intensity, copied bit for bit from the volume given to dvr_features (whose dtype
 *                     must be the feature dtype); kappa is unused.  The 8 corners of a cell are the
 *                     quads of its two x-neighbours, so the raymarcher reads a cell's intensity, and
 *                     its V, in two loads instead of four (48 / 24 bytes per voxel).  dvr_render and
 *                     dvr_render_backward read the intensity from iquad and ignore vol.  The batched
 *                     launch builds the quads itself, after each volume's last feature scale. */
typedef enum dvr_layout { DVR_PLANAR = 0, DVR_INTERLEAVED = 1, DVR_SPLIT = 2, DVR_QUAD = 3 } dvr_layout;

typedef struct dvr_grid {
    int32_t nx, ny, nz; /* >= 2 each, nx*ny*nz < 2^31 */
    float hx, hy, hz;   /* voxel spacing in mm, > 0 */
} dvr_grid;

#define DVR_MAX_SIGMA 8
#define DVR_MAX_RADIUS 14 /* Gaussian radius floor(3 sigma/h + 1/2) per axis must not exceed this */

typedef struct dvr_feature_params {
    int32_t nsigma;                 /* 1..DVR_MAX_SIGMA scales; sigma_mm[0] also defines the Hessian of k */
    float sigma_mm[DVR_MAX_SIGMA];  /* Gaussian scales in mm (per-axis sigma in voxels = sigma / h) */
    float alpha, beta;              /* Frangi plate/blob sensitivities (> 0); 0.5, 0.5 is customary */
    float c;                        /* Frangi structure sensitivity; <= 0 selects c = 1/2 max |sigma^2 H|_F */
    float eig_gap_fp64;             /* eigenvalues whose smallest gap is below eig_gap_fp64 * max|lambda|
                                       are re-solved in FP64; 0 disables the FP64 path */
} dvr_feature_params;

/* Brick table for exact empty-space skipping.  Brick (bx, by, bz) covers the cells
 * [DVR_BRICK b, DVR_BRICK (b + 1)) of each axis, i.e. the voxels DVR_BRICK b .. min(DVR_BRICK (b + 1),
 * n - 1); nb_a = ceil((n_a - 1) / DVR_BRICK) bricks per axis, nb = nbx nby nbz in all.  The table is
 * nb (min, max) float pairs of the intensity the raymarcher samples in each brick ([nbz][nby][nbx][2],
 * written by dvr_features), followed by ceil(nb / 32) uint32 words: one bit per brick, set by
 * dvr_render when every intensity the trilinear interpolation can produce there maps onto TF segments
 * of zero extinction.  Samples in such a brick have alpha = 0 exactly (Sec. 2.4 Eq. 4-6 give them no
 * weight), so the forward raymarch passes them without fetching features; the result is unchanged. */
#define DVR_BRICK 4

typedef struct dvr_features_buf {
    void *grad;   /* device; see dvr_layout */
    void *kappa;  /* device, PLANAR only */
    void *ves;    /* device, PLANAR, SPLIT and QUAD */
    float *gmax;  /* device scalar: max over voxels of |grad I|_2 (the |grad I|_max of Eq. 4) */
    int32_t dtype;  /* DVR_F32 or DVR_F16 (storage type; arithmetic is FP32) */
    int32_t layout; /* dvr_layout */
    float *bricks;  /* device brick table of dvr_bricks_bytes() bytes, 8-byte aligned, or NULL.  Its
                       (min, max) pairs are written by dvr_features from the intensity the raymarcher
                       samples (the volume passed to dvr_features for PLANAR, the records' I for
                       INTERLEAVED); when non-NULL, dvr_render writes the empty-brick bits for its TF
                       and skips those bricks (the volume must then be the one the table was built
                       from, and renders sharing one table must be ordered on one stream).
                       dvr_render_backward and the batched launch do not use it. */
    void *iquad;    /* device, QUAD only: [nz][ny][nx][4] intensity quads, 16-byte aligned; NULL otherwise */
} dvr_features_buf;

typedef struct dvr_tf {
    int32_t K;          /* 2..64 knots */
    const float *knots; /* device [K], strictly increasing intensities */
    const float *rgba;  /* device [K][4]: R, G, B in [0,1] (not premultiplied); A = extinction per mm >= 0 */
} dvr_tf;

typedef struct dvr_render_params {
    float lambda_g; /* weight of the edge-strength factor |g|/|g|_max in Eq. 4, in [0,1] */
    float lambda_k; /* weight of the curvature factor w(k) = |k| / (|k| + kappa0), in [0,1] */
    float kappa0;   /* curvature half-saturation in 1/mm^2, > 0 */
    float lambda_v; /* vesselness emphasis u = 1 + lambda_v V, >= 0 */
    float step_vox; /* segment length as a fraction of min(h), >= 1/64 */
    float et_alpha; /* early termination once accumulated opacity >= et_alpha; <= 0 disables it */
} dvr_render_params;

/* Camera, pixel (i, j) with row j = 0 at the top:
 *   orthographic (persp = 0): origin o + (i+1/2) du + (j+1/2) dv, direction d0 (unit length);
 *   perspective  (persp = 1): origin o, direction normalize(d0 + (i+1/2) du + (j+1/2) dv).
 * 1 <= width, height <= 2^23 (DVR_E_INVALID_ARG otherwise). */
typedef struct dvr_camera {
    int32_t persp, width, height;
    float o[3], d0[3], du[3], dv[3];
} dvr_camera;

/* Per-ray state the forward pass leaves for the adjoint: the transmittance before the last
 * evaluated sample and that sample's index (-1 for a ray that misses the volume). */
typedef struct dvr_ray_state {
    float *T_last;      /* device [ncam][H][W] */
    int32_t *k_last;    /* device [ncam][H][W] */
    uint64_t *counters; /* device [2], 8-byte aligned, nullable; dvr_render overwrites it with the
                           number of evaluated samples and of those with non-zero extinction (the
                           rest are exactly transparent and skip the feature fetch).  Counting adds
                           one pair of 64-bit atomics per 256-ray workgroup, all on these two words
                           (the L2 serializes them): ~8 % of the raymarch on 1024^2 views. */
} dvr_ray_state;

/* Library version, for the binding's load check. */
int32_t dvr_version(void);

/* Thread-local message of the last non-OK status returned on this thread. */
const char *dvr_last_error(void);

/* Eq. 1 (Sec. 2.2): out = (raw - min) / (max - min) over all n values, 0 where max == min.
 * raw: device, DVR_U16 or DVR_F32 or DVR_F16; out: device, DVR_F16 (round to nearest even) or
 * DVR_F32.  ws: device workspace of at least dvr_normalize_workspace() bytes. */
dvr_status dvr_normalize_workspace(int64_t n, size_t *bytes);
dvr_status dvr_normalize(const void *raw, int32_t raw_dtype, void *out, int32_t out_dtype, int64_t n,
                         void *ws, size_t ws_bytes, hipStream_t stream);

/* dvr_normalize without a caller workspace and without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * it).  Same arguments, results and errors as dvr_normalize; the two reduction words live in a
 * 256-byte static device array that the library holds on each GPU it runs on until the process
 * ends (cleared by a fill kernel at the start of every call).  Every call on one GPU shares that
 * array: calls that overlap on one GPU (different streams, or host threads) race and may give
 * wrong results; calls ordered on one stream do not.  Returns DVR_E_WORKSPACE if the reduction
 * would need more than the array holds (it needs 8 bytes for any n), DVR_E_DEVICE if the array's
 * address cannot be looked up on the current device. */
dvr_status dvr_normalize_noalloc(const void *raw, int32_t raw_dtype, void *out, int32_t out_dtype, int64_t n,
                                 hipStream_t stream);

/* Feature pass (Sec. 2.3 Eq. 2-3; Sec. 1 multi-scale Hessian and vesselness).
 *   gradient  g_a = (I[a+1] - I[a-1]) / (2 h_a), indices clamped to the grid (Eq. 2);
 *   gmax      max |g|_2 over all voxels, written to out->gmax;
 *   Hessian   of the volume smoothed with the sampled, normalized Gaussian of radius
 *             floor(3 sigma/h + 1/2) (clamped indices), by central second differences (clamped);
 *             computed as derivative-of-Gaussian filters, which is the same linear operator;
 *   kappa     g^T H g / g^T g with H at sigma_mm[0] (units I/mm^2); 0 where g = 0 (Eq. 3);
 *   V         max over scales of Frangi's bright-tube vesselness of the magnitude-sorted
 *             eigenvalues of sigma^2 H (0 unless lambda2 < 0 and lambda3 < 0).
 * vol: device [nz][ny][nx] of vol_dtype (DVR_F32 or DVR_F16).  ws: device workspace of at least
 * dvr_features_workspace() bytes.  out: see dvr_features_buf (F32 or F16, any dvr_layout; INTERLEAVED
 * and QUAD need vol_dtype equal to the feature dtype). */
dvr_status dvr_features_workspace(const dvr_grid *grid, const dvr_feature_params *fp, size_t *bytes);
/* Number of bricks nb = nbx * nby * nbz, and the byte size 8 nb + 4 ceil(nb / 32) of the brick table,
 * for this grid. */
dvr_status dvr_bricks_count(const dvr_grid *grid, int64_t *count);
dvr_status dvr_bricks_bytes(const dvr_grid *grid, size_t *bytes);
dvr_status dvr_features(const void *vol, int32_t vol_dtype, const dvr_grid *grid, const dvr_feature_params *fp,
                        const dvr_features_buf *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Optional denoise pre-pass (Sec. 5.3: spatial smoothing or median filtering as an optional compute
 * pass before the feature pass).
 *   DVR_DENOISE_MEDIAN3  3x3x3 median with clamped indices (exact: the result is one of the inputs);
 *   DVR_DENOISE_GAUSS    separable sampled, normalized Gaussian of sigma_mm (per-axis radius
 *                        floor(3 sigma/h + 1/2) <= DVR_MAX_RADIUS, clamped indices), FP32 arithmetic.
 * vol, out: device [nz][ny][nx] of dtype (DVR_F32 or DVR_F16, rounded to nearest even), distinct,
 * 16-byte aligned; ws: device workspace of dvr_denoise_workspace() bytes (GAUSS: two FP32 volumes;
 * MEDIAN3: none, ws may be NULL). */
typedef enum dvr_denoise_mode { DVR_DENOISE_GAUSS = 0, DVR_DENOISE_MEDIAN3 = 1 } dvr_denoise_mode;
dvr_status dvr_denoise_workspace(const dvr_grid *grid, int32_t mode, size_t *bytes);
dvr_status dvr_denoise(const void *vol, int32_t dtype, const dvr_grid *grid, int32_t mode, float sigma_mm, void *out,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/* Automatic tissue windows (Sec. 2.2: a 256-bin density analysis of I_norm shows three tissue peaks;
 * Sec. 3.1, Table 2: target windows CSF 0.05..0.12, GM 0.12..0.18, WM > 0.18).
 * Histogram: counts of the values x > floor of a normalized volume in bin floor(256 x) clamped to
 * [0, 255] (x = 1 falls in the last bin).  vol: device, DVR_F32 or DVR_F16, 16-byte aligned, n < 2^32
 * values; hist: device uint32[256], overwritten; used: device uint32 (the number counted) or NULL. */
#define DVR_HIST_BINS 256
dvr_status dvr_histogram(const void *vol, int32_t dtype, int64_t n, float floor_, uint32_t *hist, uint32_t *used,
                         hipStream_t stream);

/* The three tissue peaks of a histogram: the local maxima of the [1, 2, 1]-smoothed counts
 * (S[b] > S[b-1] and S[b] >= S[b+1], clamped ends), taken greedily by S (lower bin first on a tie) at
 * least min_sep bins apart, at most three, ordered by bin as CSF, GM, WM; peak = (bin + 1/2) / 256;
 * a missing peak has bin -1 and peak -1; in_window tells whether the peak lies in its Table 2
 * window (CSF [0.05, 0.12), GM [0.12, 0.18), WM (0.18, 1]). */
typedef struct dvr_peaks {
    int32_t bin[3];
    float peak[3];
    int32_t in_window[3];
} dvr_peaks;
/* hist: device uint32[256]; out: device dvr_peaks, overwritten; min_sep >= 1. */
dvr_status dvr_tissue_peaks(const uint32_t *hist, int32_t min_sep, dvr_peaks *out, hipStream_t stream);

/* A transfer function from the peaks (the "zero-shot" TF of Sec. 3.1): 8 knots
 * (0, 0.05, m_CSF, m_GM, m_WM, u, u + 1/256, 1), m_c the peak (a missing one: the window centre
 * 0.085, 0.15, 0.24), kept strictly increasing at least one bin apart with m_WM <= 1 - 3/256, and
 * u = m_WM + (m_WM - m_GM) within [m_WM + 1/256, 1 - 2/256].  RGBA: extinction 0 at the first two
 * knots (low-intensity bone and air clipped, Sec. 2.2), rgb[c] / tau[c] at the peaks, the WM plateau
 * up to u, rgb_hi / tau_hi above it (tau_hi = 0 also clips extracranial fat and enhancing tissue). */
typedef struct dvr_tissue_tf_params {
    float rgb[3][3]; /* CSF, GM, WM colours in [0, 1] */
    float tau[3];    /* their extinctions per mm, >= 0 */
    float rgb_hi[3];
    float tau_hi;
} dvr_tissue_tf_params;
/* peaks: device dvr_peaks; knots: device float[8]; rgba: device float[8][4] (16-byte aligned). */
dvr_status dvr_tissue_tf(const dvr_peaks *peaks, const dvr_tissue_tf_params *params, float *knots, float *rgba,
                         hipStream_t stream);

/* Raymarch (Sec. 2.4 Eq. 4-6), one ray per pixel of each camera.  The box [0,(n-1)h] is clipped
 * by the slab method; the chord [tn, tf] is cut into N = ceil(L / delta) segments of
 * delta = step_vox * min(h) (the last one shorter) and sampled at segment midpoints.  Each sample
 * trilinearly interpolates I, g, kappa, V; the TF (piecewise linear, clamped) gives colour c and
 * extinction tau; sigma = tau * m * w * u with m = (1 - lambda_g) + lambda_g min(|g|/gmax, 1),
 * w = (1 - lambda_k) + lambda_k |k| / (|k| + kappa0), u = 1 + lambda_v V; alpha = 1 - exp(-sigma
 * delta_k); C += T alpha c, A += T alpha, T *= 1 - alpha (Eq. 5-6; A equals 1 - T in exact
 * arithmetic and is summed so that faint rays keep their relative accuracy).
 * vol: device [nz][ny][nx] of vol_dtype, 16-byte aligned, the feature dtype: the intensity that is
 * sampled for PLANAR and SPLIT features; ignored (may be NULL) for INTERLEAVED and QUAD, whose
 * records or iquad carry it (the same holds for the adjoints below).
 * rgba: device [ncam][H][W][4] float (premultiplied R, G, B and A).  All cameras must share W and
 * H.  state: nullable; filled for dvr_render_backward.  Without early termination a ray still
 * stops once T <= 2^-24 (the light left is below FP32 resolution). */
dvr_status dvr_render(const void *vol, int32_t vol_dtype, const dvr_grid *grid, const dvr_features_buf *feat,
                      const dvr_tf *tf, const dvr_render_params *rp, const dvr_camera *cams, int32_t ncam,
                      float *rgba, const dvr_ray_state *state, hipStream_t stream);

/* Gather ceiling of dvr_render, for measurement (the bound on a raymarch with this access pattern,
 * Sec. 2.4): walks the rays of dvr_render with the same arguments over the same samples, 0 .. k_last
 * of each ray (k_last from that forward pass), with the same empty-brick skipping, and issues the
 * same loads: the intensity corners of every sample, the TF segment test, and the feature corners of
 * the samples with non-zero extinction.  Eq. 4, the exponential and the compositing are left out.
 * k_last: device [ncam][H][W] int32 (dvr_ray_state.k_last of the forward pass); sink: device
 * [ncam][H][W] float, overwritten with a per-ray sum of the fetched features (it only keeps the loads
 * live); counters: device [2], 8-byte aligned, nullable, overwritten with the samples walked and
 * those whose feature corners were fetched (equal to the forward pass's counters). */
dvr_status dvr_render_gather(const void *vol, int32_t vol_dtype, const dvr_grid *grid, const dvr_features_buf *feat,
                             const dvr_tf *tf, const dvr_render_params *rp, const dvr_camera *cams, int32_t ncam,
                             const int32_t *k_last, float *sink, uint64_t *counters, hipStream_t stream);

/* Adjoint of dvr_render with respect to the TF values and the voxel intensities; the features
 * are held constant.  Each ray is walked back to front from the stored (T_last, k_last),
 * recomputing every sample exactly as the forward pass did.
 * dL_drgba: device [ncam][H][W][4]; dL_dtf: device [K][4] float, overwritten;
 * dL_dvol: device [nz][ny][nx] float, overwritten, nullable. */
dvr_status dvr_render_backward(const void *vol, int32_t vol_dtype, const dvr_grid *grid,
                               const dvr_features_buf *feat, const dvr_tf *tf, const dvr_render_params *rp,
                               const dvr_camera *cams, int32_t ncam, const dvr_ray_state *state,
                               const float *dL_drgba, float *dL_dtf, float *dL_dvol, hipStream_t stream);

/* Gradients with respect to the feature values (dense FP32 in [nz][ny][nx] order whatever the
 * feature layout), for the feature-pass adjoint: dfeat = device [5][nz][ny][nx] holding
 * dL/d(gx, gy, gz, k, V); dgmax = device [1] holding dL/d|g|_max. */
typedef struct dvr_feature_grads {
    float *dfeat;
    float *dgmax;
} dvr_feature_grads;

/* dvr_render_backward plus the gradients with respect to the feature values that Eq. 4 reads
 * (Sec. 2.4): sigma = tau m w u with m = (1 - lambda_g) + lambda_g min(|g| / |g|_max, 1),
 * w = (1 - lambda_k) + lambda_k |k| / (|k| + kappa0), u = 1 + lambda_v V; through the trilinear
 * interpolation to each voxel's g, k and V, and to |g|_max.  Where min(., 1) is at 1 the m term
 * has no gradient, and w has none at k = 0.  fg: required, both arrays overwritten (FP32 atomics:
 * the summation order, and so the last bits, vary from run to run).  The other arguments and
 * outputs are those of dvr_render_backward. */
dvr_status dvr_render_backward_features(const void *vol, int32_t vol_dtype, const dvr_grid *grid,
                                        const dvr_features_buf *feat, const dvr_tf *tf, const dvr_render_params *rp,
                                        const dvr_camera *cams, int32_t ncam, const dvr_ray_state *state,
                                        const float *dL_drgba, float *dL_dtf, float *dL_dvol,
                                        const dvr_feature_grads *fg, hipStream_t stream);

/* Workspace of dvr_features_backward in bytes (about 57 + 24 nsigma bytes per voxel plus the band
 * tables). */
dvr_status dvr_features_backward_workspace(const dvr_grid *grid, const dvr_feature_params *fp, size_t *bytes);

/* Adjoint of dvr_features: adds to dL_dvol the gradient with respect to the voxel intensities I of
 *   sum_v dL/dg(v) . g(v) + dL/dk(v) k(v) + dL/dV(v) V(v) + dL/d|g|_max |g|_max,
 * with g the clamped central difference of I (Sec. 2.3 Eq. 2), k = g^T H g / g^T g at the first
 * scale (Sec. 2.3 Eq. 3, 0 where g = 0), V the maximum over the scales of Frangi's bright-tube
 * vesselness of sigma^2 H (Sec. 1), H the Hessian of the Gaussian-smoothed volume, all as
 * dvr_features defines them; fg holds the upstream gradients (the output of
 * dvr_render_backward_features).  Conventions where the forward is not differentiable: V is
 * differentiated at the first scale reaching the maximum (FP64 comparison), and not where V = 0;
 * |g|_max at the voxel of largest |g| (the lowest index on a tie of the FP32-rounded norms); k not
 * at g = 0; the eigenvalue derivative assumes distinct eigenvalues.  The local derivatives are
 * evaluated in FP64 (Jacobi eigenvectors), the transposed filters in FP32.
 * vol: device [nz][ny][nx] F32 or F16 (16-byte aligned), the volume the features were computed
 * from; fp: as for dvr_features, with c > 0 (the adjoint does not differentiate the automatic c);
 * dL_dvol: device [nz][ny][nx] float, ACCUMULATED into (add the TF-lookup part from
 * dvr_render_backward first); ws: device, 256-byte aligned, at least
 * dvr_features_backward_workspace bytes.  Stream-ordered; nothing is enqueued on a
 * validation error. */
dvr_status dvr_features_backward(const void *vol, int32_t vol_dtype, const dvr_grid *grid,
                                 const dvr_feature_params *fp, const dvr_feature_grads *fg, float *dL_dvol, void *ws,
                                 size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Batched launch: the feature pass of many volumes (uneven shapes, anisotropic spacing) and the
 * raymarch of many views of them, in one persistent kernel recorded in a HIP graph.  The kernel
 * drains a queue of work items in a fixed order (z-filter slabs, then feature tiles, then ray
 * tiles); a feature tile waits for its volume's z-filter items and a ray tile for its volume's
 * feature items (per-volume completion counters, release/acquire at device scope).  Because items
 * are taken in queue order and an item only waits for items taken before it, every awaited item
 * is held by a running workgroup and the launch cannot deadlock; each wait is still bounded and
 * reports DVR_E_TIMEOUT through dvr_batch_check instead of hanging.
 * The transfer function is read from device memory at every launch: editing it needs no new plan
 * (the analogue of the paper's uniform buffers, Sec. 4). */

typedef struct dvr_batch_volume {
    const void *vol;        /* device [nz][ny][nx] of vol_dtype (DVR_F32 or DVR_F16) */
    int32_t vol_dtype;
    dvr_grid grid;
    dvr_features_buf feat;  /* device feature buffers written by each launch (all volumes share dtype and layout) */
} dvr_batch_volume;

typedef struct dvr_batch_view {
    int32_t volume;         /* index into the volume array */
    dvr_camera cam;         /* each view has its own image size */
    float *rgba;            /* device [H][W][4] */
    float *T_last;          /* device [H][W], nullable */
    int32_t *k_last;        /* device [H][W], nullable (written only if T_last is given) */
} dvr_batch_view;

/* Tile and brick shapes of a batched launch (chosen by dvr_batch_autotune or given). */
typedef struct dvr_tune {
    int32_t wg_per_cu; /* persistent workgroups per compute unit, 1..8 */
    int32_t xy_tile;   /* feature tile (x by y voxels): 0 = 64x8, 1 = 32x16, 2 = 128x4 */
    int32_t xy_zrun;   /* z slices per feature item, 1..32 */
    int32_t z_chunk;   /* z slices per z-filter item, 1..64 */
    int32_t ray_tile;  /* rays per wave within a 16x16 workgroup tile: 0 = 8x8, 1 = 16x4, 2 = 4x16 */
} dvr_tune;

typedef struct dvr_batch_desc {
    int32_t nvol;
    const dvr_batch_volume *vols;  /* host array */
    int32_t nview;
    const dvr_batch_view *views;   /* host array */
    dvr_feature_params fp;         /* shared by all volumes; c must be > 0 */
    dvr_tf tf;                     /* shared; device memory */
    dvr_render_params rp;          /* shared */
    const dvr_tune *tune;          /* nullable: defaults */
} dvr_batch_desc;

typedef struct dvr_batch dvr_batch; /* opaque plan: owns its work tables, workspace, counters and graph */

/* Builds the plan (validates, allocates, uploads the tables, records the graph).  Synchronous. */
dvr_status dvr_batch_create(const dvr_batch_desc *desc, dvr_batch **plan);
/* Enqueues one replay of the plan's graph on stream.  Asynchronous. */
dvr_status dvr_batch_launch(dvr_batch *plan, hipStream_t stream);
/* Waits for stream and reports DVR_E_TIMEOUT if a dependency wait of the last launch expired. */
dvr_status dvr_batch_check(dvr_batch *plan, hipStream_t stream);
dvr_status dvr_batch_destroy(dvr_batch *plan);
/* Picks the tile shapes: times candidate dvr_tune values on this batch (graph replays, HIP events) by
 * coordinate descent from the defaults (two sweeps over wg_per_cu 2, 3, 4, 6, 8; xy_tile 0-2; xy_zrun
 * 8, 16, 32; z_chunk 4, 8, 16, 32; ray_tile 0-2, each field with the others at the best so far) and
 * returns the fastest.  With cache_path, results are kept in a JSON file keyed by the batch's
 * shape class and reused.  Synchronous; overwrites the batch's outputs. */
dvr_status dvr_batch_autotune(const dvr_batch_desc *desc, const char *cache_path, dvr_tune *best);

#ifdef __cplusplus
}
#endif
#endif /* DVR_H */
