// Kernel-argument records of the raymarcher (passed by value; no device-side parameter buffers,
// so a launch records into a HIP graph with nothing else to copy).
#pragma once

#include <stdint.h>

#include "dvr.h"

namespace dvr {

constexpr int kCamChunk = 32;  // cameras per launch (kernel arguments stay under 4 KB)

struct KCam {
    int32_t persp;
    float o[3], d0[3], du[3], dv[3];
};

struct KFeat {
    const void *vol;  // planar: the intensity volume (same dtype as the features)
    const void *grad, *kappa, *ves;
    const float *gmax;
    int32_t dtype, layout;
    const float *bricks;  // [nb2][nb1][nb0][2] intensity (min, max) per brick, or null (no skipping)
    int32_t nb[3];
};

struct KGrid {
    int32_t n[3];
    float h[3];
    float delta_hi, delta_lo;    // step_vox * min(h) in mm, exactly: the sum of the two (the product of
                                 // two FP32 numbers has at most 48 significant bits)
    float ih_hi[3], ih_lo[3];    // 1 / h as a double-float pair (~48 bits)
    float idelta_hi, idelta_lo;  // 1 / (step_vox * min(h)) likewise
};

struct KTF {
    int32_t K;
    const float *knots, *rgba;
};

struct KRender {
    float lg, omlg, lk, omlk, k0, lv;
    float Tstop;  // stop once T <= Tstop (1 - et_alpha, or 2^-24 without early termination)
};

struct KLaunch {
    int32_t W, H, ncam, cam_base;
    float *out;             // [cam][H][W][4]
    float *T_last;          // [cam][H][W] or null
    int32_t *k_last;        // [cam][H][W] or null
    const float *dout;      // backward: dL/d rgba
    float *dtf;             // backward: dL/d TF values [K][4]
    float *dvol;            // backward: dL/d I [N] or null
    float *dfeat = nullptr;  // backward with feature gradients: dL/d(gx, gy, gz, k, V) as [5][N], or null
    float *dgmax = nullptr;  // backward with feature gradients: dL/d gmax [1]
    unsigned long long *counters;  // forward: evaluated samples, shaded samples (or null)
    KCam cams[kCamChunk];
};

struct RenderArgs {
    KFeat feat;
    KGrid grid;
    KTF tf;
    KRender rp;
    KLaunch launch;  // template: cams filled per chunk
    const KCam *cams;
    int32_t ncam;
};

// Host: a double as the pair hi + lo of FP32 numbers (exact for the 48-bit product step_vox * hmin).
inline void split2(double v, float &hi, float &lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

// the grid's spacing and segment-length fields of KGrid, from the FP32 spacings and step
inline void set_grid_steps(KGrid &g, const float h[3], float step_vox)
{
    float hmin = h[0];
    if (h[1] < hmin) hmin = h[1];
    if (h[2] < hmin) hmin = h[2];
    const double d = (double)step_vox * (double)hmin;
    split2(d, g.delta_hi, g.delta_lo);
    split2(1.0 / d, g.idelta_hi, g.idelta_lo);
    for (int a = 0; a < 3; ++a) {
        g.h[a] = h[a];
        split2(1.0 / (double)h[a], g.ih_hi[a], g.ih_lo[a]);
    }
}

}  // namespace dvr
