// Host-side helpers of libdvr shared by the C ABI entry points (api.hip) and the batched plan
// (batch.hip): validation, error reporting, Gaussian tap tables.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "common.hpp"
#include "render_args.hpp"

namespace dvr::host {

extern thread_local std::string g_err;

dvr_status fail(dvr_status s, const char *fmt, ...);
dvr_status dev_fail(hipError_t e, const char *what);
bool aligned16(const void *p);
bool finite_pos(float v);
dvr_status check_grid(const dvr_grid *g);
int64_t nvox(const dvr_grid *g);
int gauss_radius(double sigma_vox);
dvr_status check_fparams(const dvr_grid *g, const dvr_feature_params *fp);
dvr_status check_feat_buf(const dvr_features_buf *f, bool need_writable);
void axis_taps(double sigma_vox, double h, dvr::AxisTaps &t);
size_t features_ws_bytes(const dvr_grid *g);
// Validates the shared render inputs and fills the kernel-argument records (cameras into kc).
dvr_status build_render_args(const void *vol, int32_t vol_dtype, const dvr_grid *grid, const dvr_features_buf *feat,
                             const dvr_tf *tf, const dvr_render_params *rp, const dvr_camera *cams, int32_t ncam,
                             dvr::RenderArgs &a, dvr::KCam *kc);

}  // namespace dvr::host
