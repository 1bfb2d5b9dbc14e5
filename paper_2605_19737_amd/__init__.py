"""MI355X (gfx950) hot path of the direct-volume-rendering method of Beckley, "Decentralized Direct
Volume Rendering: A Browser-Native GPU Architecture for MRI Digital Twins in Resource-Constrained
Settings": the per-voxel morphology pass (Sec. 2.3 Eq. 2-3, Sec. 1 multi-scale Hessian and
vesselness) and the front-to-back raymarcher (Sec. 2.4 Eq. 4-6), with its adjoint.

The Python layer is a thin binding: PyTorch supplies device memory and the current stream, and
every arithmetic step runs in the HIP kernels of libdvr.so (see include/dvr.h).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from . import _abi as abi
from ._abi import DVRError

__all__ = ["Features", "features", "render", "render_gather", "render_backward", "normalize", "DVRRender",
           "DVRRenderFromVolume", "DVRError", "camera_struct", "lib", "Batch"]


def lib():
    return abi.load()


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return abi.DVR_F32
    if t.dtype == torch.float16:
        return abi.DVR_F16
    if t.dtype in (torch.uint16, torch.int16):
        return abi.DVR_U16
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _require_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous CUDA (HIP) tensors")


def grid_struct(shape_zyx, spacing):
    nz, ny, nx = shape_zyx
    return abi.Grid(int(nx), int(ny), int(nz), float(spacing[0]), float(spacing[1]), float(spacing[2]))


def camera_struct(cam):
    """From any object with persp, width, height, o, d0, du, dv (e.g. phantoms.Camera)."""
    c = abi.Camera()
    c.persp, c.width, c.height = int(cam.persp), int(cam.width), int(cam.height)
    for name in ("o", "d0", "du", "dv"):
        arr = getattr(c, name)
        v = getattr(cam, name)
        for k in range(3):
            arr[k] = float(v[k])
    return c


@dataclass
class Features:
    """Device-resident feature fields.  planar: grad [3][nz][ny][nx], kappa, ves [nz][ny][nx];
    interleaved: grad [nz][ny][nx][8] = (I, gx, gy, gz, kappa, V, 0, 0); split: grad [nz][ny][nx][4] =
    (gx, gy, gz, kappa), ves [nz][ny][nx]; quad: grad as split, ves and iquad [nz][ny][nx][4] quads
    (v(x,y,z), v(x,y+1,z), v(x,y,z+1), v(x,y+1,z+1)) of V and of the intensity; gmax: 1-element tensor."""
    grad: torch.Tensor
    kappa: torch.Tensor | None
    ves: torch.Tensor | None
    gmax: torch.Tensor
    layout: int
    shape: tuple
    spacing: tuple
    bricks: torch.Tensor | None = None  # brick table (flat float32: (min, max) pairs, then mask words), or None
    iquad: torch.Tensor | None = None  # quad layout: [nz][ny][nx][4] intensity quads

    @property
    def dtype(self):
        return self.grad.dtype

    def buf(self):
        return abi.FeaturesBuf(self.grad.data_ptr(), self.kappa.data_ptr() if self.kappa is not None else None,
                               self.ves.data_ptr() if self.ves is not None else None, self.gmax.data_ptr(),
                               _dt(self.grad), self.layout,
                               self.bricks.data_ptr() if self.bricks is not None else None,
                               self.iquad.data_ptr() if self.iquad is not None else None)

    def brick_minmax(self):
        """[nbz][nby][nbx][2] view of the (min, max) part of the brick table."""
        nb = brick_dims(self.shape)
        return self.bricks[:2 * nb[0] * nb[1] * nb[2]].view(*nb, 2)

    def without_bricks(self):
        """The same fields with no brick table (the raymarch then visits every sample)."""
        return Features(self.grad, self.kappa, self.ves, self.gmax, self.layout, self.shape, self.spacing, None,
                        self.iquad)


def _fparams(sigmas, alpha, beta, c, eig_gap):
    fp = abi.FeatureParams()
    if not 1 <= len(sigmas) <= abi.DVR_MAX_SIGMA:
        raise ValueError("1..8 scales")
    fp.nsigma = len(sigmas)
    for i, s in enumerate(sigmas):
        fp.sigma_mm[i] = float(s)
    fp.alpha, fp.beta, fp.c, fp.eig_gap_fp64 = float(alpha), float(beta), float(c), float(eig_gap)
    return fp


def brick_dims(shape_zyx):
    """(nbz, nby, nbx) of the brick table for a [nz][ny][nx] volume."""
    return tuple((n - 1 + abi.DVR_BRICK - 1) // abi.DVR_BRICK for n in shape_zyx)


def alloc_features(shape_zyx, spacing, dtype=torch.float32, layout=abi.DVR_PLANAR, device="cuda", bricks=True):
    """Uninitialized feature fields; bricks=True also allocates the brick table for empty-space skipping."""
    nz, ny, nx = shape_zyx
    if layout == abi.DVR_PLANAR:
        grad = torch.empty((3, nz, ny, nx), dtype=dtype, device=device)
        kappa = torch.empty((nz, ny, nx), dtype=dtype, device=device)
        ves = torch.empty((nz, ny, nx), dtype=dtype, device=device)
    elif layout == abi.DVR_SPLIT:
        grad = torch.empty((nz, ny, nx, 4), dtype=dtype, device=device)
        kappa = None
        ves = torch.empty((nz, ny, nx), dtype=dtype, device=device)
    elif layout == abi.DVR_QUAD:
        grad = torch.empty((nz, ny, nx, 4), dtype=dtype, device=device)
        kappa = None
        ves = torch.empty((nz, ny, nx, 4), dtype=dtype, device=device)
    else:
        grad = torch.empty((nz, ny, nx, 8), dtype=dtype, device=device)
        kappa = ves = None
    gmax = torch.empty(1, dtype=torch.float32, device=device)
    nb = math.prod(brick_dims(shape_zyx))
    bt = torch.empty(2 * nb + (nb + 31) // 32, dtype=torch.float32, device=device) if bricks else None
    iq = torch.empty((nz, ny, nx, 4), dtype=dtype, device=device) if layout == abi.DVR_QUAD else None
    return Features(grad, kappa, ves, gmax, layout, tuple(shape_zyx), tuple(spacing), bt, iq)


def features_workspace_bytes(shape_zyx, spacing, sigmas, alpha=0.5, beta=0.5, c=0.1, eig_gap=1e-3):
    n = C.c_size_t()
    abi.check(lib().dvr_features_workspace(C.byref(grid_struct(shape_zyx, spacing)),
                                           C.byref(_fparams(sigmas, alpha, beta, c, eig_gap)), C.byref(n)))
    return n.value


def features(vol, spacing, sigmas, alpha=0.5, beta=0.5, c=0.1, eig_gap=1e-3, dtype=None, layout=abi.DVR_PLANAR,
             out=None, ws=None):
    """Feature pass (dvr_features): gradient, |grad I|_max, k and vesselness of vol [nz][ny][nx]."""
    _require_cuda(vol)
    dtype = vol.dtype if dtype is None else dtype
    g = grid_struct(vol.shape, spacing)
    fp = _fparams(sigmas, alpha, beta, c, eig_gap)
    out = alloc_features(tuple(vol.shape), spacing, dtype, layout, vol.device) if out is None else out
    nbytes = features_workspace_bytes(tuple(vol.shape), spacing, sigmas, alpha, beta, c, eig_gap)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=vol.device)
    fb = out.buf()
    abi.check(lib().dvr_features(_ptr(vol), _dt(vol), C.byref(g), C.byref(fp), C.byref(fb), _ptr(ws), nbytes,
                                 _stream()))
    return out


def _tf_struct(knots, rgba):
    _require_cuda(knots, rgba)
    if knots.dtype != torch.float32 or rgba.dtype != torch.float32:
        raise TypeError("TF knots and rgba are float32")
    return abi.TF(int(knots.numel()), knots.data_ptr(), rgba.data_ptr())


def _rparams(p):
    return abi.RenderParams(float(p["lambda_g"]), float(p["lambda_k"]), float(p["kappa0"]), float(p["lambda_v"]),
                            float(p["step_vox"]), float(p["et_alpha"]))


def _cams(cams):
    arr = (abi.Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c if isinstance(c, abi.Camera) else camera_struct(c)
    return arr


def render(vol, feats: Features, knots, rgba, params, cams, want_state=True, out=None, counters=None):
    """dvr_render: returns (rgba [ncam][H][W][4], T_last, k_last) (state tensors None if not wanted).
    counters: optional int64 device tensor [2] overwritten with (evaluated, shaded) sample counts."""
    _require_cuda(vol)
    carr = _cams(cams)
    W, H = carr[0].width, carr[0].height
    n = len(cams)
    dev = feats.grad.device
    img = torch.empty((n, H, W, 4), dtype=torch.float32, device=dev) if out is None else out
    T_last = k_last = None
    st = None
    if want_state:
        T_last = torch.empty((n, H, W), dtype=torch.float32, device=dev)
        k_last = torch.empty((n, H, W), dtype=torch.int32, device=dev)
        st = abi.RayState(T_last.data_ptr(), k_last.data_ptr(),
                          counters.data_ptr() if counters is not None else None)
    g = grid_struct(feats.shape, feats.spacing)
    fb = feats.buf()
    tf = _tf_struct(knots, rgba)
    rp = _rparams(params)
    abi.check(lib().dvr_render(_ptr(vol), _dt(vol) if vol is not None else abi.DVR_F32, C.byref(g), C.byref(fb),
                               C.byref(tf), C.byref(rp), carr, n, _ptr(img), C.byref(st) if st else None, _stream()))
    return img, T_last, k_last


def render_gather(vol, feats: Features, knots, rgba, params, cams, k_last, sink=None, counters=None):
    """dvr_render_gather (measurement): the loads of dvr_render over samples 0 .. k_last of each ray,
    without the optics.  Returns the sink tensor [ncam][H][W] (a sum that keeps the loads live).
    counters: optional int64 device tensor [2] overwritten with (walked, feature-fetching) samples."""
    _require_cuda(vol)
    carr = _cams(cams)
    W, H = carr[0].width, carr[0].height
    n = len(cams)
    dev = feats.grad.device
    sink = torch.empty((n, H, W), dtype=torch.float32, device=dev) if sink is None else sink
    g = grid_struct(feats.shape, feats.spacing)
    fb = feats.buf()
    tf = _tf_struct(knots, rgba)
    rp = _rparams(params)
    abi.check(lib().dvr_render_gather(_ptr(vol), _dt(vol) if vol is not None else abi.DVR_F32, C.byref(g),
                                      C.byref(fb), C.byref(tf), C.byref(rp), carr, n, _ptr(k_last), _ptr(sink),
                                      _ptr(counters), _stream()))
    return sink


def render_backward(vol, feats: Features, knots, rgba, params, cams, T_last, k_last, dout, want_dvol=True,
                    want_features=False):
    """dvr_render_backward: returns (dL/dTF [K][4], dL/dvol [nz][ny][nx] or None); with want_features
    (dvr_render_backward_features) also dict(g [3][nz][ny][nx], kappa, V, gmax [1]) of the gradients
    with respect to the feature values."""
    carr = _cams(cams)
    dev = feats.grad.device
    dtf = torch.empty((knots.numel(), 4), dtype=torch.float32, device=dev)
    dvol = torch.empty(feats.shape, dtype=torch.float32, device=dev) if want_dvol else None
    dout = dout.contiguous().float()
    g = grid_struct(feats.shape, feats.spacing)
    fb = feats.buf()
    tf = _tf_struct(knots, rgba)
    rp = _rparams(params)
    st = abi.RayState(T_last.data_ptr(), k_last.data_ptr(), None)
    args = (_ptr(vol), _dt(vol) if vol is not None else abi.DVR_F32, C.byref(g), C.byref(fb), C.byref(tf),
            C.byref(rp), carr, len(cams), C.byref(st), _ptr(dout), _ptr(dtf), _ptr(dvol))
    if not want_features:
        abi.check(lib().dvr_render_backward(*args, _stream()))
        return dtf, dvol
    dfeat = torch.empty((5,) + tuple(feats.shape), dtype=torch.float32, device=dev)
    dgmax = torch.empty(1, dtype=torch.float32, device=dev)
    fg = abi.FeatureGrads(dfeat.data_ptr(), dgmax.data_ptr())
    abi.check(lib().dvr_render_backward_features(*args, C.byref(fg), _stream()))
    return dtf, dvol, dict(g=dfeat[:3], kappa=dfeat[3], V=dfeat[4], gmax=dgmax, packed=dfeat)


def features_backward_workspace_bytes(shape_zyx, spacing, sigmas, alpha=0.5, beta=0.5, c=0.1):
    n = C.c_size_t()
    abi.check(lib().dvr_features_backward_workspace(C.byref(grid_struct(shape_zyx, spacing)),
                                                    C.byref(_fparams(sigmas, alpha, beta, c, 0.0)), C.byref(n)))
    return n.value


def features_backward(vol, spacing, sigmas, fgrads, dvol=None, alpha=0.5, beta=0.5, c=0.1, ws=None):
    """dvr_features_backward: adds dL/dI of the feature pass for the upstream fgrads (the dict that
    render_backward(..., want_features=True) returns, or g [3][...], kappa, V, gmax [1] tensors) to
    dvol (zeros when None) and returns dvol."""
    _require_cuda(vol)
    g = grid_struct(vol.shape, spacing)
    fp = _fparams(sigmas, alpha, beta, c, 0.0)
    packed = fgrads.get("packed")
    if packed is None:
        packed = torch.cat([fgrads["g"].reshape(3, -1), fgrads["kappa"].reshape(1, -1),
                            fgrads["V"].reshape(1, -1)]).float().contiguous()
    dgmax = fgrads["gmax"].reshape(1).float().contiguous()
    if dvol is None:
        dvol = torch.zeros(vol.shape, dtype=torch.float32, device=vol.device)
    n = C.c_size_t()
    abi.check(lib().dvr_features_backward_workspace(C.byref(g), C.byref(fp), C.byref(n)))
    if ws is None or ws.numel() < n.value:
        ws = torch.empty(n.value, dtype=torch.uint8, device=vol.device)
    fg = abi.FeatureGrads(packed.data_ptr(), dgmax.data_ptr())
    abi.check(lib().dvr_features_backward(_ptr(vol), _dt(vol), C.byref(g), C.byref(fp), C.byref(fg), _ptr(dvol),
                                          _ptr(ws), n.value, _stream()))
    return dvol


def normalize(raw, out_dtype=torch.float16):
    """dvr_normalize (Eq. 1) of a device tensor (uint16 counts, float32 or float16)."""
    _require_cuda(raw)
    out = torch.empty(raw.shape, dtype=out_dtype, device=raw.device)
    n = C.c_size_t()
    abi.check(lib().dvr_normalize_workspace(raw.numel(), C.byref(n)))
    ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=raw.device)
    abi.check(lib().dvr_normalize(_ptr(raw), _dt(raw), _ptr(out), _dt(out), raw.numel(), _ptr(ws), n.value,
                                  _stream()))
    return out


def denoise(vol, spacing, mode="median3", sigma_mm=1.0, out=None):
    """dvr_denoise (Sec. 5.3): 3x3x3 median (mode "median3") or separable Gaussian of sigma_mm
    (mode "gauss") of vol [nz][ny][nx] (float32 or float16); returns a new tensor (or out)."""
    _require_cuda(vol)
    m = abi.DVR_DENOISE_MEDIAN3 if mode == "median3" else abi.DVR_DENOISE_GAUSS
    g = grid_struct(vol.shape, spacing)
    n = C.c_size_t()
    abi.check(lib().dvr_denoise_workspace(C.byref(g), m, C.byref(n)))
    ws = torch.empty(max(n.value, 16), dtype=torch.uint8, device=vol.device)
    out = torch.empty_like(vol) if out is None else out
    abi.check(lib().dvr_denoise(_ptr(vol), _dt(vol), C.byref(g), m, float(sigma_mm), _ptr(out), _ptr(ws), n.value,
                                _stream()))
    return out


def histogram(vol, floor=0.0):
    """dvr_histogram (Sec. 2.2): 256-bin counts of the normalized values > floor -> (int64 [256] device
    tensor, number used)."""
    _require_cuda(vol)
    h = torch.empty(256, dtype=torch.int32, device=vol.device)
    used = torch.empty(1, dtype=torch.int32, device=vol.device)
    abi.check(lib().dvr_histogram(_ptr(vol), _dt(vol), vol.numel(), float(floor), _ptr(h), _ptr(used), _stream()))
    return h.long() & 0xFFFFFFFF, int(used.long().item() & 0xFFFFFFFF)


def tissue_peaks(hist, min_sep=2):
    """dvr_tissue_peaks: the three tissue peaks of a 256-bin histogram (device tensor of counts) ->
    (device dvr_peaks buffer, dict(bin, peak, in_window))."""
    _require_cuda(hist)
    h = hist.to(torch.int64).clamp_(0, 0xFFFFFFFF).to(torch.int32) if hist.dtype != torch.int32 else hist.contiguous()
    buf = torch.empty(C.sizeof(abi.Peaks), dtype=torch.uint8, device=hist.device)
    abi.check(lib().dvr_tissue_peaks(_ptr(h), int(min_sep), _ptr(buf), _stream()))
    pk = abi.Peaks.from_buffer_copy(bytes(buf.cpu().numpy()))
    return buf, dict(bin=list(pk.bin), peak=list(pk.peak), in_window=[bool(x) for x in pk.in_window])


def tissue_tf(peaks_buf, colours, taus, tau_hi=0.0, colour_hi=(1.0, 1.0, 1.0)):
    """dvr_tissue_tf: the 8-knot TF of the peaks -> (knots [8], rgba [8][4]) device tensors."""
    p = abi.TissueTFParams()
    for c in range(3):
        for k in range(3):
            p.rgb[c][k] = float(colours[c][k])
        p.tau[c] = float(taus[c])
        p.rgb_hi[c] = float(colour_hi[c])
    p.tau_hi = float(tau_hi)
    knots = torch.empty(8, dtype=torch.float32, device=peaks_buf.device)
    rgba = torch.empty((8, 4), dtype=torch.float32, device=peaks_buf.device)
    abi.check(lib().dvr_tissue_tf(_ptr(peaks_buf), C.byref(p), _ptr(knots), _ptr(rgba), _stream()))
    return knots, rgba


class DVRRender(torch.autograd.Function):
    """rgba = render(vol, TF values) with gradients for the voxel intensities and the TF values
    (knot positions, gradient, k and V are held constant).  The backward is the hand-written adjoint
    raymarch, which recomputes the samples from the stored per-ray (T_last, k_last).

    vol.grad here is the gradient through the TF lookup only: the features are inputs.  For the
    gradient through the features as well (|grad I| / |grad I|_max, k and V of Eq. 4, computed from
    vol), use DVRRenderFromVolume."""

    @staticmethod
    def forward(ctx, vol, tf_rgba, feats, knots, params, cams):
        img, T_last, k_last = render(vol, feats, knots, tf_rgba.contiguous(), params, cams, want_state=True)
        ctx.save_for_backward(vol, tf_rgba, knots, T_last, k_last)
        ctx.feats, ctx.params, ctx.cams = feats, params, cams
        return img

    @staticmethod
    def backward(ctx, dimg):
        vol, tf_rgba, knots, T_last, k_last = ctx.saved_tensors
        dtf, dvol = render_backward(vol, ctx.feats, knots, tf_rgba.contiguous(), ctx.params, ctx.cams, T_last,
                                    k_last, dimg, want_dvol=ctx.needs_input_grad[0])
        return (dvol if ctx.needs_input_grad[0] else None, dtf if ctx.needs_input_grad[1] else None,
                None, None, None, None)


class DVRRenderFromVolume(torch.autograd.Function):
    """rgba = render(vol, features(vol), TF values): the feature pass runs on vol inside the forward,
    and the backward chains the render adjoint with feature gradients (dvr_render_backward_features)
    into the feature-pass adjoint (dvr_features_backward), so vol.grad is the whole dL/dI: through the
    TF lookup and through the gradient, |grad I|_max, k and the vesselness the raymarch reads.

    apply(vol, tf_rgba, knots, params, cams, spacing, sigmas, alpha, beta, c, layout); c must be > 0
    (the automatic Frangi c is not differentiated)."""

    @staticmethod
    def forward(ctx, vol, tf_rgba, knots, params, cams, spacing, sigmas, alpha, beta, c, layout):
        if not (c > 0):
            raise ValueError("DVRRenderFromVolume needs an explicit Frangi c > 0")
        feats = features(vol, spacing, sigmas, alpha=alpha, beta=beta, c=c, layout=layout)
        rv = vol if layout in (abi.DVR_PLANAR, abi.DVR_SPLIT) else None
        img, T_last, k_last = render(rv, feats, knots, tf_rgba.contiguous(), params, cams, want_state=True)
        ctx.save_for_backward(vol, tf_rgba, knots, T_last, k_last)
        ctx.feats, ctx.params, ctx.cams = feats, params, cams
        ctx.fp = (spacing, sigmas, alpha, beta, c, layout)
        return img

    @staticmethod
    def backward(ctx, dimg):
        vol, tf_rgba, knots, T_last, k_last = ctx.saved_tensors
        spacing, sigmas, alpha, beta, c, layout = ctx.fp
        rv = vol if layout in (abi.DVR_PLANAR, abi.DVR_SPLIT) else None
        dtf, dvol, fg = render_backward(rv, ctx.feats, knots, tf_rgba.contiguous(), ctx.params, ctx.cams, T_last,
                                        k_last, dimg, want_dvol=True, want_features=True)
        if ctx.needs_input_grad[0]:
            dvol = features_backward(vol, spacing, sigmas, fg, dvol=dvol, alpha=alpha, beta=beta, c=c)
        return (dvol if ctx.needs_input_grad[0] else None, dtf if ctx.needs_input_grad[1] else None,
                None, None, None, None, None, None, None, None, None)


class Batch:
    """A batched plan (dvr_batch_*): the feature pass of every volume and the raymarch of every view
    in one persistent kernel recorded in a HIP graph.

    vols: list of device volumes [nz][ny][nx]; spacings: list of (hx, hy, hz); feats: list of
    Features (outputs, one per volume, same dtype and layout); views: list of
    (volume index, camera, rgba [H][W][4] tensor, T_last or None, k_last or None).
    The TF tensors are read at every launch: edit them in place to change the transfer function."""

    def __init__(self, vols, spacings, feats, views, sigmas, knots, rgba, params, alpha=0.5, beta=0.5, c=0.1,
                 eig_gap=1e-3, tune=None):
        self._keep = (list(vols), list(feats), list(views), knots, rgba)
        self.desc = self._desc(vols, spacings, feats, views, sigmas, knots, rgba, params, alpha, beta, c, eig_gap, tune)
        self.plan = C.c_void_p()
        abi.check(lib().dvr_batch_create(C.byref(self.desc), C.byref(self.plan)))

    def _desc(self, vols, spacings, feats, views, sigmas, knots, rgba, params, alpha, beta, c, eig_gap, tune):
        self._va = (abi.BatchVolume * len(vols))()
        for i, (v, sp, f) in enumerate(zip(vols, spacings, feats)):
            _require_cuda(v)
            self._va[i] = abi.BatchVolume(v.data_ptr(), _dt(v), grid_struct(v.shape, sp), f.buf())
        self._wa = (abi.BatchView * max(len(views), 1))()
        for i, (vi, cam, img, T, k) in enumerate(views):
            _require_cuda(img)
            self._wa[i] = abi.BatchView(int(vi), cam if isinstance(cam, abi.Camera) else camera_struct(cam),
                                        img.data_ptr(), T.data_ptr() if T is not None else None,
                                        k.data_ptr() if k is not None else None)
        self._tune = None
        if tune is not None:
            self._tune = tune if isinstance(tune, abi.Tune) else abi.Tune(*[int(tune[k]) for k in TUNE_FIELDS])
        d = abi.BatchDesc()
        d.nvol, d.vols = len(vols), self._va
        d.nview, d.views = len(views), self._wa
        d.fp = _fparams(sigmas, alpha, beta, c, eig_gap)
        d.tf = _tf_struct(knots, rgba)
        d.rp = _rparams(params)
        d.tune = C.pointer(self._tune) if self._tune is not None else None
        return d

    def launch(self):
        abi.check(lib().dvr_batch_launch(self.plan, _stream()))

    def check(self):
        abi.check(lib().dvr_batch_check(self.plan, _stream()))

    def close(self):
        if self.plan:
            lib().dvr_batch_destroy(self.plan)
            self.plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def autotune(vols, spacings, feats, views, sigmas, knots, rgba, params, alpha=0.5, beta=0.5, c=0.1, eig_gap=1e-3,
                 cache_path=None):
        """dvr_batch_autotune: returns the fastest tune as a dict (and caches it in cache_path)."""
        tmp = Batch.__new__(Batch)
        d = tmp._desc(vols, spacings, feats, views, sigmas, knots, rgba, params, alpha, beta, c, eig_gap, None)
        t = abi.Tune()
        abi.check(lib().dvr_batch_autotune(C.byref(d), cache_path.encode() if cache_path else None, C.byref(t)))
        return {k: getattr(t, k) for k in TUNE_FIELDS}


TUNE_FIELDS = ("wg_per_cu", "xy_tile", "xy_zrun", "z_chunk", "ray_tile")
