#!/usr/bin/env python3
"""Benchmark of the DVR hot path on one MI355X.

One step = the feature pass of the 181x217x181 FP32 head phantom (gradient, 3-scale Hessian,
curvature, vesselness) followed by the raymarch of all 360 perspective orbit views at 1024^2
(8-knot TF, early termination at alpha >= 0.99).  Inputs are resident in HBM before the timed
region; K steps are timed with HIP events on the stream the kernels are launched on.

The JSON line's value is evaluated ray samples per second over the whole step (feature pass
included).  Components: feature-pass voxels/s, raymarch samples/s, and forward+backward ms per
view of the differentiable-render workload (128^3 phantom, 8 views at 512^2, L2 loss against a
target from a perturbed 16-knot TF).  The roofline object covers the dominant kernel (the
raymarch); the CPU baseline is the FP64 oracle on a bounded sample of the same step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxels/s (features), ray-samples/s + fwd+bwd ms/view; % HBM roofline"
# Dense FP32 vector peak without packed-FP32 instructions (this build forbids them):
# 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.
PEAK_FP32_TFLOPS = 78.6432
PEAK_FP32_PUBLISHED = 157.3
PEAK_HBM_GBS = 8000.0
# Algorithmic flops per raymarch sample (FMA = 2); see the design notes for the breakdown.
FLOP_SHADED = 144
FLOP_TRANSPARENT = 40
RENDER_SOURCES = ["render.hip", "render_dev.hpp", "render_args.hpp", "common.hpp"]
# Feature pass: compulsory bytes per voxel in FP32 (read I, write g, k, V) and the algorithmic flop
# estimate per voxel at three scales (stencils, eigenvalues, vesselness; see the design notes).
FEAT_BYTES_F32 = 24
FEAT_FLOP_3SCALE = 830
FEAT_FLOP_1SCALE = 270


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2605_19737_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key, sha):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(kernel_key)
    if not rec or rec.get("source_sha") != sha:
        return None
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--views", type=int, default=360, help="views per step (the workload has 360)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward-leg", action="store_true")
    ap.add_argument("--no-fp16-leg", action="store_true")
    ap.add_argument("--no-batch-leg", action="store_true")
    ap.add_argument("--no-c5-leg", action="store_true")
    ap.add_argument("--no-feature-adjoint-leg", action="store_true")
    ap.add_argument("--only-main", action="store_true", help="just the timed head-phantom steps (for profiling)")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="just the render adjoint of 8 head views (every 45th) after one forward, without and then "
                         "with the feature gradients (for profiling)")
    ap.add_argument("--only-features", action="store_true",
                    help="just the feature passes, for profiling: the head's 3 scales (quad layout) 4 times, then "
                         "the 512x512x400 volume's single scale in FP32 planar 4 times")
    ap.add_argument("--only-batch", action="store_true",
                    help="just the batched leg (64 volumes, autotuned graph launch against per-call launches), for "
                         "profiling")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling the HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the design notes describe how "
              "the work would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_19737_amd as dvr
    import phantoms

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dvr.lib()
    if args.only_batch:
        out = leg_batch(dev, torch.cuda.current_stream(), dvr, torch, np, log)
        print(json.dumps(out), flush=True)
        return

    # ------------------------------------------------------------------ workload (inputs into HBM)
    log("building the head phantom and cameras")
    w = phantoms.c2(1024, 1024, nviews=args.views)
    vol = torch.from_numpy(w.vol).to(dev)
    knots = torch.from_numpy(w.tf_knots).to(dev)
    tf = torch.from_numpy(w.tf_rgba).to(dev)
    cams = [dvr.camera_struct(c) for c in w.cams]
    nvox = vol.numel()
    nz, ny, nx = vol.shape
    # FP32 features in the quad layout (one (gx, gy, gz, k) record per voxel; V and the intensity as
    # per-voxel (y, z) quads): the same values as planar, a cell's corners in 2 + 8 + 2 loads instead
    # of 8 + 8 + 8.  No brick table here: the head's
    # Rician background leaves few empty 4^3 bricks, and the per-brick lookups cost more than the
    # transparent samples they save (the table pays off where empty space is clean: see the
    # 512x512x400 leg)
    from paper_2605_19737_amd import _abi as abi_
    feats = dvr.alloc_features(tuple(vol.shape), w.spacing, torch.float32, abi_.DVR_QUAD, bricks=False)
    wsb = dvr.features_workspace_bytes(tuple(vol.shape), w.spacing, w.sigmas, c=w.c)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    V = len(cams)
    img = torch.empty((V, 1024, 1024, 4), dtype=torch.float32, device=dev)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    if args.only_features:
        for _ in range(4):
            dvr.features(vol, w.spacing, w.sigmas, c=w.c, layout=feats.layout, out=feats, ws=ws)
        torch.cuda.synchronize()
        del feats, ws, img
        w5 = phantoms.c5(8, 8, views=[0])
        raw = torch.from_numpy(w5.vol.view(np.int16)).to(dev)
        v32 = dvr.normalize(raw, torch.float32)
        f32 = dvr.alloc_features(tuple(raw.shape), w5.spacing, torch.float32, abi_.DVR_PLANAR, bricks=False)
        ws32 = torch.empty(dvr.features_workspace_bytes(tuple(raw.shape), w5.spacing, w5.sigmas, c=w5.c),
                           dtype=torch.uint8, device=dev)
        for _ in range(4):
            dvr.features(v32, w5.spacing, w5.sigmas, c=w5.c, eig_gap=1e-3, layout=abi_.DVR_PLANAR, out=f32, ws=ws32)
        if args.copy_calibration:
            src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
            torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        log("feature passes done (head x4, 512x512x400 single scale x4)")
        return

    if args.only_adjoint:
        dvr.features(vol, w.spacing, w.sigmas, c=w.c, layout=feats.layout, out=feats, ws=ws)
        sel = cams[::45][:8]
        im8, T8, k8 = dvr.render(vol, feats, knots, tf, w.params, sel)
        g = torch.Generator(device=dev).manual_seed(45)
        dout = 0.01 * torch.randn(im8.shape, generator=g, device=dev)
        dvr.render_backward(vol, feats, knots, tf, w.params, sel, T8, k8, dout)
        dvr.render_backward(vol, feats, knots, tf, w.params, sel, T8, k8, dout, want_features=True)
        torch.cuda.synchronize()
        log("adjoint of 8 head views done (without, then with the feature gradients)")
        return

    def step(timing=None):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        dvr.features(vol, w.spacing, w.sigmas, c=w.c, layout=feats.layout, out=feats, ws=ws)
        e1.record(stream)
        _, T, k = dvr.render(vol, feats, knots, tf, w.params, cams, out=img)
        e2.record(stream)
        if timing is not None:
            timing.append((e0, e1, e2))
        return T, k

    log(f"warmup x{args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps of {V} views")
    timing = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        T_last, k_last = step(timing)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_feat = sum(a.elapsed_time(b) for a, b, _ in timing) / 1e3
    t_rend = sum(b.elapsed_time(c) for _, b, c in timing) / 1e3
    t_step = sum(a.elapsed_time(c) for a, _, c in timing) / 1e3
    # sample counts from one instrumented render after the timed steps (the counts are deterministic;
    # the counters' same-address atomics would otherwise add ~0.15 ms per view to the timed raymarch)
    dvr.render(vol, feats, knots, tf, w.params, cams, out=img, counters=counters)
    evaluated, shaded = (int(x) for x in counters.cpu().tolist())
    # nominal samples (every segment midpoint of every ray, no early termination): the same walk with a
    # TF of zero extinction everywhere, whose rays all run to the end of their chord, untimed
    tf_clear = tf.clone()
    tf_clear[:, 3] = 0.0
    p_clear = dict(w.params)
    p_clear["et_alpha"] = 0.0
    dvr.render(vol, feats, knots, tf_clear, p_clear, cams, out=img, counters=counters)
    nominal = int(counters[0].item())
    log(f"step {1e3 * t_step / args.steps:.2f} ms (features {1e3 * t_feat / args.steps:.3f} ms, render "
        f"{1e3 * t_rend / args.steps:.2f} ms); samples/step evaluated {evaluated:.4g} shaded {shaded:.4g}; wall {wall:.2f}s")

    K = args.steps
    # gather ceiling: the same rays, samples and loads without the optics (dvr_render_gather), timed
    # the same way on the same stream; its counters must equal the forward pass's
    sink = torch.empty((V, 1024, 1024), dtype=torch.float32, device=dev)
    cg = torch.zeros(2, dtype=torch.int64, device=dev)
    dvr.render_gather(vol, feats, knots, tf, w.params, cams, k_last, sink=sink, counters=cg)
    torch.cuda.synchronize()
    if [int(x) for x in cg.cpu().tolist()] != [evaluated, shaded]:
        raise RuntimeError(f"gather walk counts {cg.cpu().tolist()} differ from the raymarch's {[evaluated, shaded]}")
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(K):
        dvr.render_gather(vol, feats, knots, tf, w.params, cams, k_last, sink=sink)
    g1.record(stream)
    torch.cuda.synchronize()
    t_gather = g0.elapsed_time(g1) / 1e3
    del sink
    samples_per_s = evaluated * K / t_step
    render_sps = evaluated * K / t_rend
    vox_per_s = nvox * K / t_feat
    launches_per_step = math.ceil(V / 32)
    render_launch_s = t_rend / (K * launches_per_step)
    flops_per_step = shaded * FLOP_SHADED + (evaluated - shaded) * FLOP_TRANSPARENT
    achieved_tflops = flops_per_step * K / t_rend / 1e12
    sha = source_sha(RENDER_SOURCES)
    tr = load_traffic("render_head_1024_persp", sha)
    traffic = None
    if tr is not None:
        traffic = {"fetch_bytes_per_launch": tr["fetch_bytes_per_launch"],
                   "write_bytes_per_launch": tr["write_bytes_per_launch"],
                   "hbm_gbs": (tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"]) / render_launch_s / 1e9,
                   "views_per_launch": tr.get("views_per_launch"), "source_sha": sha}
    # The raymarch is bound by its gathers (texture-path counters), not by HBM bytes or ALU: the
    # roofline is the measured gather ceiling, the same walk and loads without the optics; the ALU
    # fraction (shaded and transparent samples at their own flop counts) against the published
    # FP32 peak stands beside it.
    gather_sps = evaluated * K / t_gather
    roofline = {"bound": "gather", "achieved": round(render_sps / 1e9, 3), "peak": round(gather_sps / 1e9, 3),
                "unit": "Gsamples/s", "frac": round(render_sps / gather_sps, 4),
                "traffic": traffic, "kernel": "k_render (FP32 quad layout, K<=8)",
                "avg_launch_ms": round(1e3 * render_launch_s, 4),
                "gather_kernel": "k_render_gather (same rays, samples and loads; no Eq. 4, exp or compositing)",
                "gather_avg_launch_ms": round(1e3 * t_gather / (K * launches_per_step), 4),
                "samples_per_launch": evaluated / launches_per_step,
                "alu": {"achieved": round(achieved_tflops, 3), "peak": PEAK_FP32_PUBLISHED, "unit": "TFLOP/s",
                        "frac": round(achieved_tflops / PEAK_FP32_PUBLISHED, 4),
                        "flops_per_launch": flops_per_step / launches_per_step,
                        "flop_per_sample": {"shaded": FLOP_SHADED, "transparent": FLOP_TRANSPARENT},
                        "frac_of_unpacked_fp32_peak": round(achieved_tflops / PEAK_FP32_TFLOPS, 4)}}

    comps = {"features_voxels_per_s": vox_per_s, "features_ms": 1e3 * t_feat / K,
             "features_hbm_frac": FEAT_BYTES_F32 * vox_per_s / (PEAK_HBM_GBS * 1e9),
             "features_valu_frac": FEAT_FLOP_3SCALE * vox_per_s / (PEAK_FP32_TFLOPS * 1e12),
             "render_samples_per_s": render_sps, "render_ms_per_view": 1e3 * t_rend / (K * V),
             "samples_evaluated_per_step": evaluated, "samples_shaded_per_step": shaded,
             "rays_per_step": V * 1024 * 1024, "samples_nominal_per_step": nominal,
             "nominal_samples_per_s": nominal * K / t_step}

    # ------------------------------------------------------------------ fwd+bwd ms/view leg
    if args.only_main:
        args.no_backward_leg = args.no_fp16_leg = args.no_batch_leg = args.no_c5_leg = True
        args.no_feature_adjoint_leg = True
        args.no_cpu_baseline = True
    if not args.no_fp16_leg:
        comps["fp16_records"] = leg_fp16(w, vol, knots, tf, cams, stream, K, dvr, torch, log)
    if not args.no_batch_leg:
        comps["batched"] = leg_batch(dev, stream, dvr, torch, np, log)
    if not args.no_c5_leg:
        comps["c5_fp16_fwd_bwd"] = leg_c5(dev, stream, dvr, torch, np, log)
    if not args.no_backward_leg:
        log("differentiable-render leg: 128^3, 8 views at 512^2, forward + adjoint")
        w3 = phantoms.c3(512, 512)
        v3 = torch.from_numpy(w3.vol).to(dev)
        k3 = torch.from_numpy(w3.tf_knots).to(dev)
        tf3 = torch.from_numpy(w3.tf_rgba).to(dev)
        tgt_tf = torch.from_numpy(w3.extra["target_tf_rgba"]).to(dev)
        c3 = [dvr.camera_struct(c) for c in w3.cams]
        from paper_2605_19737_amd import _abi as abi3
        # quad layout, no brick table (the fastest forward + adjoint on this workload)
        f3 = dvr.features(v3, w3.spacing, w3.sigmas, c=w3.c, layout=abi3.DVR_QUAD).without_bricks()
        target, _, _ = dvr.render(v3, f3, k3, tgt_tf, w3.params, c3, want_state=False)
        times = []
        for it in range(8):
            a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            a.record(stream)
            im, T3, kl3 = dvr.render(v3, f3, k3, tf3, w3.params, c3)
            b.record(stream)
            dvr.render_backward(v3, f3, k3, tf3, w3.params, c3, T3, kl3, im - target)
            c.record(stream)
            torch.cuda.synchronize()
            if it >= 2:
                times.append((a.elapsed_time(b), b.elapsed_time(c)))
        fw = float(np.median([t[0] for t in times]))
        bw = float(np.median([t[1] for t in times]))
        comps.update({"fwd_bwd_ms_per_view": (fw + bw) / len(c3), "fwd_ms_per_view": fw / len(c3),
                      "bwd_ms_per_view": bw / len(c3), "fwd_bwd_workload": "128^3 phantom, 8 ortho views 512^2, 16-knot TF, FP32 quad layout"})
        log(f"fwd+bwd {comps['fwd_bwd_ms_per_view']:.3f} ms/view (fwd {fw / 8:.3f}, bwd {bw / 8:.3f})")

    if not args.no_feature_adjoint_leg:
        comps["feature_adjoint"] = leg_feature_adjoint(w, vol, feats, knots, tf, cams, stream, dvr, torch, np, log)

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # ------------------------------------------------------------------ CPU baseline (oracle)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        nv_cpu = min(36, V)
        sel = [w.cams[(i * V) // nv_cpu] for i in range(nv_cpu)]
        log(f"CPU baseline: FP64 oracle, full feature pass + {nv_cpu} whole views of the {V}")
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        sp = tuple(float(np.float32(h)) for h in w.spacing)
        prm = {k: float(np.float32(v)) for k, v in w.params.items()}
        v64 = w.vol.astype(np.float64)
        t = time.perf_counter()
        of = oracle.features(v64, sp, [float(np.float32(s)) for s in w.sigmas], c=float(np.float32(w.c)))
        t_cf = time.perf_counter() - t
        t = time.perf_counter()
        ro = oracle.render(v64, of, of["gmax"], sp, w.tf_knots, w.tf_rgba, prm, sel)
        t_cr = time.perf_counter() - t
        s_per_sample = t_cr / max(ro["nsamp"], 1)
        t_cpu_step = t_cf + s_per_sample * evaluated
        one = cpu_one_thread(oracle, w, v64, of, sp, prm, evaluated, nvox, np, log)
        cpu = {"value": evaluated / t_cpu_step, "unit": "ray-samples/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(), "one_thread": one,
               "sample": f"FP64 oracle: full 3-scale feature pass ({t_cf:.2f} s) + {nv_cpu} whole 1024^2 views "
                         f"evenly spaced over the {V} ({ro['nsamp']} samples, {t_cr:.2f} s); step time = features "
                         f"+ per-sample time x the step's {evaluated} evaluated samples",
               "features_voxels_per_s": nvox / t_cf, "render_samples_per_s": ro["nsamp"] / t_cr}
        log(f"CPU baseline {cpu['value']:.4g} samples/s on {threads} threads")

    # the 60 %-of-HBM goal for the feature pass and the raymarch, stated against what was measured
    goal = {"goal_frac_of_hbm": 0.6, "met": False,
            "features_head_3_scales": comps["features_hbm_frac"],
            "raymarch_measured_traffic": (traffic["hbm_gbs"] / PEAK_HBM_GBS if traffic else None),
            "why": "neither kernel is bound by HBM: the feature pass by executed instructions (~381 VALU per voxel "
                   "at one scale, VALU issue ~86 %), the raymarch by its gathers (at 0.92 of the measured "
                   "gather ceiling, texture data ~96 % busy) with ~0.73 TB/s of traffic"}
    c5 = comps.get("c5_fp16_fwd_bwd")
    if c5:
        goal["features_512x512x400_single_scale_fp32"] = c5["single_scale_fp32_features_hbm_frac"]
        goal["features_512x512x400_fp16"] = c5["features_hbm_frac"]
    comps["hbm_goal"] = goal

    out = {"metric": METRIC, "value": samples_per_s, "unit": "ray-samples/s", "n_gpus": 1, "steps": K,
           "warmup": args.warmup, "ms_per_step": 1e3 * t_step / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"head phantom {nx}x{ny}x{nz} FP32 at 1 mm with 24 vessel tubes and 3% Rician "
                                  f"noise; features at sigma {{1,2,3}} mm; {V} perspective orbit views at 1024^2, "
                                  f"step 0.5 voxel, 8-knot TF, early termination 0.99",
                      "voxels": nvox, "views": V, "image": [1024, 1024]},
           "roofline": roofline, "cpu_baseline": cpu, "components": comps}
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_one_thread(oracle, w, v64, of, sp, prm, evaluated, nvox, np, log):
    """The oracle on one thread (OpenMP limited to 1 for the call): the feature pass on a 24-slice
    slab of the head, scaled to the whole volume, and the central 128 x 128 pixels of 16 views, scaled to
    the step's evaluated samples (the render sample reads the whole-volume features of)."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(1)
    try:
        z0 = v64.shape[0] // 2 - 12
        slab = np.ascontiguousarray(v64[z0:z0 + 24])
        t = time.perf_counter()
        oracle.features(slab, sp, [float(np.float32(s)) for s in w.sigmas], c=float(np.float32(w.c)))
        t_f = (time.perf_counter() - t) * nvox / slab.size
    finally:
        gomp.omp_set_num_threads(prev)
    # 16 views evenly spaced over the orbit, a 128 x 128 pixel block at the image centre of each (where
    # the rays cross the head), in row order: 2^18 rays walked as the whole-view baseline walks them
    nv = len(w.cams)
    cams = [w.cams[(i * nv) // 16] for i in range(min(16, nv))]
    H, W = cams[0].height, cams[0].width
    b = min(128, H, W)
    y0, x0 = (H - b) // 2, (W - b) // 2
    vv, yy, xx = np.meshgrid(np.arange(len(cams)), np.arange(y0, y0 + b), np.arange(x0, x0 + b), indexing="ij")
    pix = np.stack([vv.ravel(), yy.ravel(), xx.ravel()], 1).astype(np.int32)
    M = len(pix)
    gomp.omp_set_num_threads(1)
    try:
        t = time.perf_counter()
        ro = oracle.render(v64, of, of["gmax"], sp, w.tf_knots, w.tf_rgba, prm, cams, pix=pix)
        t_r = time.perf_counter() - t
    finally:
        gomp.omp_set_num_threads(prev)
    per_sample = t_r / max(ro["nsamp"], 1)
    value = evaluated / (t_f + per_sample * evaluated)
    log(f"CPU one thread: features {t_f:.1f} s (scaled), {ro['nsamp']} samples in {t_r:.1f} s")
    return {"value": value, "unit": "ray-samples/s", "cores": 1,
            "sample": f"FP64 oracle on one thread: the 3-scale feature pass on 24 of {v64.shape[0]} slices "
                      f"({t_f * slab.size / nvox:.2f} s, scaled by the voxel count) + the central {b}x{b} pixels "
                      f"of 16 views spread over the orbit ({M} rays, {ro['nsamp']} samples, {t_r:.2f} s, scaled "
                      f"to the step's samples)",
            "features_voxels_per_s": nvox / t_f, "render_samples_per_s": ro["nsamp"] / t_r}


def leg_feature_adjoint(w, vol, feats, knots, tf, cams, stream, dvr, torch, np, log):
    """Gradient through the morphology terms on the head: the render adjoint with feature gradients
    (8 views spread over the orbit) against the plain adjoint, and the feature-pass adjoint (3 scales)
    that takes dL/d(g, k, V, gmax) to dL/dI."""
    log("feature-adjoint leg: head, 8 views, render adjoint with feature gradients + feature-pass adjoint")
    sel = cams[:: max(1, len(cams) // 8)][:8]
    img, T, k = dvr.render(vol, feats, knots, tf, w.params, sel)
    dout = torch.randn(img.shape, generator=torch.Generator(device=img.device).manual_seed(7), device=img.device)
    dvol = torch.zeros_like(vol)
    nfb = dvr.features_backward_workspace_bytes(tuple(vol.shape), w.spacing, w.sigmas, c=w.c)
    wsb = torch.empty(nfb, dtype=torch.uint8, device=vol.device)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    plain = timed(lambda: dvr.render_backward(vol, feats, knots, tf, w.params, sel, T, k, dout))
    res = {}

    def with_feat():
        res["r"] = dvr.render_backward(vol, feats, knots, tf, w.params, sel, T, k, dout, want_features=True)

    fgt = timed(with_feat)
    fg = res["r"][2]
    fb = timed(lambda: dvr.features_backward(vol, w.spacing, w.sigmas, fg, dvol=dvol, c=w.c, ws=wsb))
    N = vol.numel()
    # compulsory bytes of the feature-pass adjoint: read I (4) and dL/d(g, k, V) (20), read and write dL/dI (8)
    out = {"render_bwd_ms_per_view": plain / len(sel), "render_bwd_feature_grads_ms_per_view": fgt / len(sel),
           "features_backward_ms": fb, "features_backward_voxels_per_s": N / (fb * 1e-3),
           "features_backward_hbm_frac": 32.0 * N / (fb * 1e-3) / 8e12, "workspace_bytes": nfb,
           "workload": f"head {tuple(vol.shape)} FP32 quad layout, sigma {{1,2,3}} mm, {len(sel)} views 1024^2"}
    log(f"render adjoint {out['render_bwd_ms_per_view']:.3f} ms/view, with feature gradients "
        f"{out['render_bwd_feature_grads_ms_per_view']:.3f} ms/view; feature-pass adjoint {fb:.2f} ms")
    return out


def leg_fp16(w, vol, knots, tf, cams, stream, K, dvr, torch, log):
    """Same head workload with FP16 volume and FP16 quad-layout features (FP32 arithmetic)."""
    from paper_2605_19737_amd import _abi as abi
    log("FP16 leg: same step with an FP16 volume and FP16 quad-layout features")
    v16 = vol.half()
    f16 = dvr.alloc_features(tuple(vol.shape), w.spacing, torch.float16, abi.DVR_QUAD, bricks=False)
    ws = torch.empty(dvr.features_workspace_bytes(tuple(vol.shape), w.spacing, w.sigmas, c=w.c), dtype=torch.uint8,
                     device=vol.device)
    img = torch.empty((len(cams), 1024, 1024, 4), dtype=torch.float32, device=vol.device)
    cnt = torch.zeros(2, dtype=torch.int64, device=vol.device)
    ev = []
    for it in range(K + 1):
        a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a.record(stream)
        dvr.features(v16, w.spacing, w.sigmas, c=w.c, dtype=torch.float16, layout=abi.DVR_QUAD, out=f16, ws=ws)
        b.record(stream)
        dvr.render(None, f16, knots, tf, w.params, cams, out=img)
        c.record(stream)
        if it > 0:
            ev.append((a, b, c))
    torch.cuda.synchronize()
    tf_ = sum(a.elapsed_time(b) for a, b, _ in ev) / 1e3
    tr = sum(b.elapsed_time(c) for _, b, c in ev) / 1e3
    dvr.render(None, f16, knots, tf, w.params, cams, out=img, counters=cnt)  # counts, untimed
    evaluated = int(cnt[0].item())
    out = {"samples_per_s": evaluated * K / (tf_ + tr), "render_samples_per_s": evaluated * K / tr,
           "render_ms_per_view": 1e3 * tr / (K * len(cams)), "features_ms": 1e3 * tf_ / K,
           "image_error_bound": "compute 1e-5 of range given the stored FP16 values; storage 2^-11 per feature; "
                                "end to end 5.4e-4 max / 1.2e-5 mean measured at 512x512x400"}
    log(f"FP16 quad features: {out['samples_per_s']:.4g} samples/s over the step ({out['render_ms_per_view']:.3f} ms/view)")
    return out


def leg_batch(dev, stream, dvr, torch, np, log, nvol=64):
    """64 uneven anisotropic volumes, features + 4 views each at 512^2, in one persistent graph launch
    (autotuned), against the same work as per-call launches."""
    import phantoms
    log(f"batched leg: building {nvol} volumes")
    ws = [phantoms.c4_volume(b, 512, 512) for b in range(nvol)]
    vols = [torch.from_numpy(w.vol).to(dev) for w in ws]
    sps = [w.spacing for w in ws]
    from paper_2605_19737_amd import _abi as abi_b
    # split layout on both sides of the comparison (on these small thick-slice volumes the quad layout's
    # extra quad-building step costs the batched launch more than its two-load corners save: 85.8 vs 83.1 ms)
    lay = abi_b.DVR_SPLIT
    # no brick tables on either side: on these volumes the per-call raymarch ran 84.8 ms with them and
    # 82.0 ms without (the lookups cost more than the transparent samples they skip)
    feats = [dvr.alloc_features(tuple(v.shape), sp, torch.float32, lay, bricks=False) for v, sp in zip(vols, sps)]
    views = []
    for i, w in enumerate(ws):
        for cam in w.cams:
            views.append((i, dvr.camera_struct(cam), torch.empty((512, 512, 4), dtype=torch.float32, device=dev),
                          None, None))
    knots = torch.from_numpy(ws[0].tf_knots).to(dev)
    tf = torch.from_numpy(ws[0].tf_rgba).to(dev)
    nvox = sum(v.numel() for v in vols)
    log("batched leg: autotuning")
    tune = dvr.Batch.autotune(vols, sps, feats, views, ws[0].sigmas, knots, tf, ws[0].params, c=ws[0].c,
                              cache_path=os.path.join("/tmp", "dvr_tune_cache.json"))
    b = dvr.Batch(vols, sps, feats, views, ws[0].sigmas, knots, tf, ws[0].params, c=ws[0].c, tune=tune)
    b.launch()
    b.check()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record(stream)
    for _ in range(reps):
        b.launch()
    e1.record(stream)
    b.check()
    t_batch = e0.elapsed_time(e1) / 1e3 / reps
    b.close()
    # the same work as per-call launches (features per volume, then 4 views per volume), with counters
    cnt = torch.zeros(2, dtype=torch.int64, device=dev)
    total = 0
    pf = [dvr.alloc_features(tuple(v.shape), sp, torch.float32, lay, bricks=False) for v, sp in zip(vols, sps)]
    wsp = [torch.empty(dvr.features_workspace_bytes(tuple(v.shape), sp, ws[0].sigmas, c=ws[0].c), dtype=torch.uint8,
                       device=dev) for v, sp in zip(vols, sps)]
    imgs = [torch.empty((4, 512, 512, 4), dtype=torch.float32, device=dev) for _ in vols]

    def per_call(count):
        nonlocal total
        for i, (w, v, sp) in enumerate(zip(ws, vols, sps)):
            dvr.features(v, sp, w.sigmas, c=w.c, layout=lay, out=pf[i], ws=wsp[i])
            dvr.render(v, pf[i], knots, tf, w.params, [dvr.camera_struct(c) for c in w.cams], out=imgs[i],
                       counters=cnt if count else None)
            if count:
                torch.cuda.synchronize()
                total += int(cnt[0].item())

    per_call(True)
    e0.record(stream)
    per_call(False)
    e1.record(stream)
    torch.cuda.synchronize()
    t_calls = e0.elapsed_time(e1) / 1e3
    out = {"volumes": nvol, "voxels": nvox, "views": len(views), "image": [512, 512], "tune": tune,
           "graph_launch_ms": 1e3 * t_batch, "samples_evaluated": total, "samples_per_s": total / t_batch,
           "per_call_ms": 1e3 * t_calls, "per_call_samples_per_s": total / t_calls,
           "graph_speedup": t_calls / t_batch,
           "like_for_like": "both sides: split FP32 features, no brick tables, the same TF, sigma and views"}
    log(f"batched: {1e3 * t_batch:.2f} ms per graph launch ({total / t_batch:.4g} samples/s) vs per-call "
        f"{1e3 * t_calls:.2f} ms ({total / t_calls:.4g} samples/s); tune {tune}")
    return out


def leg_c5(dev, stream, dvr, torch, np, log):
    """512x512x400 uint16 -> Eq. 1 -> FP16 records -> 8 views at 2048^2, forward + adjoint."""
    import phantoms
    from paper_2605_19737_amd import _abi as abi
    log("FP16 scale leg: 512x512x400 uint16, 8 views at 2048^2, forward + adjoint")
    w = phantoms.c5(2048, 2048)
    raw = torch.from_numpy(w.vol.view(np.int16)).to(dev)
    knots = torch.from_numpy(w.tf_knots).to(dev)
    tf = torch.from_numpy(w.tf_rgba).to(dev)
    tgt = torch.from_numpy(w.extra["target_tf_rgba"]).to(dev)
    cams = [dvr.camera_struct(c) for c in w.cams]
    f = dvr.alloc_features(tuple(raw.shape), w.spacing, torch.float16, abi.DVR_INTERLEAVED)
    wsf = torch.empty(dvr.features_workspace_bytes(tuple(raw.shape), w.spacing, w.sigmas, c=w.c),
                      dtype=torch.uint8, device=dev)
    cnt = torch.zeros(2, dtype=torch.int64, device=dev)
    times = []
    for it in range(3):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        v16 = dvr.normalize(raw, torch.float16)
        ev[1].record(stream)
        dvr.features(v16, w.spacing, w.sigmas, c=w.c, eig_gap=1e-3, dtype=torch.float16, layout=abi.DVR_INTERLEAVED,
                     out=f, ws=wsf)
        ev[2].record(stream)
        img, T, k = dvr.render(None, f, knots, tf, w.params, cams)
        ev[3].record(stream)
        if it == 0:
            target, _, _ = dvr.render(None, f, knots, tgt, w.params, cams, want_state=False)
        dvr.render_backward(None, f, knots, tf, w.params, cams, T, k, img - target)
        ev[4].record(stream)
        torch.cuda.synchronize()
        if it > 0:
            times.append([ev[i].elapsed_time(ev[i + 1]) for i in range(4)])
    t = np.median(np.array(times), axis=0)
    dvr.render(None, f, knots, tf, w.params, cams, counters=cnt)  # sample counts, untimed
    evaluated = int(cnt[0].item())
    # automatic tissue windows on the normalized volume: histogram (2 B/voxel read), peaks, TF
    ht = []
    for it in range(4):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        h, _ = dvr.histogram(v16, 0.0)
        e1.record(stream)
        buf, pk = dvr.tissue_peaks(h, 2)
        kn_t, tf_t = dvr.tissue_tf(buf, [(0.2, 0.4, 1.0), (0.9, 0.6, 0.5), (1.0, 0.95, 0.85)], (0.1, 0.3, 0.6))
        e2.record(stream)
        torch.cuda.synchronize()
        if it > 0:
            ht.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
    th = float(np.median([x[0] for x in ht]))
    # optional denoise pre-pass (3x3x3 median of the FP16 volume: 2 B read + 2 B written per voxel)
    dn = torch.empty_like(v16)
    dt_ = []
    for it in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dvr.denoise(v16, w.spacing, "median3", out=dn)
        e1.record(stream)
        torch.cuda.synchronize()
        if it > 0:
            dt_.append(e0.elapsed_time(e1))
    tdn = float(np.median(dt_))
    # the single-scale method on this large volume in FP32 (planar features: the compulsory 24 B/voxel,
    # read I, write g, k, V; ~270 flop/voxel): the one configuration near the HBM ridge
    v32 = dvr.normalize(raw, torch.float32)
    f32 = dvr.alloc_features(tuple(raw.shape), w.spacing, torch.float32, abi.DVR_PLANAR, bricks=False)
    ws32 = torch.empty(dvr.features_workspace_bytes(tuple(raw.shape), w.spacing, w.sigmas, c=w.c),
                       dtype=torch.uint8, device=dev)
    t32 = []
    for it in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dvr.features(v32, w.spacing, w.sigmas, c=w.c, eig_gap=1e-3, layout=abi.DVR_PLANAR, out=f32, ws=ws32)
        e1.record(stream)
        torch.cuda.synchronize()
        if it > 0:
            t32.append(e0.elapsed_time(e1))
    tf32 = float(np.median(t32))
    del v32, f32, ws32
    out = {"normalize_ms": float(t[0]), "features_ms": float(t[1]), "fwd_ms_per_view": float(t[2]) / 8,
           "bwd_ms_per_view": float(t[3]) / 8, "fwd_bwd_ms_per_view": float(t[2] + t[3]) / 8,
           "features_voxels_per_s": raw.numel() / (t[1] / 1e3), "render_samples_per_s": evaluated / (t[2] / 1e3),
           # compulsory bytes: normalize reads 2 B twice (reduce, scale) and writes 2 B
           "normalize_hbm_frac": 6 * raw.numel() / (t[0] / 1e3) / (PEAK_HBM_GBS * 1e9),
           "histogram_ms": th, "histogram_hbm_frac": 2 * raw.numel() / (th / 1e3) / (PEAK_HBM_GBS * 1e9),
           "tissue_peaks": pk,
           # the median is ALU work: 388 min/max per voxel (forgetful selection over 27 values) against
           # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 32-bit operations per second
           "median3_ms": tdn, "median3_hbm_frac": 4 * raw.numel() / (tdn / 1e3) / (PEAK_HBM_GBS * 1e9),
           "median3_alu_frac": 388.0 * raw.numel() / (tdn / 1e3) / 3.93216e13,
           # the feature pass's compulsory bytes: read the 2-byte volume, write g, k, V in FP16 (10 B)
           "features_hbm_frac": 12 * raw.numel() / (t[1] / 1e3) / (PEAK_HBM_GBS * 1e9),
           "single_scale_fp32_features_ms": tf32,
           "single_scale_fp32_features_voxels_per_s": raw.numel() / (tf32 / 1e3),
           "single_scale_fp32_features_hbm_frac": FEAT_BYTES_F32 * raw.numel() / (tf32 / 1e3) / (PEAK_HBM_GBS * 1e9),
           "single_scale_fp32_features_valu_frac": FEAT_FLOP_1SCALE * raw.numel() / (tf32 / 1e3) / (PEAK_FP32_TFLOPS * 1e12)}
    log(f"C5: normalize {t[0]:.2f} ms, features {t[1]:.2f} ms, fwd {t[2] / 8:.2f} ms/view, bwd {t[3] / 8:.2f} ms/view")
    return out


if __name__ == "__main__":
    main()
