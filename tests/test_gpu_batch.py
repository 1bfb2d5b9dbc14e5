"""Batched persistent launch (dvr_batch_*): the features of several uneven, anisotropic volumes and
4 views of each, in one persistent kernel recorded in a HIP graph.  On eight volumes of the
64-volume set at 512^2 the launch is compared with the FP64 oracle directly (features of every
volume, one whole view of each and sampled pixels of the other three).  Every volume's features and
every view's image and ray state also equal the standalone dvr_features / dvr_render results bitwise
(the same arithmetic per voxel and per ray), for every tile shape the autotuner can choose; a TF
edited in place is picked up by the next replay; the dependency-wait timeout path reports
DVR_E_TIMEOUT while the kernel still exits normally."""
import os

import numpy as np
import pytest
import torch

import paper_2605_19737_amd as dvr
import phantoms
from paper_2605_19737_amd import _abi as abi
import oracle  # noqa: E402  (the checker)
from tests.gpu_common import compare_features, compare_images, f32, feats_np, oracle_params, sp32, to_dev

pytestmark = pytest.mark.gpu


def _scene(nvol=5, res=96, layout=abi.DVR_PLANAR, dtype=torch.float32, sigmas=(1.0,)):
    ws = [phantoms.c4_volume(b, res, res) for b in range(nvol)]
    vols = [to_dev(w.vol, dtype) for w in ws]
    spacings = [w.spacing for w in ws]
    feats = [dvr.alloc_features(tuple(v.shape), sp, dtype, layout) for v, sp in zip(vols, spacings)]
    views = []
    for i, w in enumerate(ws):
        for cam in w.cams:
            img = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device="cuda")
            T = torch.empty((cam.height, cam.width), dtype=torch.float32, device="cuda")
            k = torch.empty((cam.height, cam.width), dtype=torch.int32, device="cuda")
            views.append((i, cam, img, T, k))
    knots, rgba = to_dev(ws[0].tf_knots), to_dev(ws[0].tf_rgba)
    return ws, vols, spacings, feats, views, knots, rgba, list(sigmas)


def _standalone(ws, vols, spacings, views, knots, rgba, sigmas, layout, dtype):
    out_f, out_v = [], []
    for w, v, sp in zip(ws, vols, spacings):
        out_f.append(dvr.features(v, sp, sigmas, c=w.c, dtype=dtype, layout=layout))
    for (i, cam, _, _, _) in views:
        vv = vols[i] if layout != abi.DVR_INTERLEAVED else None
        out_v.append(dvr.render(vv, out_f[i], knots, rgba, ws[i].params, [cam]))
    return out_f, out_v


def _assert_equal(feats, views, ref_f, ref_v):
    for a, b in zip(feats, ref_f):
        assert torch.equal(a.grad, b.grad)
        if a.kappa is not None:
            assert torch.equal(a.kappa, b.kappa)
        if a.ves is not None:
            assert torch.equal(a.ves, b.ves)
        if a.iquad is not None:
            assert torch.equal(a.iquad, b.iquad)
        assert torch.equal(a.gmax, b.gmax)
    for (i, cam, img, T, k), (rimg, rT, rk) in zip(views, ref_v):
        assert torch.equal(img, rimg[0]) and torch.equal(T, rT[0]) and torch.equal(k, rk[0])


def test_batch_against_oracle_c4_subset():
    """Volumes 0-7 of the 64-volume batched set (uneven shapes from 100x219x123 to 252x124x71, 2.2-6.1 M
    voxels, in-plane 0.54-1.10 mm, slices 3.6-5.0 mm), each with its 4 orthographic 512^2 views, in one graph launch with the split
    layout the benchmark's batched leg uses.  Every volume's g, kappa, V and |g|_max against the oracle
    (1e-5 / 1e-6); view 0 of every volume whole and 3000 sampled pixels of each other view (RGBA and
    T_last within 1e-5, k_last equal)."""
    nvol = 8
    ws = [phantoms.c4_volume(b, 512, 512) for b in range(nvol)]
    vols = [to_dev(w.vol) for w in ws]
    sps = [w.spacing for w in ws]
    lay = abi.DVR_SPLIT
    feats = [dvr.alloc_features(tuple(v.shape), sp, torch.float32, lay) for v, sp in zip(vols, sps)]
    views = []
    for i, w in enumerate(ws):
        for cam in w.cams:
            views.append((i, cam, torch.empty((512, 512, 4), dtype=torch.float32, device="cuda"),
                          torch.empty((512, 512), dtype=torch.float32, device="cuda"),
                          torch.empty((512, 512), dtype=torch.int32, device="cuda")))
    knots, rgba = to_dev(ws[0].tf_knots), to_dev(ws[0].tf_rgba)
    print(f"[batch-oracle] {nvol} volumes {[tuple(v.shape) for v in vols]}, {len(views)} views 512^2", flush=True)
    b = dvr.Batch(vols, sps, feats, views, ws[0].sigmas, knots, rgba, ws[0].params, c=ws[0].c)
    b.launch()
    b.check()
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    for i, w in enumerate(ws):
        sp = sp32(w.spacing)
        v64 = vols[i].cpu().numpy().astype(np.float64)
        of = oracle.features(v64, sp, [f32(s) for s in w.sigmas], c=f32(w.c), want_lam=True)
        compare_features(feats_np(feats[i]), of, f"batched volume {i} {tuple(v64.shape)}")
        mine = [vw for vw in views if vw[0] == i]
        prm = oracle_params(w.params)
        et = f32(w.params["et_alpha"])
        # view 0 whole
        _, cam, img, T, k = mine[0]
        ref = oracle.render(v64, of, of["gmax"], sp, w.tf_knots, w.tf_rgba, prm, [cam])
        compare_images(img[None], T[None], k[None], ref, et, f"batched volume {i} view 0 (whole)")
        # views 1-3 on sampled pixels
        M = 3000
        pix = np.stack([rng.integers(0, 3, M), rng.integers(0, 512, M), rng.integers(0, 512, M)], 1).astype(np.int32)
        cams = [vw[1] for vw in mine[1:]]
        ref = oracle.render(v64, of, of["gmax"], sp, w.tf_knots, w.tf_rgba, prm, cams, pix=pix)
        compare_images(torch.stack([vw[2] for vw in mine[1:]]), torch.stack([vw[3] for vw in mine[1:]]),
                       torch.stack([vw[4] for vw in mine[1:]]), ref, et, f"batched volume {i} views 1-3 (sampled)",
                       pix=pix)
    b.close()


@pytest.mark.parametrize("tune", [None, dict(wg_per_cu=2, xy_tile=1, xy_zrun=3, z_chunk=5, ray_tile=1),
                                  dict(wg_per_cu=8, xy_tile=2, xy_zrun=1, z_chunk=64, ray_tile=2)])
def test_batch_equals_standalone(tune):
    ws, vols, spacings, feats, views, knots, rgba, sig = _scene()
    print(f"[batch] {len(vols)} volumes {[tuple(v.shape) for v in vols]}, {len(views)} views, tune {tune}", flush=True)
    b = dvr.Batch(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c, tune=tune)
    b.launch()
    b.check()
    ref_f, ref_v = _standalone(ws, vols, spacings, views, knots, rgba, sig, abi.DVR_PLANAR, torch.float32)
    torch.cuda.synchronize()
    _assert_equal(feats, views, ref_f, ref_v)
    # replay twice more: counters and |g|_max are reset by the graph itself
    b.launch()
    b.launch()
    b.check()
    _assert_equal(feats, views, ref_f, ref_v)
    b.close()


@pytest.mark.parametrize("layout,dtype", [(abi.DVR_SPLIT, torch.float32), (abi.DVR_SPLIT, torch.float16),
                                          (abi.DVR_QUAD, torch.float32), (abi.DVR_QUAD, torch.float16)])
def test_batch_split_and_quad_equal_standalone(layout, dtype):
    """The split layout (I and V planes, (gx, gy, gz, k) records) and the quad layout (whose V and
    intensity quads the launch builds in Q items after each volume's last scale) in the batched
    launch, two scales."""
    ws, vols, spacings, feats, views, knots, rgba, sig = _scene(nvol=3, layout=layout, dtype=dtype,
                                                                sigmas=(1.0, 2.0))
    b = dvr.Batch(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c)
    b.launch()
    b.check()
    ref_f, ref_v = _standalone(ws, vols, spacings, views, knots, rgba, sig, layout, dtype)
    torch.cuda.synchronize()
    _assert_equal(feats, views, ref_f, ref_v)
    b.launch()
    b.check()
    _assert_equal(feats, views, ref_f, ref_v)
    b.close()


def test_batch_multiscale_fp16_interleaved():
    ws, vols, spacings, feats, views, knots, rgba, sig = _scene(nvol=3, layout=abi.DVR_INTERLEAVED,
                                                                dtype=torch.float16, sigmas=(1.0, 2.0))
    b = dvr.Batch(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c)
    b.launch()
    b.check()
    ref_f, ref_v = _standalone(ws, vols, spacings, views, knots, rgba, sig, abi.DVR_INTERLEAVED, torch.float16)
    torch.cuda.synchronize()
    _assert_equal(feats, views, ref_f, ref_v)
    b.close()


def test_batch_tf_update_without_new_plan():
    """The TF is read from device memory at each replay (the paper's uniform-buffer interaction)."""
    ws, vols, spacings, feats, views, knots, rgba, sig = _scene(nvol=2)
    b = dvr.Batch(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c)
    b.launch()
    b.check()
    rgba.copy_(to_dev(phantoms.perturb_tf(np.random.default_rng(2), ws[0].tf_rgba)))
    b.launch()
    b.check()
    ref_f, ref_v = _standalone(ws, vols, spacings, views, knots, rgba, sig, abi.DVR_PLANAR, torch.float32)
    torch.cuda.synchronize()
    _assert_equal(feats, views, ref_f, ref_v)
    b.close()


def test_batch_autotune_and_cache(tmp_path):
    ws, vols, spacings, feats, views, knots, rgba, sig = _scene(nvol=3, res=64)
    cache = str(tmp_path / "tune.json")
    t = dvr.Batch.autotune(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c, cache_path=cache)
    print(f"[batch] autotuned {t}", flush=True)
    assert os.path.exists(cache) and open(cache).read().count("[") == 1
    t2 = dvr.Batch.autotune(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c, cache_path=cache)
    assert t2 == t
    b = dvr.Batch(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c, tune=t)
    b.launch()
    b.check()
    ref_f, ref_v = _standalone(ws, vols, spacings, views, knots, rgba, sig, abi.DVR_PLANAR, torch.float32)
    torch.cuda.synchronize()
    _assert_equal(feats, views, ref_f, ref_v)
    b.close()


def test_batch_timeout_reported(monkeypatch):
    """Host-forced condition: the rays of volume 0 wait for one feature item more than exist, with a
    short bound; the launch finishes and dvr_batch_check reports DVR_E_TIMEOUT."""
    ws, vols, spacings, feats, views, knots, rgba, sig = _scene(nvol=2, res=32)
    monkeypatch.setenv("DVR_BATCH_TEST_TIMEOUT", "1")
    b = dvr.Batch(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c)
    monkeypatch.delenv("DVR_BATCH_TEST_TIMEOUT")
    b.launch()
    with pytest.raises(dvr.DVRError) as e:
        b.check()
    assert e.value.status == -8
    b.close()
    b2 = dvr.Batch(vols, spacings, feats, views, sig, knots, rgba, ws[0].params, c=ws[0].c)
    b2.launch()
    b2.check()
    b2.close()
