"""Gather ceiling (dvr_render_gather): the measurement walk visits exactly the samples the forward
raymarch evaluated and fetches feature corners for exactly the samples it shaded, so its two counters
equal the forward pass's, for every layout and storage type, with and without the brick table."""
import numpy as np
import pytest
import torch

import paper_2605_19737_amd as dvr
import phantoms
from paper_2605_19737_amd import _abi as abi
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("layout,dtype,bricks", [
    (abi.DVR_PLANAR, torch.float32, True), (abi.DVR_PLANAR, torch.float16, False),
    (abi.DVR_INTERLEAVED, torch.float32, False), (abi.DVR_INTERLEAVED, torch.float16, True),
    (abi.DVR_SPLIT, torch.float32, False), (abi.DVR_SPLIT, torch.float16, False),
    (abi.DVR_QUAD, torch.float32, False), (abi.DVR_QUAD, torch.float16, False)])
def test_gather_walks_the_forward_samples(layout, dtype, bricks):
    w = phantoms.c2(96, 80, views=[0, 77, 200])
    vol = to_dev(w.vol, dtype)
    print(f"[gather] layout {layout} {dtype} bricks {bricks}", flush=True)
    f = dvr.features(vol, w.spacing, w.sigmas, c=w.c, dtype=dtype, layout=layout)
    if not bricks:
        f = f.without_bricks()
    kn, tf = to_dev(w.tf_knots), to_dev(w.tf_rgba)
    cf = torch.zeros(2, dtype=torch.int64, device="cuda")
    cg = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    vv = vol if layout in (abi.DVR_PLANAR, abi.DVR_SPLIT) else None
    img, T, k = dvr.render(vv, f, kn, tf, w.params, w.cams, counters=cf)
    sink = dvr.render_gather(vv, f, kn, tf, w.params, w.cams, k, counters=cg)
    torch.cuda.synchronize()
    a, b = cf.cpu().tolist(), cg.cpu().tolist()
    assert a[0] == int((k.long() + 1).sum()) and a[0] > 0 and 0 < a[1] < a[0]
    assert a == b, (a, b)
    assert torch.isfinite(sink).all()
    # rays that miss the volume walk nothing
    assert bool((sink[k < 0] == 0).all())


def test_gather_rejects_missing_buffers():
    w = phantoms.c1(16, 16)
    vol = to_dev(w.vol)
    f = dvr.features(vol, w.spacing, w.sigmas, c=w.c)
    kn, tf = to_dev(w.tf_knots), to_dev(w.tf_rgba)
    with pytest.raises(dvr.DVRError) as e:
        dvr.render_gather(vol, f, kn, tf, w.params, w.cams, None)
    assert e.value.status == -2  # DVR_E_NULL
