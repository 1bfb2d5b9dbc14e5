"""The allocation-free normalize (dvr_normalize_noalloc, for callers that cannot allocate) against
dvr_normalize, called through the C ABI on the same inputs: bit-identical outputs on two calls in a
row, the second with a smaller input whose range lies inside the first's (a reduction that kept the
previous call's min and max would show there), for U16 -> F16 and F32 -> F32 (ragged lengths)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2605_19737_amd import _abi as abi

pytestmark = pytest.mark.gpu


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _with_ws(L, raw, rdt, out, odt):
    n = C.c_size_t()
    abi.check(L.dvr_normalize_workspace(raw.numel(), C.byref(n)))
    ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device="cuda")
    abi.check(L.dvr_normalize(C.c_void_p(raw.data_ptr()), rdt, C.c_void_p(out.data_ptr()), odt, raw.numel(),
                              C.c_void_p(ws.data_ptr()), n.value, _stream()))


def _no_alloc(L, raw, rdt, out, odt):
    abi.check(L.dvr_normalize_noalloc(C.c_void_p(raw.data_ptr()), rdt, C.c_void_p(out.data_ptr()), odt, raw.numel(),
                                      _stream()))


@pytest.mark.parametrize("kind", ["u16_f16", "f32_f32"])
def test_noalloc_matches_workspace_entry_point(kind):
    L = abi.load()
    rng = np.random.default_rng(19737)
    sizes = [(512, 512, 3), (37, 29, 11)]  # the second smaller and ragged (not a multiple of 8)
    ranges = [(100, 60000), (5000, 20000)]  # the second range strictly inside the first
    for (nz, ny, nx), (lo, hi) in zip(sizes, ranges):
        if kind == "u16_f16":
            a = rng.integers(lo, hi + 1, size=(nz, ny, nx)).astype(np.uint16)
            raw = torch.from_numpy(a.view(np.int16)).cuda()
            rdt, odt, tdt = abi.DVR_U16, abi.DVR_F16, torch.float16
        else:
            a = rng.uniform(lo, hi, size=(nz, ny, nx)).astype(np.float32)
            raw = torch.from_numpy(a).cuda()
            rdt, odt, tdt = abi.DVR_F32, abi.DVR_F32, torch.float32
        ref = torch.full(raw.shape, float("nan"), dtype=tdt, device="cuda")
        got = torch.full(raw.shape, float("nan"), dtype=tdt, device="cuda")
        _with_ws(L, raw, rdt, ref, odt)
        _no_alloc(L, raw, rdt, got, odt)
        torch.cuda.synchronize()
        r = ref.view(torch.int16 if tdt == torch.float16 else torch.int32).cpu().numpy()
        g = got.view(torch.int16 if tdt == torch.float16 else torch.int32).cpu().numpy()
        print(f"{kind} {nz}x{ny}x{nx}: {int((r != g).sum())} differing elements", flush=True)
        assert np.array_equal(r, g)
        # the call's own min and max define the output: 0 at the minimum, 1 at the maximum
        v = got.float().cpu().numpy()
        assert v.min() == 0.0 and v.max() == 1.0


def test_noalloc_rejects_bad_arguments():
    L = abi.load()
    x = torch.zeros(64, dtype=torch.float32, device="cuda")
    assert L.dvr_normalize_noalloc(None, abi.DVR_F32, C.c_void_p(x.data_ptr()), abi.DVR_F32, 64, _stream()) == -2
    assert L.dvr_normalize_noalloc(C.c_void_p(x.data_ptr()), abi.DVR_F32, C.c_void_p(x.data_ptr() + 4), abi.DVR_F32, 8,
                                   _stream()) == -3
    assert L.dvr_normalize_noalloc(C.c_void_p(x.data_ptr()), abi.DVR_F32, C.c_void_p(x.data_ptr()), abi.DVR_F32, 0,
                                   _stream()) == -1
