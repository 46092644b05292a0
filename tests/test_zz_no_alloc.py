"""The allocation-free peak search (asp_find_peak_noalloc) against the
context's asp_find_peak on the same images, through the C ABI: two calls in
a row, the second on a smaller image (the shared scratch must not carry the
first call's keys), and the host-side refusals."""
import ctypes

import numpy as np
import pytest

import skygen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
asp = pytest.importorskip("paper_1606_07872_amd")


def image(H, W, seed):
    rng = np.random.default_rng(seed)
    img = rng.normal(0.0, 1.0, size=(H, W)).astype(np.float32)
    # a tie of the maximum |R| at two pixels, the lower index must win
    m = float(np.abs(img).max()) + 1.0
    img.flat[(H * W) // 3] = -m
    img.flat[(2 * H * W) // 3] = m
    return img


def noalloc_peak(img, stream):
    H, W = img.shape
    R = torch.from_numpy(img).cuda()
    idx = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    val = torch.zeros((1,), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    rc = asp.lib().asp_find_peak_noalloc(R.data_ptr(), H, W, idx.data_ptr(), val.data_ptr(),
                                         stream.cuda_stream)
    assert rc == asp.ASP_OK
    stream.synchronize()
    return int(idx.item()), float(val.item())


def context_peak(img):
    psf = skygen.gaussian_psf(15, 3.0).astype(np.float32)
    ctx = asp.Context(img, psf, 0.1, 0.0, max_iter=10)
    rc, idx, val = ctx.find_peak()
    ctx.close()
    return int(idx), float(val)


def test_noalloc_peak_matches_find_peak_twice():
    stream = torch.cuda.Stream()
    for shape, seed in [((4096, 4096), 1), ((301, 257), 2)]:
        img = image(*shape, seed)
        print("noalloc peak", shape, flush=True)
        got = noalloc_peak(img, stream)
        want = context_peak(img)
        assert got[0] == want[0] and np.float32(got[1]) == np.float32(want[1]), (shape, got, want)
        a = np.abs(img.ravel())
        assert got[0] == int(np.flatnonzero(a == a.max())[0])


def test_noalloc_peak_refusals():
    img = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
    out_i = torch.zeros((1,), dtype=torch.int64, device="cuda")
    out_v = torch.zeros((1,), dtype=torch.float32, device="cuda")
    L = asp.lib()
    # beyond the maximum size: refused on the host before any launch
    assert L.asp_find_peak_noalloc(img.data_ptr(), 70000, 70000, out_i.data_ptr(),
                                   out_v.data_ptr(), None) == asp.ASP_ERR_INVALID_ARG
    # an image that is not 16-byte aligned
    assert L.asp_find_peak_noalloc(img.data_ptr() + 4, 8, 8, out_i.data_ptr(),
                                   out_v.data_ptr(), None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_find_peak_noalloc(None, 8, 8, out_i.data_ptr(), out_v.data_ptr(),
                                   None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_find_peak_noalloc(img.data_ptr(), 0, 8, out_i.data_ptr(), out_v.data_ptr(),
                                   None) == asp.ASP_ERR_INVALID_ARG
