"""The allocation-free contour entry point (litho_contours_noalloc) against
litho_contours, through the C ABI: two calls in a row, the second on a
smaller image, each bit-identical to the allocating entry point (cells,
codes, successors, crossing parameters and the count).  It also refuses an
image side beyond its static scratch.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _run(L, fn, img, level, cap):
    import torch
    n = img.shape[0]
    cell = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    code = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    nxt = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    u = torch.full((cap, 2), -1.0, dtype=torch.float32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = fn(n, img.data_ptr(), float(level), cap, cell.data_ptr(), code.data_ptr(), u.data_ptr(), nxt.data_ptr(),
            cnt.data_ptr(), None)
    assert rc == 0, L._lib.litho_last_error()
    torch.cuda.synchronize()
    return int(cnt.item()), cell.cpu().numpy(), code.cpu().numpy(), u.cpu().numpy(), nxt.cpu().numpy()


def test_noalloc_contours_match_allocating_entry_point():
    import torch
    from paper_2602_15036_amd import litho as L
    for n, seed, level in ((1024, 11, 0.5), (200, 12, 0.45)):
        img = torch.from_numpy(W.curvilinear_mask(n, seed).astype(np.float32)).cuda()
        total, *_ = _run(L, L._lib.litho_contours, img, level, 0)
        cap = total + 16
        ref = _run(L, L._lib.litho_contours, img, level, cap)
        got = _run(L, L._lib.litho_contours_noalloc, img, level, cap)
        assert ref[0] == got[0] == total and total > 0
        for a, b in zip(ref[1:], got[1:]):
            assert np.array_equal(a, b)
    img = torch.zeros((8192, 8), device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert L._lib.litho_contours_noalloc(8192, img.data_ptr(), 0.5, 0, None, None, None, None, cnt.data_ptr(),
                                         None) == L.A.LITHO_E_UNSUPPORTED
