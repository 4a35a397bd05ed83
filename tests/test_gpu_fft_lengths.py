"""Every transform length the library supports, through the Gaussian
low-pass of a clip of that side (forward row DFT of real rows, column DFTs
both ways, band multiply, inverse row DFT to real rows), against the oracle's
FP64 periodic Gaussian filter.  Together with the imaging tests (which run the
per-kernel passes on each inner grid they reach) this exercises every FFT
plan and its LDS exchange schedule on the GPU.  Gate: 1e-6 of the image's
largest value (FP32 transforms of length <= 4096; measured 1.4e-7 to 5.6e-7).
"""
import numpy as np
import pytest

import oracle.post as OP
import workloads as W

pytestmark = pytest.mark.gpu

LENGTHS = [64, 96, 128, 160, 192, 256, 320, 384, 512, 640, 768, 1024, 1280, 1536, 2048, 2560, 3072, 4096]


@pytest.fixture(scope="module")
def L():
    from paper_2602_15036_amd import litho
    return litho


@pytest.mark.parametrize("n", LENGTHS)
def test_lowpass_at_every_supported_side(L, n):
    import torch
    bank = L.Bank.from_spec(W.fd_clip_optics(n).with_(K=2))
    rng = np.random.default_rng(9000 + n)
    imgs = np.stack([W.manhattan_target(n, 90 + n), rng.uniform(0, 1, (n, n))]).astype(np.float32)
    # sigma 1.5 px keeps most of the spectrum (the band reaches |f| ~ 0.79 n,
    # clamped below Nyquist); sigma n / 16 keeps a narrow band
    for s in (1.5, n / 16.0):
        got = L.lowpass(bank, torch.from_numpy(imgs).cuda(), s).cpu().numpy()
        for i in range(2):
            ref = OP.gaussian_filter(imgs[i].astype(np.float64), s)
            err = np.abs(got[i] - ref).max() / np.abs(imgs[i]).max()
            print(f"lowpass n={n} sigma={s:g} image {i}: max err {err:.2e}")
            assert err < 1e-6, (n, s, i, err)
