"""Properties of the GPU image that hold at any size, checked at full size
(the 16-clip 1024^2 batch and the 4096^2 three-plane tile): circular-shift
equivariance, x- and y-mirror symmetry for sources symmetric under those
mirrors, I(+F) = I(-F) for a real mask with a centrosymmetric source and a
defocus-only pupil, non-negativity, and linearity of the adjoint
(<G, J v> = <J^T G, v> through the VJP mode).  Tolerance: 1e-6 relative L2
(FP32 arithmetic on both sides of each identity).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-6


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def L():
    from paper_2602_15036_amd import litho
    return litho


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_shift_and_mirror_at_the_bench_size(L):
    spec = W.CONFIG2
    bank = L.Bank.from_spec(spec)
    masks = np.stack([W.as_f32_exact(W.curvilinear_mask(1024, 1000 + s)) for s in range(16)]).astype(np.float32)
    img = L.image(bank, dev(masks)).cpu().numpy()[:, 0]
    assert img.min() >= -1e-6 * img.max()
    shifted = np.roll(np.roll(masks, 37, axis=1), -211, axis=2)
    img_s = L.image(bank, dev(shifted)).cpu().numpy()[:, 0]
    assert rel_l2(img_s, np.roll(np.roll(img, 37, axis=1), -211, axis=2)) < TOL
    # mirrors: index i -> (n - i) mod n along x, then along y
    mx = np.roll(masks[:, :, ::-1], 1, axis=2)
    img_mx = L.image(bank, dev(mx)).cpu().numpy()[:, 0]
    assert rel_l2(img_mx, np.roll(img[:, :, ::-1], 1, axis=2)) < TOL
    my = np.roll(masks[:, ::-1, :], 1, axis=1)
    img_my = L.image(bank, dev(my)).cpu().numpy()[:, 0]
    assert rel_l2(img_my, np.roll(img[:, ::-1, :], 1, axis=1)) < TOL


def test_focus_symmetry_shift_and_positivity_at_4096(L):
    spec = W.CONFIG5.with_(focus_nm=(-30.0, 30.0), K=16)
    bank = L.Bank.from_spec(spec)
    m = W.as_f32_exact(W.curvilinear_mask(4096, 4000)).astype(np.float32)
    img = L.image(bank, dev(m[None])).cpu().numpy()[0]
    assert img.min() >= -1e-6 * img.max()
    assert rel_l2(img[0], img[1]) < TOL
    ms = np.roll(m, (1024, -333), axis=(0, 1))
    img_s = L.image(bank, dev(ms[None])).cpu().numpy()[0]
    assert rel_l2(img_s[0], np.roll(img[0], (1024, -333), axis=(0, 1))) < TOL


def test_adjoint_identity_at_the_bench_size(L):
    # <G, J v> = <J^T G, v>: J v by a central difference of the image (a
    # linear check of the adjoint, independent of the oracle), at 1024^2
    import torch
    spec = W.CONFIG2
    bank = L.Bank.from_spec(spec)
    m = W.as_f32_exact(W.curvilinear_mask(1024, 1000)).astype(np.float32)
    rng = np.random.default_rng(12)
    G = np.zeros((1, 1, 1024, 1024), np.float32)        # supported around v, so rounding far away cancels
    G[0, 0, 440:624, 240:424] = rng.standard_normal((184, 184))
    _, _, g = L.image_grad(bank, dev(m[None]), grad_image=dev(G), want_image=False)
    g = g.cpu().numpy()[0].astype(np.float64)
    v = np.zeros((1024, 1024))
    v[500:564, 300:364] = rng.standard_normal((64, 64))
    h = 5e-2
    ip = L.image(bank, dev((m + h * v)[None])).cpu().numpy()[0, 0].astype(np.float64)
    im = L.image(bank, dev((m - h * v)[None])).cpu().numpy()[0, 0].astype(np.float64)
    jv = (ip - im) / (2 * h)              # exact for the quadratic image up to rounding
    lhs = float(np.sum(G[0, 0] * jv))
    rhs = float(np.sum(g * v))
    assert abs(lhs - rhs) < 1e-4 * abs(rhs), (lhs, rhs)
    del torch
