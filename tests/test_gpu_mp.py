"""Split-precision modes against the FP64 oracle (through the C ABI).

Inner grids 32 P <= 1024 of the resampled route (here 96, 160, 320 and the
1024^2 bench batch's 640) run the forward row pass as two MFMA DFT stages
with FP32 column passes; the others (Q = N, and the 4096^2 tile's 2560) run
the column passes as band DFT-GEMMs.  Each mode's relative L2 error of the
image and the gradient is printed (run with -s to see the table).  The gates
sit at about three times the largest error measured for the mode over these
tests (128-4096 clips, 1-3 planes, both placements), so that an accuracy
regression of a few times fails:
  f16x3:  image 5.7e-7, gradient 1.1e-6 measured (FP32 level: hi*hi + hi*lo + lo*hi of 11-bit halves);
  bf16x3: image 5.3e-6, gradient 9.2e-6 measured (~2^-16 per product);
  f16:    image 4.1e-4, gradient 7.4e-4 measured (one 11-bit term);
  bf16:   image 3.3e-3, gradient 6.0e-3 measured (one 8-bit term).
FP32 keeps the path's own gates (image 1e-5, gradient 1e-4).
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

MODES = ["fp32", "f16x3", "bf16x3", "f16", "bf16"]
IMG_GATE = {"fp32": 1e-5, "f16x3": 2e-6, "bf16x3": 1.5e-5, "f16": 1.2e-3, "bf16": 9e-3}
GRAD_GATE = {"fp32": 1e-4, "f16x3": 4e-6, "bf16x3": 3e-5, "f16": 2.5e-3, "bf16": 1.7e-2}
SLOPE, THR = 50.0, 0.3


def rel_l2(a, b):
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def L():
    from paper_2602_15036_amd import litho
    return litho


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _banks(spec, K):
    return [O.socs_kernels(spec, F, K=K) for F in spec.focus_nm]


@pytest.mark.parametrize("n,inner", [(128, 0), (256, 0), (256, 256), (512, 0)])
def test_mp_image_and_gradient_mid_sizes(L, n, inner):
    # three focus planes, dipole source; inner grids 96 (n=128), 160, 256, 320
    spec = W.fd_clip_optics(n).with_(K=12)
    bank = L.Bank.from_spec(spec)
    bank.set_inner_grid(inner)
    m = W.as_f32_exact(W.curvilinear_mask(n, 70 + n))
    T = W.manhattan_target(n, 71 + n)
    banks = _banks(spec, 12)
    Lo, go, imgs = O.gradient(m, T, banks, SLOPE, THR)
    rows = []
    for mode in MODES:
        img, loss, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR,
                                       prec=mode)
        e_img = max(rel_l2(img.cpu().numpy()[0, p], imgs[p]) for p in range(3))
        e_grad = rel_l2(grad.cpu().numpy()[0], go)
        e_loss = abs(loss.item() - Lo) / Lo
        rows.append((mode, e_img, e_grad, e_loss))
    for mode, e_img, e_grad, e_loss in rows:
        print(f"n={n} Q={bank.inner_grid} {mode:7s} image {e_img:.2e} grad {e_grad:.2e} loss {e_loss:.2e}")
    for mode, e_img, e_grad, _ in rows:
        assert e_img < IMG_GATE[mode], (mode, e_img)
        assert e_grad < GRAD_GATE[mode], (mode, e_grad)


def test_mp_bench_launch_config(L):
    # 1024 x 1024, K = 24, batch of 16 (inner grid 640): sampled pixels vs the
    # oracle and the whole batch vs the FP32 path
    spec = W.CONFIG2
    bank = L.Bank.from_spec(spec)
    masks = np.stack([W.as_f32_exact(W.curvilinear_mask(1024, 1000 + s)) for s in range(16)])
    d = dev(masks)
    ref32 = L.image(bank, d).cpu().numpy()
    lam, phi = O.socs_kernels(spec, 0.0, K=24)
    rng = np.random.default_rng(5)
    ys = rng.integers(0, 1024, 64)
    xs = rng.integers(0, 1024, 64)
    refs = {i: O.image_at(O.mask_spectrum(masks[i], bank.b, "fft"), lam, phi, 1024, ys, xs) for i in (0, 15)}
    for mode in MODES[1:]:
        img = L.image(bank, d, prec=mode).cpu().numpy()
        e32 = rel_l2(img, ref32)
        eo = max(rel_l2(img[i, 0][ys, xs], refs[i]) for i in refs)
        print(f"1024x16 K=24 {mode:7s} vs fp32 {e32:.2e} vs oracle (sampled) {eo:.2e}")
        assert eo < IMG_GATE[mode], (mode, eo)


GOLDEN_4096 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tile4096_gradient_window.npz")


def test_mp_full_tile_4096_window(L):
    # 4096 x 4096, three planes, K = 32: image on the central 256 x 256 window
    # vs the oracle, loss and gradient window vs the oracle's stored values
    # (tests/golden/make_tile4096_gradient_window.py), gradient vs the FP32 path
    gold = np.load(GOLDEN_4096)
    y0, x0, h = (int(v) for v in gold["window"])
    assert (y0, x0, h) == (1920, 1920, 256)
    spec = W.CONFIG5
    bank = L.Bank.from_spec(spec)
    m = W.as_f32_exact(W.curvilinear_mask(4096, 4000))
    T = W.manhattan_target(4096, 4001)
    mh = O.mask_spectrum(m, bank.b, "fft")
    refs = []
    for F in spec.focus_nm:
        lam, phi = O.socs_kernels(spec, F, K=32)
        refs.append(O.image_window(mh, lam, phi, 4096, 1920, 1920, 256, 256))
    win = (slice(1920, 2176), slice(1920, 2176))
    out = {}
    for mode in MODES:
        img, loss, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR,
                                       prec=mode)
        out[mode] = (img.cpu().numpy()[0], grad.cpu().numpy()[0], loss.item())
    g32 = out["fp32"][1]
    for mode in MODES:
        img, grad, loss = out[mode]
        e_img = max(rel_l2(img[p][win], refs[p]) for p in range(3))
        e_go = rel_l2(grad[win], gold["grad"])
        e_lo = abs(loss - float(gold["loss"])) / float(gold["loss"])
        e_g = rel_l2(grad, g32)
        print(f"4096 P=3 K=32 {mode:7s} vs oracle: image(window) {e_img:.2e} grad(window) {e_go:.2e} "
              f"loss {e_lo:.2e} | grad vs fp32 (tile) {e_g:.2e}")
        assert e_img < IMG_GATE[mode], (mode, e_img)
        assert e_go < GRAD_GATE[mode], (mode, e_go)
        assert e_lo < 10 * IMG_GATE[mode], (mode, e_lo)
        assert e_g < GRAD_GATE[mode], (mode, e_g)


def test_mp_mode_validation(L):
    bank = L.Bank.from_spec(W.CONFIG1)
    m = dev(W.manhattan_mask(128, 1)[None])
    with pytest.raises(L.LithoError):
        L.image(bank, m, prec=7)
    with pytest.raises(ValueError):
        L.image(bank, m, prec="fp8")
