"""Full-size GPU parity against the FP64 oracle and its stored finite differences.

* Every pixel of the bench batch's images (four of the sixteen 1024 x 1024
  clips, K = 24) and of the 2048 x 2048 three-plane images, on each inner grid
  the library can choose for them (automatic, the other supported sides,
  the full grid).
* Finite differences (the gradient check of the through-focus ILT step):
  every pixel of the periodic 64 x 64 clip, and eight directions supported on
  64 x 64 windows of the 2048 x 2048 clip; the FD values are stored under
  tests/golden/ by scripts that call only the oracle.
* The 4096 x 4096 three-plane tile (K = 32) on the inner grids 3072 and 4096
  (the full grid, whose transforms span two wavefronts): window image against
  the oracle, loss and gradient window against the oracle's stored values.

Gates: image relative L2 <= 1e-5, gradient <= 1e-4 (relative L2 against the
oracle's gradient, and against every finite difference relative to the
largest), loss relative <= 1e-5.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

ITOL, GTOL = 1e-5, 1e-4
SLOPE, THR = 50.0, 0.3
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


# ---------------------------------------------------------------- 1024 x 1024 x 16, K = 24

@pytest.fixture(scope="module")
def bench_batch():
    spec = W.CONFIG2
    masks = np.stack([W.as_f32_exact(W.curvilinear_mask(1024, 1000 + s)) for s in range(16)])
    lam, phi = O.socs_kernels(spec, 0.0, K=24)
    refs = {i: O.image(masks[i], lam, phi, method="fft") for i in (0, 5, 10, 15)}
    return spec, masks, refs


@pytest.mark.parametrize("inner", [0, 768, 1024])
def test_bench_batch_full_images(L, bench_batch, inner):
    spec, masks, refs = bench_batch
    bank = L.Bank.from_spec(spec)
    bank.set_inner_grid(inner)
    assert bank.inner_grid == (640 if inner == 0 else inner)
    img = L.image(bank, dev(masks)).cpu().numpy()
    assert img.shape == (16, 1, 1024, 1024)
    assert np.isfinite(img).all() and img.min() >= 0
    errs = {i: rel_l2(img[i, 0], ref) for i, ref in refs.items()}
    print(f"1024x16 K=24 Q={bank.inner_grid}: image rel L2 per clip {errs}")
    for i, e in errs.items():
        assert e < ITOL, (i, e)


# ---------------------------------------------------------------- 2048 x 2048, three planes, K = 24

@pytest.fixture(scope="module")
def clip2048():
    spec = W.CONFIG3
    m = W.as_f32_exact(W.curvilinear_mask(2048, 2000))
    T = W.manhattan_target(2048, 2001)
    Lo, go, Io = O.gradient(m, T, _banks(spec, 24), SLOPE, THR, method="fft")
    return spec, m, T, Lo, go, Io


@pytest.mark.parametrize("inner", [0, 1536, 2048])
def test_through_focus_2048_full(L, clip2048, inner):
    spec, m, T, Lo, go, Io = clip2048
    bank = L.Bank.from_spec(spec)
    bank.set_inner_grid(inner)
    assert bank.inner_grid == (1280 if inner == 0 else inner)
    img, loss, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR)
    img, g = img.cpu().numpy()[0], grad.cpu().numpy()[0]
    e_img = [rel_l2(img[p], Io[p]) for p in range(3)]
    e_loss = abs(loss.item() - Lo) / Lo
    e_grad = rel_l2(g, go)
    print(f"2048 P=3 K=24 Q={bank.inner_grid}: image {e_img} loss {e_loss:.2e} grad {e_grad:.2e}")
    for p in range(3):
        assert e_img[p] < ITOL, (p, e_img[p])
    assert e_loss < ITOL
    assert e_grad < GTOL
    assert rel_l2(g[992:1056, 992:1056], go[992:1056, 992:1056]) < GTOL
    # the eight stored directional finite differences (same clip, optics, loss)
    gold = np.load(os.path.join(GOLDEN, "fd2048_directions.npz"))
    assert tuple(gold["seeds"][:2]) == (2000, 2001)
    win = int(gold["v"].shape[-1])
    for d, ((y, x), v) in enumerate(zip(gold["windows"], gold["v"])):
        got = float(np.sum(g[y:y + win, x:x + win].astype(np.float64) * v))
        fd = float(gold["fd_richardson"][d])
        print(f"  direction {d} at ({y},{x}): <grad, v> {got:.8e} fd {fd:.8e} rel {abs(got - fd) / abs(fd):.2e}")
        assert abs(got - fd) <= GTOL * abs(fd), (d, got, fd)


# ---------------------------------------------------------------- 64 x 64, every pixel

def test_gradient_every_pixel_fd_64(L):
    gold = np.load(os.path.join(GOLDEN, "fd64_every_pixel.npz"))
    ms, ts = (int(v) for v in gold["seeds"])
    spec = W.fd_clip_optics(64)
    m = W.as_f32_exact(W.curvilinear_mask(64, ms))
    T = W.manhattan_mask(64, ts, n_rects=4, side_min=6, side_max=20)
    bank = L.Bank.from_spec(spec)
    assert bank.inner_grid == 64
    _, loss, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR,
                                 want_image=False)
    g = grad.cpu().numpy()[0].astype(np.float64)
    fd = gold["fd"]
    e_max = float(np.abs(g - fd).max() / np.abs(fd).max())
    e_l2 = rel_l2(g, fd)
    e_loss = abs(loss.item() - float(gold["loss"])) / float(gold["loss"])
    print(f"64x64 every pixel vs FD: max {e_max:.2e} (of max |fd|), rel L2 {e_l2:.2e}, loss {e_loss:.2e}")
    assert e_max < GTOL and e_l2 < GTOL and e_loss < ITOL


# ---------------------------------------------------------------- 4096 x 4096, three planes, K = 32

@pytest.fixture(scope="module")
def tile4096():
    gold = np.load(os.path.join(GOLDEN, "tile4096_gradient_window.npz"))
    y0, x0, h = (int(v) for v in gold["window"])
    spec = W.CONFIG5
    m = W.as_f32_exact(W.curvilinear_mask(4096, 4000))
    T = W.manhattan_target(4096, 4001)
    b = O.band_geometry(spec)[0]
    mh = O.mask_spectrum(m, b, "fft")
    refs = []
    for F in spec.focus_nm:
        lam, phi = O.socs_kernels(spec, F, K=32)
        refs.append(O.image_window(mh, lam, phi, 4096, y0, x0, h, h))
    return spec, m, T, gold, (y0, x0, h), refs


@pytest.mark.parametrize("inner", [3072, 4096])
def test_full_tile_4096_inner_grids(L, tile4096, inner):
    spec, m, T, gold, (y0, x0, h), refs = tile4096
    bank = L.Bank.from_spec(spec)
    bank.set_inner_grid(inner)
    assert bank.inner_grid == inner
    img, loss, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR)
    win = (slice(y0, y0 + h), slice(x0, x0 + h))
    img, g = img.cpu().numpy()[0], grad.cpu().numpy()[0]
    e_img = [rel_l2(img[p][win], refs[p]) for p in range(3)]
    e_grad = rel_l2(g[win], gold["grad"])
    e_loss = abs(loss.item() - float(gold["loss"])) / float(gold["loss"])
    print(f"4096 P=3 K=32 Q={inner}: image(window) {e_img} grad(window) {e_grad:.2e} loss {e_loss:.2e}")
    for p in range(3):
        assert e_img[p] < ITOL, (p, e_img[p])
    assert e_grad < GTOL and e_loss < ITOL
