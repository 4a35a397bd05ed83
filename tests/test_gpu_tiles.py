"""GPU parity of the halo tiling of layouts larger than one clip against the
oracle's tiled method (oracle.tiles): image relative L2 <= 1e-5, loss
relative <= 1e-5, gradient relative L2 <= 1e-4; at 6144 x 6144 (beyond the
largest clip) on windows of each tile and across the seams.
"""
import numpy as np
import pytest

import oracle as O
import oracle.tiles as OT
import workloads as W

pytestmark = pytest.mark.gpu

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


@pytest.mark.parametrize("H,Wd,n,halo,P", [(300, 200, 128, 16, 1), (384, 256, 128, 32, 3), (96, 80, 64, 8, 2),
                                           (1000, 700, 512, 64, 1)])
def test_tiled_image_and_gradient(L, H, Wd, n, halo, P):
    spec = W.fd_clip_optics(n).with_(K=8, focus_nm=(-30.0, 0.0, 30.0)[:P] if P != 2 else (0.0, 30.0))
    bank = L.Bank.from_spec(spec)
    banks = [O.socs_kernels(spec, F, K=8) for F in spec.focus_nm]
    lay = W.as_f32_exact(W.curvilinear_mask(max(H, Wd), 120 + H)[:H, :Wd])
    T = W.manhattan_mask(max(H, Wd), 121 + H, n_rects=max(1, H * Wd // 800), side_min=8, side_max=30)[:H, :Wd]
    img = L.image_tiled(bank, dev(lay), halo).cpu().numpy()
    img2, loss, grad = L.image_grad_tiled(bank, dev(lay), dev(T), halo, slope=SLOPE, threshold=THR)
    Lo, go, Io = OT.tiled_gradient(lay, T, banks, SLOPE, THR, n, halo)
    for p in range(P):
        assert rel_l2(img[p], Io[p]) < 1e-5, p
        assert rel_l2(img2.cpu().numpy()[p], Io[p]) < 1e-5, p
    e_loss = abs(loss.item() - Lo) / Lo
    e_grad = rel_l2(grad.cpu().numpy(), go)
    print(f"tiled {H}x{Wd} n={n} halo={halo} P={P}: loss {e_loss:.2e} grad {e_grad:.2e}")
    assert e_loss < 1e-5 and e_grad < 1e-4


def test_tiled_l1_and_plane_weights(L):
    spec = W.fd_clip_optics(128).with_(K=8, focus_nm=(0.0, 30.0))
    bank = L.Bank.from_spec(spec)
    lay = W.as_f32_exact(W.curvilinear_mask(256, 5)[:200, :256])
    T = W.manhattan_mask(256, 6, n_rects=60, side_min=8, side_max=30)[:200, :256]
    banks = [O.socs_kernels(spec, F, K=8) for F in spec.focus_nm]
    _, loss, grad = L.image_grad_tiled(bank, dev(lay), dev(T), 16, slope=SLOPE, threshold=THR,
                                       plane_weights=[0.5, 2.0], want_image=False)
    Lo, go, _ = OT.tiled_gradient(lay, T, banks, SLOPE, THR, 128, 16, weights=[0.5, 2.0])
    assert abs(loss.item() - Lo) < 1e-5 * Lo and rel_l2(grad.cpu().numpy(), go) < 1e-4
    with pytest.raises(L.LithoError):
        L.image_grad_tiled(bank, dev(lay), dev(T), 64)             # no core left
    with pytest.raises(L.LithoError):
        L.image_grad_tiled(bank, dev(lay), dev(T), 16, blur_sigma_px=2.0)


def test_layout_beyond_the_largest_clip(L):
    # 6144 x 6144 layout through 4096 x 4096 windows (halo 256, 2 x 2 tiles),
    # one plane, K = 8: windows of the image inside each core and across the seams
    n, halo, H = 4096, 256, 6144
    spec = W.CONFIG2.with_(n=n, K=8)
    bank = L.Bank.from_spec(spec)
    lay = W.as_f32_exact(W.curvilinear_mask(H, 6144))
    img = L.image_tiled(bank, dev(lay), halo).cpu().numpy()[0]
    lam, phi = O.socs_kernels(spec, 0.0, K=8)
    origins, c = OT.tile_origins(H, H, n, halo)
    assert len(origins) == 4
    b = bank.b
    for (y0, x0) in origins:
        mh = O.mask_spectrum(OT.window(lay, y0, x0, n), b, "fft")
        # a 64 x 64 window at the core's corner nearest the layout centre (the seam)
        wy = halo + (c - 64 if y0 < 0 else 0)
        wx = halo + (c - 64 if x0 < 0 else 0)
        ref = O.image_window(mh, lam, phi, n, wy, wx, 64, 64)
        got = img[y0 + wy:y0 + wy + 64, x0 + wx:x0 + wx + 64]
        assert rel_l2(got, ref) < 1e-5, (y0, x0)
