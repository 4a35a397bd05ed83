"""GPU parity of the loss and the ILT adjoint against the FP64 oracle.

Gates: loss relative error <= 1e-5; gradient relative L2 error <= 1e-4
against the oracle's analytic gradient, which the CPU tests pin to central
finite differences; and directly against central finite differences of the
oracle loss at sampled pixels.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

GTOL = 1e-4
SLOPE, THR = 50.0, 0.3


def rel_l2(a, b):
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


@pytest.fixture(scope="module")
def clip64():
    spec = W.fd_clip_optics(64)
    masks = np.stack([W.as_f32_exact(W.curvilinear_mask(64, 31 + s)) for s in range(2)])
    targets = np.stack([W.manhattan_mask(64, 41 + s, n_rects=4, side_min=6, side_max=20) for s in range(2)])
    return spec, masks, targets, _banks(spec, spec.K)


def test_fused_loss_and_gradient_64(L, clip64):
    spec, masks, targets, banks = clip64
    bank = L.Bank.from_spec(spec)
    img, loss, grad = L.image_grad(bank, dev(masks), target=dev(targets), slope=SLOPE, threshold=THR)
    img, loss, grad = img.cpu().numpy(), loss.cpu().numpy(), grad.cpu().numpy()
    for i in range(2):
        Lo, go, Io = O.gradient(masks[i], targets[i], banks, SLOPE, THR)
        assert abs(loss[i] - Lo) < 1e-5 * Lo, (loss[i], Lo)
        assert rel_l2(grad[i], go) < GTOL
        for p in range(3):
            assert rel_l2(img[i, p], Io[p]) < 1e-5


def test_gradient_against_central_differences_64(L, clip64):
    spec, masks, targets, banks = clip64
    bank = L.Bank.from_spec(spec)
    _, _, grad = L.image_grad(bank, dev(masks[:1]), target=dev(targets[:1]), slope=SLOPE, threshold=THR,
                              want_image=False)
    grad = grad.cpu().numpy()[0]
    rng = np.random.default_rng(3)
    pix = [tuple(int(v) for v in rng.integers(0, 64, 2)) for _ in range(10)]
    pix.append(tuple(int(v) for v in np.unravel_index(np.argmax(np.abs(grad)), grad.shape)))
    fd = O.fd_gradient(masks[0], targets[0], banks, SLOPE, THR, pix, h=1e-5)
    got = np.array([grad[p] for p in pix])
    assert np.abs(got - fd).max() < GTOL * np.abs(grad).max()


def test_vjp_mode_matches_oracle(L, clip64):
    spec, masks, _, banks = clip64
    bank = L.Bank.from_spec(spec)
    rng = np.random.default_rng(5)
    G = rng.standard_normal((2, 3, 64, 64)).astype(np.float32)
    assert bank.inner_grid == 64
    _, _, grad = L.image_grad(bank, dev(masks), grad_image=dev(G), want_image=False)
    grad = grad.cpu().numpy()
    for i in range(2):
        _, go, _ = O.gradient(masks[i], None, banks, SLOPE, THR, G_override=[G[i, p].astype(np.float64)
                                                                              for p in range(3)])
        assert rel_l2(grad[i], go) < GTOL


def test_autograd_functions(L, clip64):
    import torch
    spec, masks, targets, banks = clip64
    bank = L.Bank.from_spec(spec)
    m = dev(masks).requires_grad_(True)
    img = L.LithoImage.apply(m, bank, None)
    w = torch.linspace(-1, 1, img.numel(), device="cuda").view_as(img)
    (img * w).sum().backward()
    _, go, _ = O.gradient(masks[1], None, banks, SLOPE, THR,
                          G_override=[w[1, p].double().cpu().numpy() for p in range(3)])
    assert rel_l2(m.grad[1].cpu().numpy(), go) < GTOL
    m2 = dev(masks).requires_grad_(True)
    loss = L.LithoILTLoss.apply(m2, dev(targets), bank, None, SLOPE, THR)
    (loss * torch.tensor([1.0, 2.0], device="cuda", dtype=torch.float64)).sum().backward()
    _, g1, _ = O.gradient(masks[1], targets[1], banks, SLOPE, THR)
    assert rel_l2(m2.grad[1].cpu().numpy(), 2.0 * g1) < GTOL


def test_autograd_functions_precision_and_plane_weights(L, clip64):
    # the wrappers pass the precision mode and plane weights through to the
    # library: f16x3 keeps FP32-level agreement with the oracle
    import torch
    spec, masks, targets, banks = clip64
    bank = L.Bank.from_spec(spec)
    pw = [0.5, 1.0, 2.0]
    m = dev(masks).requires_grad_(True)
    loss = L.LithoILTLoss.apply(m, dev(targets), bank, None, SLOPE, THR, "f16x3", pw)
    loss.sum().backward()
    for i in range(2):
        Lo, go, _ = O.gradient(masks[i], targets[i], banks, SLOPE, THR, weights=pw)
        assert abs(loss[i].item() - Lo) < 1e-5 * Lo
        assert rel_l2(m.grad[i].cpu().numpy(), go) < GTOL
    m2 = dev(masks).requires_grad_(True)
    img = L.LithoImage.apply(m2, bank, None, "f16x3")
    w = torch.linspace(-1, 1, img.numel(), device="cuda").view_as(img)
    (img * w).sum().backward()
    _, go, _ = O.gradient(masks[0], None, banks, SLOPE, THR,
                          G_override=[w[0, p].double().cpu().numpy() for p in range(3)])
    assert rel_l2(m2.grad[0].cpu().numpy(), go) < GTOL


@pytest.mark.parametrize("n,inner", [(128, 0), (256, 0), (256, 256), (512, 0)])
def test_gradient_parity_mid_sizes(L, n, inner):
    spec = W.fd_clip_optics(n).with_(K=12)
    bank = L.Bank.from_spec(spec)
    bank.set_inner_grid(inner)
    m = W.as_f32_exact(W.curvilinear_mask(n, 7))
    T = W.manhattan_target(n, 8)
    _, loss, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR,
                                 want_image=False)
    Lo, go, _ = O.gradient(m, T, _banks(spec, 12), SLOPE, THR)
    assert abs(loss.item() - Lo) < 1e-5 * Lo
    assert rel_l2(grad.cpu().numpy()[0], go) < GTOL


@pytest.mark.parametrize("inner", [0, 1024])
def test_bench_launch_config_gradient(L, inner):
    # 1024 x 1024, K = 24, batch of 16: compare two clips of the batch in full
    spec = W.CONFIG2
    bank = L.Bank.from_spec(spec)
    bank.set_inner_grid(inner)
    masks = np.stack([W.as_f32_exact(W.curvilinear_mask(1024, 1000 + s)) for s in range(16)])
    targets = np.stack([W.manhattan_target(1024, 1100 + s) for s in range(16)])
    _, loss, grad = L.image_grad(bank, dev(masks), target=dev(targets), slope=SLOPE, threshold=THR,
                                 want_image=False)
    loss, grad = loss.cpu().numpy(), grad.cpu().numpy()
    banks = _banks(spec, 24)
    for i in (0, 9):
        Lo, go, _ = O.gradient(masks[i], targets[i], banks, SLOPE, THR, method="fft")
        assert abs(loss[i] - Lo) < 1e-5 * Lo
        assert rel_l2(grad[i], go) < GTOL
        # and on a 64 x 64 crop window
        assert rel_l2(grad[i][480:544, 480:544], go[480:544, 480:544]) < GTOL


def test_vjp_mode_resampled_grid(L):
    # the residual is low-passed to the intensity band on the inner grid
    spec = W.fd_clip_optics(256).with_(K=10)
    bank = L.Bank.from_spec(spec)
    assert bank.inner_grid == 160
    m = W.as_f32_exact(W.curvilinear_mask(256, 12))
    rng = np.random.default_rng(9)
    G = rng.standard_normal((1, 3, 256, 256)).astype(np.float32)
    _, _, grad = L.image_grad(bank, dev(m[None]), grad_image=dev(G), want_image=False)
    _, go, _ = O.gradient(m, None, _banks(spec, 10), SLOPE, THR,
                          G_override=[G[0, p].astype(np.float64) for p in range(3)])
    assert rel_l2(grad.cpu().numpy()[0], go) < GTOL


def test_plane_weighted_loss_and_gradient(L):
    # through-focus loss with unequal plane weights against the oracle
    spec = W.fd_clip_optics(128).with_(K=10)
    bank = L.Bank.from_spec(spec)
    m = W.as_f32_exact(W.curvilinear_mask(128, 41))
    T = W.manhattan_target(128, 42)
    wts = [0.5, 1.0, 2.0]
    _, loss, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR,
                                 want_image=False, plane_weights=wts)
    Lo, go, _ = O.gradient(m, T, _banks(spec, 10), SLOPE, THR, weights=wts)
    assert abs(loss.item() - Lo) < 1e-5 * Lo
    assert rel_l2(grad.cpu().numpy()[0], go) < GTOL
    with pytest.raises(ValueError):
        L.image_grad(bank, dev(m[None]), target=dev(T[None]), plane_weights=[1.0])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_workspace_chunking_matches_single_pass(L, prec, monkeypatch):
    # a workspace limit below one clip forces one clip per chunk: results must
    # equal the single-pass call bit for bit (per-clip work does not depend on
    # the chunking)
    import torch
    spec = W.fd_clip_optics(256).with_(K=8)
    bank = L.Bank.from_spec(spec)
    masks = np.stack([W.as_f32_exact(W.curvilinear_mask(256, 60 + s)) for s in range(5)])
    tgts = np.stack([W.manhattan_target(256, 70 + s) for s in range(5)])
    img1, loss1, grad1 = L.image_grad(bank, dev(masks), target=dev(tgts), slope=SLOPE, threshold=THR, prec=prec)
    monkeypatch.setenv("LITHO_WORKSPACE_MB", "1")
    img2, loss2, grad2 = L.image_grad(bank, dev(masks), target=dev(tgts), slope=SLOPE, threshold=THR, prec=prec)
    only = L.image(bank, dev(masks), prec=prec)
    assert torch.equal(img1, img2) and torch.equal(grad1, grad2) and torch.equal(loss1, loss2)
    assert torch.equal(only, img1)


@pytest.mark.parametrize("n,inner", [(96, 0), (96, 96), (192, 0), (320, 0), (384, 384), (640, 0)])
def test_clip_sides_with_factors_three_and_five(L, n, inner):
    # clip sides 3 * 2^j and 5 * 2^j, resampled (inner 0) and on the full grid
    spec = W.fd_clip_optics(n).with_(K=8)
    bank = L.Bank.from_spec(spec)
    bank.set_inner_grid(inner)
    assert bank.inner_grid != n or inner == n
    m = W.as_f32_exact(W.curvilinear_mask(n, 90 + n))
    T = W.manhattan_target(n, 91 + n)
    img, loss, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR)
    Lo, go, imgs = O.gradient(m, T, _banks(spec, 8), SLOPE, THR, method="fft")
    for p in range(3):
        assert rel_l2(img.cpu().numpy()[0, p], imgs[p]) < 1e-5, p
    assert abs(loss.item() - Lo) < 1e-5 * Lo
    assert rel_l2(grad.cpu().numpy()[0], go) < GTOL
