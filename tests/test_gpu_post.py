"""GPU parity of the steps after the image against the FP64 oracle (oracle.post).

* litho_contours: marching squares.  Segment count, cells, codes and
  successor indices bit-exact; crossing parameters within 1e-6.
* litho_epe: edge sites bit-exact; EPE within 1e-4 px + 1e-5 relative
  (float32 arithmetic against FP64 on the same float32 latent images).
* litho_lowpass: Gaussian low-pass within 1e-6 of the image range; the
  thresholded form bit-exact away from the threshold.
* litho_image_grad with a Gaussian resist kernel (Eq. 5) and the L2 or L1
  loss (Eqs. 15-17): resist image 1e-5, loss 1e-5, gradient 1e-4 (relative).
* litho_ai_channels (Eq. 9): layout exact, image and dI/dM within 1e-5.
* The fused resampling column pass (with the resist blur folded in) against
  the two-pass route of another inner grid at 1024^2 and 2048^2: the blurred
  ILT step's image and loss within 2e-6, its gradient within 1e-5.

Every input is seeded and synthetic (workloads) or computed by the oracle,
rounded to float32 and given to both sides.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.post as OP
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


def dev(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _banks(spec, K):
    return [O.socs_kernels(spec, F, K=K) for F in spec.focus_nm]


def _oracle_image_f32(n, seed, K=8):
    spec = W.fd_clip_optics(n).with_(K=K)
    lam, phi = O.socs_kernels(spec, 0.0, K=K)
    return O.image(W.curvilinear_mask(n, seed), lam, phi, method="fft").astype(np.float32)


# ---------------------------------------------------------------- contours

def _compare_contours(got, ref):
    S = len(ref["cell"])
    assert len(got["cell"]) == S
    assert np.array_equal(got["cell"].cpu().numpy(), ref["cell"])
    assert np.array_equal(got["code"].cpu().numpy(), ref["code"])
    assert np.array_equal(got["next"].cpu().numpy(), ref["next"])
    if S:
        assert np.abs(got["u"].cpu().numpy().astype(np.float64) - ref["u"]).max() < 1e-6


@pytest.mark.parametrize("n,seed,level", [(64, 1, 0.5), (96, 2, 0.5), (200, 3, 0.4), (256, 4, 0.6),
                                          (1024, 5, 0.5)])
def test_contours_of_masks(L, n, seed, level):
    v = W.curvilinear_mask(n, seed).astype(np.float32)
    ref = OP.contours(v, level)
    got = L.contours(dev(v), level)
    print(f"contours n={n}: {len(ref['cell'])} segments")
    _compare_contours(got, ref)


@pytest.mark.parametrize("n", [128, 384])
def test_contours_of_aerial_images(L, n):
    I = _oracle_image_f32(n, 40 + n)
    lvl = float(np.float32(np.median(I)))
    _compare_contours(L.contours(dev(I), lvl), OP.contours(I, lvl))


def test_contour_special_cases(L):
    # saddles resolved both ways, a lone bright pixel, level exactly on corner
    # values, an empty image, a constant image, the periodic wrap
    v = np.zeros((64, 64), np.float32)
    v[10, 10] = v[11, 11] = 1.0
    v[30, 40] = 1.0
    v[63, 0] = v[0, 63] = 0.7
    v[20:24, 50:64] = 0.5
    for lvl in (0.45, 0.5, 0.55, 0.7, 1.0):
        _compare_contours(L.contours(dev(v), lvl), OP.contours(v, lvl))
    for c in (0.0, 1.0):
        assert len(L.contours(dev(np.full((64, 64), c, np.float32)), 0.5)["cell"]) == 0


def test_contour_capacity_and_errors(L):
    import torch
    v = W.curvilinear_mask(128, 9).astype(np.float32)
    ref = OP.contours(v, 0.5)
    S = len(ref["cell"])
    got = L.contours(dev(v), 0.5, capacity=S // 3)     # too small: the binding retries with the count
    _compare_contours(got, ref)
    # a direct call with a short capacity writes the first segments and reports the total
    cap = S // 4
    bufs = [torch.full((cap,), -7, dtype=torch.int32, device="cuda") for _ in range(3)]
    u = torch.zeros((cap, 2), device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = L._lib.litho_contours(128, dev(v).data_ptr(), 0.5, cap, bufs[0].data_ptr(), bufs[1].data_ptr(),
                               u.data_ptr(), bufs[2].data_ptr(), cnt.data_ptr(), None)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(cnt.item()) == S
    assert np.array_equal(bufs[0].cpu().numpy(), ref["cell"][:cap])
    assert np.array_equal(bufs[2].cpu().numpy(), ref["next"][:cap])
    assert L._lib.litho_contours(1, dev(v).data_ptr(), 0.5, 0, None, None, None, None, cnt.data_ptr(), None) < 0
    assert L._lib.litho_contours(128, None, 0.5, 0, None, None, None, None, cnt.data_ptr(), None) < 0


# ---------------------------------------------------------------- EPE

@pytest.mark.parametrize("n,P", [(64, 1), (128, 3), (256, 3), (1024, 3)])
def test_epe_through_focus(L, n, P):
    spec = W.fd_clip_optics(n).with_(K=8)
    T = W.manhattan_target(n, 60 + n)
    m = W.curvilinear_mask(n, 61 + n)
    lats = np.stack([O.image(m, *O.socs_kernels(spec, F, K=8), method="fft")
                     for F in spec.focus_nm[:P]]).astype(np.float32)
    t_eff, f0, tn, tp = 0.3, min(1, P - 1), -0.4, 0.4
    sites = OP.epe_sites(T)
    ref = OP.epe_through_focus([x.astype(np.float64) for x in lats], sites, t_eff, f0, tn, tp)
    got = L.epe(dev(T), dev(lats), t_eff, f0=f0, tol_neg=tn, tol_pos=tp)
    S = len(sites)
    assert len(got["site"]) == S
    ys = np.array([s[0] for s in sites])
    xs = np.array([s[1] for s in sites])
    ds = np.array([s[2] for s in sites])
    assert np.array_equal(got["site"].cpu().numpy(), ys * n + xs)
    assert np.array_equal(got["dir"].cpu().numpy(), ds)
    e = got["epe"].cpu().numpy().astype(np.float64)
    assert e.shape == (S, P + 2)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(e), fin)
    assert np.array_equal(np.sign(e[~fin]), np.sign(ref[~fin]))
    # tolerance from float32 arithmetic: the mid-value and both derivative
    # components carry a few ulp of the latent values (max M), so
    # |dEPE| <~ 8 eps M (1 + |EPE|) / |grad E|, tight where the edge is steep
    # and loose only where the gradient vanishes (EPE large)
    eps = 2.0 ** -24
    M = np.abs(lats).max()
    gmag = np.zeros((S, P))
    for p in range(P):
        Ep = lats[p].astype(np.float64)
        at = lambda yy, xx: Ep[yy % n, xx % n]
        q = np.where(ds == 0, at(ys, xs + 1), at(ys + 1, xs))
        gt = np.where(ds == 0, 0.25 * ((at(ys + 1, xs) + at(ys + 1, xs + 1)) - (at(ys - 1, xs) + at(ys - 1, xs + 1))),
                      0.25 * ((at(ys, xs + 1) + at(ys + 1, xs + 1)) - (at(ys, xs - 1) + at(ys + 1, xs - 1))))
        gmag[:, p] = np.hypot(q - at(ys, xs), gt)
    gmin = np.concatenate([gmag, gmag.min(axis=1, keepdims=True), gmag.min(axis=1, keepdims=True)], axis=1)
    tol = 8 * eps * M * (1 + np.abs(ref)) / np.maximum(gmin, 1e-30) + 1e-6
    err = np.abs(e - ref)
    ratio = np.where(fin, err / tol, 0.0)
    steep = fin & (gmin > 0.01)
    print(f"EPE n={n} P={P}: {S} sites, max err/tol {ratio.max():.2f}, max |err| on steep edges "
          f"{err[steep].max():.2e} px")
    assert (ratio <= 1).all()


def test_epe_linear_latent_image(L):
    # a linear latent image: EPE is the signed distance of the iso-line (pinned closed form)
    n = 64
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    E = (0.05 * (xx - 30.2) + 0.01 * yy).astype(np.float32)
    T = np.zeros((n, n), np.float32)
    T[:, 10:33] = 1.0
    got = L.epe(dev(T), dev(E[None]), 0.3)
    site = got["site"].cpu().numpy()
    d = got["dir"].cpu().numpy()
    e = got["epe"].cpu().numpy()
    ys, xs = site // n, site % n
    keep = (d == 0) & (ys >= 2) & (ys <= n - 3)
    want = -(0.05 * (xs[keep] + 0.5 - 30.2) + 0.01 * ys[keep] - 0.3) / math.hypot(0.05, 0.01)
    assert keep.sum() == 2 * (n - 4)
    assert np.abs(e[keep, 0] - want).max() < 1e-4


def test_epe_errors(L):
    import torch
    T = dev(np.zeros((64, 64)))
    with pytest.raises(L.LithoError):
        L.epe(T, dev(np.zeros((2, 64, 64))), 0.3, f0=2)
    with pytest.raises(L.LithoError):
        L.epe(T, dev(np.zeros((1, 64, 64))), 0.3, tol_neg=0.1)
    got = L.epe(T, dev(np.zeros((1, 64, 64))), 0.3)
    assert len(got["site"]) == 0
    del torch


# ---------------------------------------------------------------- low-pass

@pytest.mark.parametrize("n,s", [(64, 2.0), (256, 3.0), (1024, 3.0), (1024, 40.0)])
def test_lowpass_matches_oracle(L, n, s):
    bank = L.Bank.from_spec(W.fd_clip_optics(n).with_(K=2))
    rng = np.random.default_rng(n)
    imgs = np.stack([W.manhattan_target(n, 70 + n), rng.uniform(0, 1, (n, n))]).astype(np.float32)
    got = L.lowpass(bank, dev(imgs), s).cpu().numpy()
    for i in range(2):
        ref = OP.gaussian_filter(imgs[i].astype(np.float64), s)
        err = np.abs(got[i] - ref).max() / (np.abs(imgs[i]).max())
        print(f"lowpass n={n} s={s} image {i}: max err {err:.2e}")
        assert err < 1e-6


@pytest.mark.parametrize("n,s,tau", [(128, 3.0, 0.5), (512, 2.0, 0.4)])
def test_round_target_matches_oracle(L, n, s, tau):
    bank = L.Bank.from_spec(W.fd_clip_optics(n).with_(K=2))
    Zt = W.manhattan_target(n, 80 + n).astype(np.float32)
    got = L.lowpass(bank, dev(Zt[None]), s, threshold=tau).cpu().numpy()[0]
    f = OP.gaussian_filter(Zt.astype(np.float64), s)
    ref = OP.round_target(Zt.astype(np.float64), s, tau)
    assert set(np.unique(got)) <= {0.0, 1.0}
    clear = np.abs(f - tau) > 1e-5           # pixels whose side of the threshold is not decided by rounding
    assert clear.mean() > 0.999
    assert np.array_equal(got[clear], ref[clear])


# ---------------------------------------------------------------- resist blur and L1 loss

@pytest.mark.parametrize("n,inner,s,loss", [(64, 0, 2.0, "l2"), (64, 0, 2.0, "l1"), (256, 0, 3.0, "l2"),
                                            (256, 256, 3.0, "l1"), (1024, 0, 3.0, "l2")])
def test_blurred_resist_loss_and_gradient(L, n, inner, s, loss):
    K = 24 if n == 1024 else 8
    spec = (W.CONFIG2 if n == 1024 else W.fd_clip_optics(n).with_(K=K))
    bank = L.Bank.from_spec(spec)
    bank.set_inner_grid(inner)
    m = W.as_f32_exact(W.curvilinear_mask(n, 90 + n))
    T = W.manhattan_target(n, 91 + n)
    img, lo, grad = L.image_grad(bank, dev(m[None]), target=dev(T[None]), slope=SLOPE, threshold=THR,
                                 blur_sigma_px=s, loss=loss)
    Lo, go, Rs = OP.blurred_gradient(m, T, _banks(spec, K), SLOPE, THR, s, loss=loss)
    e_img = max(rel_l2(img.cpu().numpy()[0, p], Rs[p]) for p in range(len(Rs)))
    e_loss = abs(lo.item() - Lo) / Lo
    e_grad = rel_l2(grad.cpu().numpy()[0], go)
    print(f"blur n={n} Q={bank.inner_grid} s={s} {loss}: resist image {e_img:.2e} loss {e_loss:.2e} "
          f"grad {e_grad:.2e}")
    assert e_img < 1e-5 and e_loss < 1e-5 and e_grad < 1e-4


def test_litho_consistency_loss(L):
    # Eqs. 15-17: Z_round from the target by the Gaussian low-pass and
    # tau_round, then the sigmoid-relaxed L1 print loss against it
    n, s, tau_round, tau_print = 256, 3.0, 0.5, 0.3
    spec = W.fd_clip_optics(n).with_(K=8, focus_nm=(0.0,))
    bank = L.Bank.from_spec(spec)
    Zt = W.manhattan_target(n, 95)
    f = OP.gaussian_filter(Zt, s)
    assert np.abs(f - tau_round).min() > 1e-5          # no pixel decided by rounding
    zr = L.lowpass(bank, dev(Zt[None]), s, threshold=tau_round)
    Zr = OP.round_target(Zt, s, tau_round)
    assert np.array_equal(zr.cpu().numpy()[0], Zr)
    m = W.as_f32_exact(W.curvilinear_mask(n, 96))
    _, lo, grad = L.image_grad(bank, dev(m[None]), target=zr, slope=SLOPE, threshold=tau_print, loss="l1")
    Lo, go, _ = OP.blurred_gradient(m, Zr, _banks(spec, 8), SLOPE, tau_print, 0.0, loss="l1")
    assert abs(lo.item() - Lo) < 1e-5 * Lo
    assert rel_l2(grad.cpu().numpy()[0], go) < 1e-4


@pytest.mark.parametrize("spec_name,fused_q,plain_q,nb", [("CONFIG2", 640, 768, 2), ("CONFIG3", 1280, 1536, 1)])
def test_fused_resampling_pass_against_the_two_pass_route(L, spec_name, fused_q, plain_q, nb):
    """The inner grids 640 (of 1024) and 1280 (of 2048) resample through one
    column pass per direction with the resist Gaussian folded in; 768 and
    1536 take two column passes and a band multiply.  Both resamplings are
    exact, so the blurred ILT step agrees across the two routes to FP32
    rounding, at full size."""
    spec = getattr(W, spec_name)
    if spec_name == "CONFIG3":
        spec = spec.with_(focus_nm=(0.0,))
    n = spec.n
    bank = L.Bank.from_spec(spec)
    m = np.stack([W.as_f32_exact(W.curvilinear_mask(n, 60 + i)) for i in range(nb)])
    T = np.stack([W.manhattan_target(n, 70 + i) for i in range(nb)]).astype(np.float32)
    out = {}
    for q in (fused_q, plain_q):
        bank.set_inner_grid(q)
        assert bank.inner_grid == q
        img, lo, g = L.image_grad(bank, dev(m), target=dev(T), slope=SLOPE, threshold=THR, blur_sigma_px=2.5)
        out[q] = (img.cpu().numpy(), lo.cpu().numpy().astype(np.float64), g.cpu().numpy())
    (i0, l0, g0), (i1, l1, g1) = out[fused_q], out[plain_q]
    e_img, e_loss, e_grad = rel_l2(i0, i1), float(np.max(np.abs(l0 - l1) / np.abs(l1))), rel_l2(g0, g1)
    print(f"resampling routes n={n} Q={fused_q} vs {plain_q}: resist image {e_img:.2e} loss {e_loss:.2e} "
          f"grad {e_grad:.2e}")
    assert e_img < 2e-6 and e_loss < 2e-6 and e_grad < 1e-5


# ---------------------------------------------------------------- Eq. 9 channels

@pytest.mark.parametrize("n,plane", [(64, 0), (256, 1), (1024, 0)])
def test_ai_channels(L, n, plane):
    K = 24 if n == 1024 else 6
    spec = (W.CONFIG2 if n == 1024 else W.fd_clip_optics(n).with_(K=K))
    bank = L.Bank.from_spec(spec)
    Zt = np.stack([W.manhattan_target(n, 100 + n + i) for i in range(2)])
    lam, phi = O.socs_kernels(spec, spec.focus_nm[plane], K=K)
    X = L.ai_channels(bank, dev(Zt), plane=plane).cpu().numpy()
    norm = (0.0, 1.0, 0.0, 0.5, -0.05, 0.05)
    Xn = L.ai_channels(bank, dev(Zt), plane=plane, norm=norm).cpu().numpy()
    for i in range(2):
        ref = OP.ai_channels(Zt[i], lam, phi)
        assert np.array_equal(X[i, ..., 0], ref[..., 0])
        e1 = rel_l2(X[i, ..., 1], ref[..., 1])
        e2 = rel_l2(X[i, ..., 2], ref[..., 2])
        print(f"channels n={n} plane={plane}: image {e1:.2e} dI/dM {e2:.2e}")
        assert e1 < 1e-5 and e2 < 1e-5
        refn = OP.ai_channels(Zt[i], lam, phi, norm=norm)
        assert np.abs(Xn[i] - refn).max() < 1e-5
