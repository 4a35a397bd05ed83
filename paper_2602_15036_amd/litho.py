"""Python binding of liblitho.so (argument marshalling only).

Every step of the imaging path runs in the HIP library; this module turns
torch CUDA tensors (device memory) and the current torch stream into the raw
pointers of the C ABI in include/litho.h and turns error codes into
exceptions.  There is no CPU fallback: importing this module fails when the
library is missing, and every call fails when it returns an error.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch  # imported first so the library binds to torch's HIP runtime

from . import _abi as A

_lib = A.load_library()


class LithoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{A.ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise LithoError(rc, f"{what}: {_lib.litho_last_error().decode()}")
    return rc


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_ptr(t: Optional[torch.Tensor], what: str, dtype=torch.float32):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _addr(t: Optional[torch.Tensor], what: str, dtype=torch.float32):
    p = _dev_ptr(t, what, dtype)
    return None if p is None else p.value


SOURCE_KINDS = {"annular": A.LITHO_SRC_ANNULAR, "dipole_x": A.LITHO_SRC_DIPOLE_X,
                "dipole_y": A.LITHO_SRC_DIPOLE_Y, "points": A.LITHO_SRC_POINTS}


class Bank:
    """A device-resident SOCS kernel bank (Eqs. 2-3), one plane per focus value."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        info = A.BankInfo()
        _check(_lib.litho_kernels_info(self._h, C.byref(info)), "litho_kernels_info")
        self.n, self.b, self.B, self.K = info.n, info.b, info.B, info.K
        self.n_focus, self.n_source = info.n_focus, info.n_source
        self.inner_grid, self.pupil_radius = info.inner_grid, info.pupil_radius
        self.device_bytes = info.device_bytes
        self.clear_field, self.degeneracy_gap = info.clear_field, info.degeneracy_gap

    @classmethod
    def build(cls, n: int, pixel_nm: float, na: float, source: str = "annular",
              sigma_in: float = 0.5, sigma_out: float = 0.8, wavelength_nm: float = 13.5,
              source_grid: int = 15, focus_nm: Sequence[float] = (0.0,), K: int = 8,
              dose: float = 1.0, points: Sequence[Sequence[float]] = ()) -> "Bank":
        """points: (sigma_x, sigma_y, weight) samples for source="points"."""
        focus = (C.c_double * len(focus_nm))(*[float(f) for f in focus_nm])
        flat = [float(v) for p in points for v in p]
        if len(flat) != 3 * len(points):
            raise ValueError("points must be (sigma_x, sigma_y, weight) triples")
        pts = (C.c_double * max(1, len(flat)))(*flat)
        o = A.Optics(n=n, pixel_nm=pixel_nm, wavelength_nm=wavelength_nm, na=na,
                     source_kind=SOURCE_KINDS[source], source_grid=source_grid,
                     sigma_in=sigma_in, sigma_out=sigma_out, n_focus=len(focus_nm),
                     focus_nm=C.cast(focus, C.POINTER(C.c_double)), K=K, dose=dose,
                     src_points=C.cast(pts, C.POINTER(C.c_double)) if points else None,
                     n_src_points=len(points))
        h = C.c_void_p()
        _check(_lib.litho_kernels_build(C.byref(o), C.byref(h)), "litho_kernels_build")
        return cls(h)

    @classmethod
    def from_spec(cls, spec, K: Optional[int] = None) -> "Bank":
        """Build from any object with the fields of an optics spec (n, pixel_nm, ...)."""
        return cls.build(n=spec.n, pixel_nm=spec.pixel_nm, na=spec.na, source=spec.source,
                         sigma_in=spec.sigma_in, sigma_out=spec.sigma_out,
                         wavelength_nm=spec.wavelength_nm, source_grid=spec.source_grid,
                         focus_nm=tuple(spec.focus_nm), K=spec.K if K is None else K,
                         points=tuple(getattr(spec, "points", ()) or ()))

    @classmethod
    def load(cls, n: int, lam: np.ndarray, phi: np.ndarray) -> "Bank":
        """Load eigenpairs: lam [P, K], phi [P, K, B, B] complex (centred band)."""
        lam = np.ascontiguousarray(np.atleast_2d(lam), dtype=np.float64)
        phi = np.asarray(phi)
        if phi.ndim == 3:
            phi = phi[None]
        P, K, B, _ = phi.shape
        ph = np.ascontiguousarray(np.stack([phi.real, phi.imag], axis=-1), dtype=np.float64)
        h = C.c_void_p()
        _check(_lib.litho_kernels_load(n, B, K, P, lam.ctypes.data_as(C.POINTER(C.c_double)),
                                       ph.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)),
               "litho_kernels_load")
        return cls(h)

    def set_inner_grid(self, q: int = 0) -> None:
        """Side of the per-kernel transform grid: 0 automatic, n full grid."""
        _check(_lib.litho_kernels_set_inner_grid(self.handle, int(q)), "litho_kernels_set_inner_grid")
        info = A.BankInfo()
        _check(_lib.litho_kernels_info(self._h, C.byref(info)), "litho_kernels_info")
        self.inner_grid = info.inner_grid

    def eigenvalues(self) -> np.ndarray:
        out = np.zeros((self.n_focus, self.K))
        _check(_lib.litho_kernels_eigenvalues(self._h, out.ctypes.data_as(C.POINTER(C.c_double))),
               "litho_kernels_eigenvalues")
        return out

    def phi(self, plane: int, k: int) -> np.ndarray:
        out = np.zeros((self.B, self.B, 2))
        _check(_lib.litho_kernels_phi(self._h, plane, k, out.ctypes.data_as(C.POINTER(C.c_double))),
               "litho_kernels_phi")
        return out[..., 0] + 1j * out[..., 1]

    @property
    def handle(self) -> C.c_void_p:
        if self._h is None:
            raise ValueError("bank has been freed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.litho_kernels_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _mask_batch(mask: torch.Tensor, n: int) -> torch.Tensor:
    if mask.dim() == 2:
        mask = mask[None]
    if mask.dim() != 3 or mask.shape[-1] != n or mask.shape[-2] != n:
        raise ValueError(f"mask must be [batch, {n}, {n}], got {tuple(mask.shape)}")
    return mask


def prec_code(prec) -> int:
    """LITHO_PREC_* code of a mode name ("fp32", "f16x3", "bf16x3", "f16", "bf16") or code."""
    if isinstance(prec, str):
        try:
            return A.PREC_NAMES[prec.lower()]
        except KeyError:
            raise ValueError(f"unknown precision mode {prec!r}") from None
    return int(prec)


def image(bank: Bank, mask: torch.Tensor, K_use: Optional[int] = None,
          out: Optional[torch.Tensor] = None, stream=None, prec="fp32") -> torch.Tensor:
    """SOCS aerial image (Eq. 4): [batch, n_focus, n, n] float32 on the mask's device."""
    mask = _mask_batch(mask, bank.n)
    batch = mask.shape[0]
    K_use = bank.K if K_use is None else int(K_use)
    if out is None:
        out = torch.empty((batch, bank.n_focus, bank.n, bank.n), device=mask.device, dtype=torch.float32)
    _check(_lib.litho_image(bank.handle, _dev_ptr(mask, "mask"), batch, K_use, _dev_ptr(out, "image"),
                            prec_code(prec), C.c_void_p(_stream_handle(stream))), "litho_image")
    return out


LOSS_KINDS = {"l2": A.LITHO_LOSS_L2, "l1": A.LITHO_LOSS_L1}


def image_grad(bank: Bank, mask: torch.Tensor, target: Optional[torch.Tensor] = None,
               slope: float = 50.0, threshold: float = 0.3, grad_image: Optional[torch.Tensor] = None,
               K_use: Optional[int] = None, want_image: bool = True, stream=None, prec="fp32",
               plane_weights: Optional[Sequence[float]] = None, blur_sigma_px: float = 0.0, loss: str = "l2"):
    """Image, loss and mask gradient (fused sigmoid loss) or a VJP with dL/dI.

    plane_weights: loss weight of each focus plane (fused mode; default 1 each).
    blur_sigma_px: Gaussian resist kernel (fused mode; the image output is then
    the blurred resist image).  loss: "l2" or "l1" (fused mode).
    Returns (image or None, loss [batch] float64 or None, grad [batch, n, n]).
    """
    mask = _mask_batch(mask, bank.n)
    batch = mask.shape[0]
    K_use = bank.K if K_use is None else int(K_use)
    dev = mask.device
    img = torch.empty((batch, bank.n_focus, bank.n, bank.n), device=dev, dtype=torch.float32) \
        if want_image else None
    grad = torch.empty((batch, bank.n, bank.n), device=dev, dtype=torch.float32)
    loss_kind = LOSS_KINDS[loss]
    loss = None
    resist = None
    if target is not None:
        target = _mask_batch(target, bank.n)
        loss = torch.empty((batch,), device=dev, dtype=torch.float64)
        pw = None
        if plane_weights is not None:
            if len(plane_weights) != bank.n_focus:
                raise ValueError(f"plane_weights needs {bank.n_focus} values")
            pw = (C.c_double * bank.n_focus)(*[float(v) for v in plane_weights])
        resist = A.Resist(slope=slope, threshold=threshold,
                          plane_weight=None if pw is None else C.cast(pw, C.POINTER(C.c_double)),
                          blur_sigma_px=float(blur_sigma_px), loss=loss_kind)
    if grad_image is not None and grad_image.shape != (batch, bank.n_focus, bank.n, bank.n):
        raise ValueError("grad_image must be [batch, n_focus, n, n]")
    _check(_lib.litho_image_grad(
        bank.handle, _dev_ptr(mask, "mask"), batch, K_use, _dev_ptr(target, "target"),
        C.byref(resist) if resist is not None else None, _dev_ptr(grad_image, "grad_image"),
        _dev_ptr(img, "image"), _dev_ptr(loss, "loss", torch.float64), _dev_ptr(grad, "grad"),
        prec_code(prec), C.c_void_p(_stream_handle(stream))), "litho_image_grad")
    return img, loss, grad


def lowpass(bank: Bank, images: torch.Tensor, sigma_px: float, threshold: Optional[float] = None,
            out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Gaussian low-pass of [count, n, n] images (K_resist of Eq. 5, G_sigma of
    Eq. 16); with a threshold the 0/1 image of filtered >= threshold."""
    images = _mask_batch(images, bank.n)
    if out is None:
        out = torch.empty_like(images)
    thr = float("nan") if threshold is None else float(threshold)
    _check(_lib.litho_lowpass(bank.handle, _dev_ptr(images, "images"), images.shape[0], float(sigma_px), thr,
                              _dev_ptr(out, "out"), C.c_void_p(_stream_handle(stream))), "litho_lowpass")
    return out


def _compaction(call, capacity, what, stream):
    """Runs a counting call, then the filling call with enough capacity."""
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    if capacity is None:
        _check(call(0, count), what)
        capacity = int(count.item())
    _check(call(capacity, count), what)
    total = int(count.item())
    if total > capacity:
        _check(call(total, count), what)
    return total


def contours(image: torch.Tensor, level: float, capacity: Optional[int] = None, stream=None) -> dict:
    """Marching-squares contour segments of one [n, n] image at `level`
    (litho_contours): dict of cell, code (start * 4 + end), u [S, 2], next."""
    if image.dim() != 2 or image.shape[0] != image.shape[1]:
        raise ValueError("image must be [n, n]")
    n = image.shape[0]
    bufs = {}

    def call(cap, count):
        for k, shape, dt in (("cell", (cap,), torch.int32), ("code", (cap,), torch.int32),
                             ("u", (cap, 2), torch.float32), ("next", (cap,), torch.int32)):
            if k not in bufs or bufs[k].shape[0] < cap:
                bufs[k] = torch.empty(shape, dtype=dt, device=image.device)
        return _lib.litho_contours(n, _dev_ptr(image, "image"), float(level), cap,
                                   _addr(bufs["cell"], "cell", torch.int32), _addr(bufs["code"], "code", torch.int32),
                                   _addr(bufs["u"], "u"), _addr(bufs["next"], "next", torch.int32),
                                   _addr(count, "count", torch.int32), C.c_void_p(_stream_handle(stream)))
    total = _compaction(call, capacity, "litho_contours", stream)
    return {k: v[:total] for k, v in bufs.items()}


def epe(target: torch.Tensor, latent: torch.Tensor, t_eff: float, f0: int = 0, tol_neg: float = 0.0,
        tol_pos: float = 0.0, capacity: Optional[int] = None, stream=None) -> dict:
    """Edge placement error through focus (litho_epe) at the edge sites of a
    binary target [n, n] for latent images [P, n, n]: dict of site (y * n + x),
    dir (0 along x, 1 along y) and epe [S, P + 2] (per plane, average, effective)."""
    n = target.shape[-1]
    if latent.dim() == 2:
        latent = latent[None]
    P = latent.shape[0]
    rule = A.EpeRule(t_eff=float(t_eff), tol_neg=float(tol_neg), tol_pos=float(tol_pos), f0=int(f0))
    bufs = {}

    def call(cap, count):
        for k, shape, dt in (("site", (cap,), torch.int32), ("dir", (cap,), torch.int32),
                             ("epe", (cap, P + 2), torch.float32)):
            if k not in bufs or bufs[k].shape[0] < cap:
                bufs[k] = torch.empty(shape, dtype=dt, device=target.device)
        return _lib.litho_epe(n, _dev_ptr(target, "target"), _dev_ptr(latent, "latent"), P, C.byref(rule), cap,
                              _addr(bufs["site"], "site", torch.int32), _addr(bufs["dir"], "dir", torch.int32),
                              _addr(bufs["epe"], "epe"), _addr(count, "count", torch.int32),
                              C.c_void_p(_stream_handle(stream)))
    total = _compaction(call, capacity, "litho_epe", stream)
    return {k: v[:total] for k, v in bufs.items()}


def ai_channels(bank: Bank, layout: torch.Tensor, K_use: Optional[int] = None, plane: int = 0,
                norm: Optional[Sequence[float]] = None, stream=None) -> torch.Tensor:
    """Eq. 9's input tensor [batch, n, n, 3] = (Z_t, image of Z_t, dI/dM),
    optionally mapped to [0, 1] by norm = (lo0, hi0, lo1, hi1, lo2, hi2)."""
    layout = _mask_batch(layout, bank.n)
    out = torch.empty((layout.shape[0], bank.n, bank.n, 3), device=layout.device, dtype=torch.float32)
    nm = None
    if norm is not None:
        if len(norm) != 6:
            raise ValueError("norm needs six values")
        nm = (C.c_double * 6)(*[float(v) for v in norm])
    _check(_lib.litho_ai_channels(bank.handle, _dev_ptr(layout, "layout"), layout.shape[0],
                                  bank.K if K_use is None else int(K_use), int(plane), nm, _dev_ptr(out, "out"),
                                  C.c_void_p(_stream_handle(stream))), "litho_ai_channels")
    return out


def image_tiled(bank: Bank, layout: torch.Tensor, halo: int, K_use: Optional[int] = None, prec="fp32",
                stream=None) -> torch.Tensor:
    """Image of an [H, W] layout larger than a clip through halo tiling
    (litho_image_tiled): [n_focus, H, W]."""
    if layout.dim() != 2:
        raise ValueError("layout must be [H, W]")
    H, W = layout.shape
    out = torch.empty((bank.n_focus, H, W), device=layout.device, dtype=torch.float32)
    _check(_lib.litho_image_tiled(bank.handle, _dev_ptr(layout, "layout"), H, W, int(halo),
                                  bank.K if K_use is None else int(K_use), _dev_ptr(out, "image"), prec_code(prec),
                                  C.c_void_p(_stream_handle(stream))), "litho_image_tiled")
    return out


def image_grad_tiled(bank: Bank, layout: torch.Tensor, target: torch.Tensor, halo: int, slope: float = 50.0,
                     threshold: float = 0.3, K_use: Optional[int] = None, prec="fp32",
                     plane_weights: Optional[Sequence[float]] = None, loss: str = "l2", blur_sigma_px: float = 0.0,
                     want_image: bool = True, stream=None):
    """Tiled image, loss and layout gradient (litho_image_grad_tiled):
    (image [n_focus, H, W] or None, loss [1] float64, grad [H, W])."""
    if layout.dim() != 2 or target.shape != layout.shape:
        raise ValueError("layout and target must be [H, W]")
    H, W = layout.shape
    dev = layout.device
    img = torch.empty((bank.n_focus, H, W), device=dev, dtype=torch.float32) if want_image else None
    grad = torch.empty((H, W), device=dev, dtype=torch.float32)
    lo = torch.empty((1,), device=dev, dtype=torch.float64)
    pw = None
    if plane_weights is not None:
        if len(plane_weights) != bank.n_focus:
            raise ValueError(f"plane_weights needs {bank.n_focus} values")
        pw = (C.c_double * bank.n_focus)(*[float(v) for v in plane_weights])
    resist = A.Resist(slope=slope, threshold=threshold,
                      plane_weight=None if pw is None else C.cast(pw, C.POINTER(C.c_double)),
                      blur_sigma_px=float(blur_sigma_px), loss=LOSS_KINDS[loss])
    _check(_lib.litho_image_grad_tiled(bank.handle, _dev_ptr(layout, "layout"), H, W, int(halo),
                                       bank.K if K_use is None else int(K_use), _dev_ptr(target, "target"),
                                       C.byref(resist), _dev_ptr(img, "image"), _dev_ptr(lo, "loss", torch.float64),
                                       _dev_ptr(grad, "grad"), prec_code(prec), C.c_void_p(_stream_handle(stream))),
           "litho_image_grad_tiled")
    return img, lo, grad


class LithoImage(torch.autograd.Function):
    """I = SOCS image of the mask; backward is the adjoint with dL/dI (E_k recomputed)."""

    @staticmethod
    def forward(ctx, mask, bank: Bank, K_use: Optional[int] = None, prec="fp32"):
        ctx.bank, ctx.K_use, ctx.prec = bank, K_use, prec
        ctx.save_for_backward(mask)
        return image(bank, mask.contiguous(), K_use, prec=prec)

    @staticmethod
    def backward(ctx, g_image):
        (mask,) = ctx.saved_tensors
        _, _, g = image_grad(ctx.bank, mask.contiguous(), grad_image=g_image.contiguous().float(),
                             K_use=ctx.K_use, want_image=False, prec=ctx.prec)
        return g.view_as(mask), None, None, None


class LithoILTLoss(torch.autograd.Function):
    """Per-clip ILT loss sum_planes sum_r (sigmoid(a (I - t)) - T)^2 with the fused adjoint.

    The forward call computes the loss and dL/dm together; backward scales the
    stored gradient by the incoming per-clip weights.
    """

    @staticmethod
    def forward(ctx, mask, target, bank: Bank, K_use: Optional[int] = None, slope: float = 50.0,
                threshold: float = 0.3, prec="fp32", plane_weights: Optional[Sequence[float]] = None):
        _, loss, grad = image_grad(bank, mask.contiguous(), target=target.contiguous(), slope=slope,
                                   threshold=threshold, K_use=K_use, want_image=False, prec=prec,
                                   plane_weights=plane_weights)
        ctx.save_for_backward(grad)
        ctx.mask_shape = mask.shape
        return loss

    @staticmethod
    def backward(ctx, g_loss):
        (grad,) = ctx.saved_tensors
        w = g_loss.to(torch.float32).view(-1, 1, 1)
        return (grad * w).view(ctx.mask_shape), None, None, None, None, None, None, None


def profile_enable(on: bool = True) -> None:
    _check(_lib.litho_profile_enable(1 if on else 0), "litho_profile_enable")


def profile_read() -> dict:
    """{kernel name: (launch count, total milliseconds)} since the last read."""
    buf = C.create_string_buffer(1 << 16)
    _check(_lib.litho_profile_read(buf, len(buf)), "litho_profile_read")
    out = {}
    for item in buf.value.decode().split(";"):
        if not item:
            continue
        name, rest = item.split("=")
        cnt, ms = rest.split(":")
        out[name] = (int(cnt), float(ms))
    return out


class Server:
    """Continuous-batching server over resident banks (litho_serve_*).

    Requests are host arrays; submit() copies them, poll() returns the results.
    """

    def __init__(self, banks: Sequence[Bank], hbm_budget: int = 16 << 30, max_slots: int = 8,
                 max_queue: int = 4096):
        self._banks = list(banks)
        arr = (C.c_void_p * len(banks))(*[b.handle.value for b in banks])
        cfg = A.ServeCfg(hbm_budget=int(hbm_budget), max_slots=int(max_slots), max_queue=int(max_queue))
        h = C.c_void_p()
        _check(_lib.litho_serve_create(arr, len(banks), C.byref(cfg), C.byref(h)), "litho_serve_create")
        self._h = h

    def submit(self, bank: int, mask: np.ndarray, K_use: Optional[int] = None, target: Optional[np.ndarray] = None,
               slope: float = 50.0, threshold: float = 0.3, prec="fp32") -> int:
        """Queue one clip; mode 1 (image + loss + gradient) when a target is given."""
        b = self._banks[bank]
        m = np.ascontiguousarray(mask, dtype=np.float32)
        if m.shape != (b.n, b.n):
            raise ValueError(f"mask must be [{b.n}, {b.n}]")
        t = None if target is None else np.ascontiguousarray(target, dtype=np.float32)
        req = A.Request(bank=bank, K_use=b.K if K_use is None else int(K_use), mode=0 if t is None else 1,
                        h_mask=m.ctypes.data_as(C.POINTER(C.c_float)),
                        h_target=None if t is None else t.ctypes.data_as(C.POINTER(C.c_float)),
                        slope=slope, threshold=threshold, prec=prec_code(prec))
        ticket = C.c_uint64()
        _check(_lib.litho_serve_submit(self._h, C.byref(req), C.byref(ticket)), "litho_serve_submit")
        return int(ticket.value)

    def submit_device(self, bank: int, mask: torch.Tensor, image: torch.Tensor, K_use: Optional[int] = None,
                      target: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None,
                      loss: Optional[torch.Tensor] = None, slope: float = 50.0, threshold: float = 0.3,
                      prec="fp32") -> int:
        """Queue one clip whose inputs and outputs live in device memory.

        mask [n, n] (and target [n, n]) must be complete on submit; the request
        writes image [n_focus, n, n] (and grad [n, n], loss [1] float64) in place.
        Keep every tensor alive and the inputs unchanged until poll() returns it.
        """
        b = self._banks[bank]
        n = b.n
        if mask.shape != (n, n) or image.shape != (b.n_focus, n, n):
            raise ValueError(f"mask must be [{n}, {n}] and image [{b.n_focus}, {n}, {n}]")
        mode = 0 if target is None else 1
        if mode == 1 and (target.shape != (n, n) or grad is None or grad.shape != (n, n)):
            raise ValueError("mode 1 needs target and grad of shape [n, n]")
        req = A.Request(bank=bank, K_use=b.K if K_use is None else int(K_use), mode=mode, h_mask=None, h_target=None,
                        slope=slope, threshold=threshold, prec=prec_code(prec),
                        d_mask=_addr(mask, "mask"), d_target=_addr(target, "target"),
                        d_image=_addr(image, "image"), d_grad=_addr(grad, "grad"),
                        d_loss=_addr(loss, "loss", torch.float64))
        ticket = C.c_uint64()
        _check(_lib.litho_serve_submit(self._h, C.byref(req), C.byref(ticket)), "litho_serve_submit")
        return int(ticket.value)

    def poll_info(self, ticket: int, timeout_us: int = -1):
        """For device-resident requests: None while pending, else the timing dict."""
        info = A.ResultInfo()
        rc = _lib.litho_serve_poll(self._h, C.c_uint64(ticket), None, None, C.byref(info), int(timeout_us))
        if rc == A.LITHO_PENDING:
            return None
        _check(rc, "litho_serve_poll")
        return {"t_submit_us": info.t_submit_us, "t_start_us": info.t_start_us, "t_done_us": info.t_done_us}

    def poll(self, ticket: int, n: int, n_focus: int, with_grad: bool, timeout_us: int = -1):
        """None while pending, else dict(image, grad, loss, t_submit_us, t_start_us, t_done_us)."""
        img = np.empty((n_focus, n, n), dtype=np.float32)
        grad = np.empty((n, n), dtype=np.float32) if with_grad else None
        info = A.ResultInfo()
        rc = _lib.litho_serve_poll(self._h, C.c_uint64(ticket), img.ctypes.data_as(C.POINTER(C.c_float)),
                                   None if grad is None else grad.ctypes.data_as(C.POINTER(C.c_float)),
                                   C.byref(info), int(timeout_us))
        if rc == A.LITHO_PENDING:
            return None
        _check(rc, "litho_serve_poll")
        return {"image": img, "grad": grad, "loss": info.loss if with_grad else None,
                "t_submit_us": info.t_submit_us, "t_start_us": info.t_start_us, "t_done_us": info.t_done_us}

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.litho_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
