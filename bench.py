"""Throughput of the SOCS aerial image + ILT adjoint on one MI355X.

One step = one pass of the whole hot path over a batch of synthetic clips:
mask spectrum, per-kernel column/row transforms, |E_k|^2 accumulation,
sigmoid resist, L2 loss against a target, and the adjoint (mask gradient).
The headline batch is 16 curvilinear 1024 x 1024 clips at 2 nm (NA 0.55,
x-dipole 0.3-0.9, K = 24 SOCS kernels, FP32), resident in HBM before timing.

Prints one JSON line.  The metric counts clips x planes x N^2 x K
pixel-kernels per second; forward and adjoint work is counted once.  `value`
comes from a loop with kernel tracing off; per-kernel durations (HIP events
on the launch stream) come from a separate traced loop.  Further legs: the
split-precision modes, the 2048^2 three-plane ILT step and the 4096^2
three-plane tile (FP32 and split modes), the served stream (host and
device-resident I/O, FP32 and split precision), the FP64 oracle on the host
cores and a plain FP32 scipy.fft implementation on the host (a baseline only).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "aerial-image Mpixel·kernel/s (fwd+adjoint) vs plain FP32; p50/p99 clip latency"
UNIT = "Mpixel·kernel/s"
HBM_PEAK_GBS = 8000.0
# FP32 FMA issued one lane per cycle (no packed FP32): 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_NONPACKED_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
# VALU instruction issue: one wave64 instruction per SIMD every 4 cycles, i.e. one per CU per cycle
VALU_ISSUE_PER_S = 256 * 2.4e9
SETTLE_S = 0.3          # untimed steady-state lead-in of each ILT leg, seconds
SPLIT_MODES = ("f16x3", "bf16x3", "f16", "bf16")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mp-steps", type=int, default=10, help="timed steps per split-precision mode (0: skip)")
    ap.add_argument("--cpu-clips", type=int, default=10, help="clips in the oracle sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one device copy of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests in the served stream (0: skip)")
    ap.add_argument("--large-steps", type=int, default=20,
                    help="timed steps of the 2048^2 and 4096^2 three-plane legs (0: skip)")
    ap.add_argument("--only", default="", help="comma list of legs: headline,mp,large,serve,cpu")
    return ap.parse_args()


# ------------------------------------------------------------------ models

def band_of(spec):
    R = spec.na * spec.n * spec.pixel_nm / spec.wavelength_nm
    b = int(math.floor((1.0 + spec.sigma_out) * R))
    return b


def adj_chunks(nt, batch, K):
    """k-chunks of the FP32 adjoint column pass: the library takes enough of
    them for about 2048 (band tile x clip x chunk) units."""
    units = nt * batch
    want = (2048 + units - 1) // units
    kc = max(1, min(K, want))
    kper = (K + kc - 1) // kc
    return (K + kper - 1) // kper


def launch_bytes(name, g, c):
    """Algorithmic HBM bytes of one launch of pass `name` over c clips of one
    focus plane: every array the pass must read or write, once (complex64 =
    8 B, FP32 = 4 B, FP64 complex = 16 B).  N grid side, Q inner grid, B band
    side, D intensity band side (4b + 1), K kernels, KC adjoint k-chunks."""
    N, Q, B, D, K, KC, P = g["N"], g["Q"], g["B"], g["D"], g["K"], g["KC"], g["P"]
    resample = Q != N
    if name == "mask_rows":
        return c * (4 * N * N + 8 * N * B)
    if name == "mask_cols":
        return c * (8 * N * B + 8 * B * B)
    if name.startswith("pass_y_fwd"):
        return K * 8 * B * B + c * (8 * B * B + K * 8 * Q * B)
    if name == "pass_x_fwd":
        return c * (K * 8 * Q * B + (8 * Q * D if resample else 12 * N * N))
    if name in ("up_cols", "down_cols"):  # both resampling column transforms in one pass
        return c * 8 * D * (Q + N)
    if name == "up_cols_q":
        return c * 8 * D * (Q + D)
    if name == "up_cols_n":
        return c * 8 * D * (D + N)
    if name == "up_rows":
        return c * (8 * N * D + 12 * N * N)
    if name == "image_residual_rows":       # image band in, image out, target in, residual band out
        return c * (16 * N * D + 8 * N * N)
    if name == "down_rows":
        return c * (4 * N * N + 8 * N * D)
    if name == "down_cols_n":
        return c * 8 * D * (N + D)
    if name == "down_cols_q":
        return c * 8 * D * (D + Q)
    if name == "pass_x_adj":
        return c * (K * 16 * Q * B + (8 * Q * D if resample else 4 * N * N))
    if name.startswith("pass_y_adj"):
        return K * 8 * B * B + c * (K * 8 * Q * B + KC * 16 * B * B)
    if name == "grad_cols":
        return c * (P * KC * 16 * B * B + 8 * N * B)
    if name == "grad_rows":
        return c * (8 * N * B + 4 * N * N)
    if name == "loss_reduce":
        return 0
    return None


def launch_flops(name, g, c):
    """Nominal FFT flops (5 L log2 L per complex transform of length L, no
    credit for band pruning) of the four per-kernel passes, per launch."""
    Q, B, K = g["Q"], g["B"], g["K"]
    fft = 5.0 * Q * math.log2(Q)
    if name == "pass_x_fwd":
        return c * K * Q * (fft + 3 * Q)
    if name == "pass_x_adj":
        return c * K * Q * (2 * fft + 2 * Q)
    if name == "pass_y_fwd":
        return c * K * B * (fft + 6 * Q)
    if name == "pass_y_adj":
        return c * K * B * (fft + 8 * Q)
    return None


def read_summary(fname):
    """key=value pairs of a committed profile summary, or {} when absent or
    when the kernel sources differ from the ones it was measured on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if line.startswith("#"):
            continue
        for tok in line.split():
            if "=" in tok:
                k, v = tok.split("=", 1)
                vals[k] = v
    csrc = os.path.join(ROOT, "paper_2602_15036_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, n), "rb").read() for n in ("kernels.hip", "fft.hpp"))
    if hashlib.sha256(src).hexdigest()[:16] != vals.get("kernel_source_sha256_16"):
        return {}
    return vals


def measured_traffic(kernel):
    v = read_summary("hbm_traffic_ilt_step_1024x16_K24.txt").get(f"{kernel}.hbm_bytes_calibrated")
    return float(v) if v is not None else None


def measured_valu(kernel):
    """(VALU wave-instructions, LDS wave-instructions, MFMA busy cycles) per launch from
    the committed counter summary, or None."""
    s = read_summary("counters_ilt_step_1024x16_K24.txt")
    if f"{kernel}.SQ_INSTS_VALU" not in s:
        return None
    return {k.split(".", 1)[1]: float(v) for k, v in s.items() if k.startswith(kernel + ".")}


# ------------------------------------------------------------------ the ILT step

class IltLeg:
    """Resident inputs and outputs of one ILT-step workload, and its step."""

    def __init__(self, L, torch, spec, masks, targets):
        import numpy as np
        self.L, self.torch, self.spec = L, torch, spec
        self.bank = L.Bank.from_spec(spec)
        self.batch = masks.shape[0]
        self.d_mask = torch.from_numpy(masks.astype(np.float32)).cuda()
        self.d_target = torch.from_numpy(targets.astype(np.float32)).cuda()
        n, P = spec.n, len(spec.focus_nm)
        self.n, self.K, self.P = n, spec.K, P
        self.img = torch.empty((self.batch, P, n, n), device="cuda")
        self.grad = torch.empty((self.batch, n, n), device="cuda")
        self.loss = torch.empty((self.batch,), device="cuda", dtype=torch.float64)
        self.pk = self.batch * P * n * n * spec.K
        b = self.bank.b
        nt = (self.bank.B + 3) // 4
        self.geo = {"N": n, "Q": self.bank.inner_grid, "B": self.bank.B, "D": 4 * b + 1, "K": spec.K,
                    "KC": adj_chunks(nt, self.batch, spec.K), "P": P}

    def step(self, prec="fp32", g=None):
        L = self.L
        L._check(L._lib.litho_image_grad(
            self.bank.handle, L._dev_ptr(self.d_mask, "mask"), self.batch, self.K,
            L._dev_ptr(self.d_target, "target"), L.C.byref(L.A.Resist(slope=50.0, threshold=0.3)), None,
            L._dev_ptr(self.img, "image"), L._dev_ptr(self.loss, "loss", self.torch.float64),
            L._dev_ptr(self.grad if g is None else g, "grad"), L.prec_code(prec),
            L.C.c_void_p(L._stream_handle())), "litho_image_grad")

    def forward(self, prec="fp32"):
        self.L.image(self.bank, self.d_mask, out=self.img, prec=prec)

    def timed(self, fn, steps):
        torch = self.torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def settle(self, fn, seconds=SETTLE_S):
        """Untimed steps until `seconds` of wall time have passed: the device
        raises its clocks over the first ~0.1-0.2 s under load, and the timed
        and traced loops should see the steady state.  Returns the step count."""
        torch = self.torch
        t0, n = time.perf_counter(), 0
        while True:
            fn()
            n += 1
            if n % 4 == 0:
                torch.cuda.synchronize()
                if time.perf_counter() - t0 >= seconds:
                    return n

    def traced(self, fn, steps):
        """Per-kernel (launches per step, average ms) from HIP events on the launch stream."""
        L = self.L
        L.profile_read()
        L.profile_enable(True)
        for _ in range(steps):
            fn()
        self.torch.cuda.synchronize()
        L.profile_enable(False)
        return {k: (c / steps, t / max(c, 1)) for k, (c, t) in L.profile_read().items()}

    def kernels_and_roofline(self, prof, step_s, traffic_lookup=None):
        kern, step_bytes = {}, 0.0
        for name, (per_step, avg_ms) in prof.items():
            base = name.split("<")[0]
            rec = {"launches_per_step": per_step, "avg_ms": avg_ms, "share": per_step * avg_ms / (step_s * 1e3)}
            by = launch_bytes(base, self.geo, self.batch)
            if by is not None:
                rec["algorithmic_bytes"] = by
                rec["GBps"] = by / (avg_ms * 1e-3) / 1e9
                rec["hbm_frac"] = rec["GBps"] / HBM_PEAK_GBS
                step_bytes += by * per_step
            fl = launch_flops(base, self.geo, self.batch)
            if fl is not None:
                rec["nominal_TFLOPs"] = fl / (avg_ms * 1e-3) / 1e12
            kern[name] = rec
        dom = max(kern, key=lambda k: kern[k]["share"])
        d = kern[dom]
        traffic = traffic_lookup(dom) if traffic_lookup else None
        roof = {"kernel": dom, "bound": "hbm", "achieved": d["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["GBps"] / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                "algorithmic_bytes_per_launch": d["algorithmic_bytes"], "avg_launch_ms": d["avg_ms"],
                "whole_step": {"algorithmic_bytes": step_bytes, "GBps": step_bytes / step_s / 1e9,
                               "frac": step_bytes / step_s / 1e9 / HBM_PEAK_GBS}}
        fl = launch_flops(dom, self.geo, self.batch)
        alu = {"nominal_fft_TFLOPs": fl / (d["avg_ms"] * 1e-3) / 1e12 if fl else None,
               "nonpacked_fp32_peak_TFLOPs": FP32_NONPACKED_TFLOPS}
        if fl:
            alu["nominal_frac_of_nonpacked"] = alu["nominal_fft_TFLOPs"] / FP32_NONPACKED_TFLOPS
        cnt = measured_valu(dom) if traffic_lookup else None
        if cnt:
            t = d["avg_ms"] * 1e-3
            alu["valu_issue_frac"] = cnt["SQ_INSTS_VALU"] / (t * VALU_ISSUE_PER_S)
            alu["counters"] = cnt
        roof["alu_view"] = alu
        return kern, roof


def ilt_leg(L, torch, leg, steps, warmup, modes, traffic_lookup=None):
    for _ in range(warmup):
        leg.step()
    settled = leg.settle(leg.step)
    dt = leg.timed(leg.step, steps)
    prof = leg.traced(leg.step, max(2, steps // 2))
    kern, roof = leg.kernels_and_roofline(prof, dt, traffic_lookup)
    for _ in range(2):
        leg.forward()
    dtf = leg.timed(leg.forward, steps)
    out = {"value": leg.pk / dt / 1e6, "unit": UNIT, "ms_per_step": dt * 1e3,
           "forward_only": {"value": leg.pk / dtf / 1e6, "ms": dtf * 1e3},
           "settle": {"seconds": SETTLE_S, "untimed_steps": settled},
           "kernels": kern, "roofline": roof}
    if modes:
        out["split_precision"] = split_modes(torch, leg, steps, out["value"], out["forward_only"]["value"], modes)
    return out


def split_modes(torch, leg, steps, fp32_value, fp32_fwd_value, modes):
    """Each split-precision mode on the same inputs: throughput, speed-up over
    FP32 and relative L2 error of image and gradient against the FP32 path (the
    FP32 path itself is held to 1e-5 of the FP64 oracle by the tests)."""
    leg.step()
    torch.cuda.synchronize()
    img32, grad32 = leg.img.clone(), leg.grad.clone()
    g2 = torch.empty_like(leg.grad)
    res = {}
    nrm = lambda a, b: float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))
    for name in modes:
        leg.step(name, g2)
        torch.cuda.synchronize()
        e_img, e_grad = nrm(leg.img, img32), nrm(g2, grad32)
        dt = leg.timed(lambda: leg.step(name, g2), steps)
        prof = leg.traced(lambda: leg.step(name, g2), 2)
        dtf = leg.timed(lambda: leg.forward(name), steps)
        res[name] = {"value": leg.pk / dt / 1e6, "ms_per_step": dt * 1e3, "speedup_vs_fp32": leg.pk / dt / 1e6 / fp32_value,
                     "forward_value": leg.pk / dtf / 1e6,
                     "forward_speedup_vs_fp32": leg.pk / dtf / 1e6 / fp32_fwd_value,
                     "rel_l2_image_vs_fp32": e_img, "rel_l2_grad_vs_fp32": e_grad,
                     "kernels_avg_ms": {k: round(v[1], 5) for k, v in prof.items()}}
    return res


# ------------------------------------------------------------------ CPU baselines

def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count()


def cpu_oracle(spec, masks, targets, planes, K, label):
    """The FP64 oracle (direct DFT, numpy/BLAS on the host cores) as it stands,
    on a bounded sample: the given clips, the first `planes` focus planes and
    the first K kernels of each."""
    import oracle as O
    banks = [O.socs_kernels(spec, F, K=K) for F in spec.focus_nm[:planes]]
    t0 = time.perf_counter()
    for m, T in zip(masks, targets):
        O.gradient(m, T, banks, 50.0, 0.3, method="direct")
    dt = time.perf_counter() - t0
    pk = len(masks) * planes * spec.n * spec.n * K
    bt = blas_threads()
    return {"value": pk / dt / 1e6, "unit": UNIT, "cores": int(bt), "kind": "oracle",
            "host_cpus": os.cpu_count(), "blas_threads": int(bt), "seconds": dt,
            "sample": f"{label}: {len(masks)} clip(s) {spec.n}x{spec.n}, {planes} of {len(spec.focus_nm)} "
                      f"plane(s), K={K} of {spec.K}, forward+adjoint, FP64 direct-DFT oracle, {dt:.1f} s"}


def cpu_scipy_fp32(spec, masks, targets, label):
    """A plain FP32 SOCS image + sigmoid-L2 adjoint with scipy.fft on all host
    cores (kernels from the oracle's eigendecomposition, rounded to complex64).
    A baseline only: it is neither the oracle nor the product."""
    import numpy as np
    import scipy.fft as sf

    import oracle as O
    workers = os.cpu_count()
    n, K = spec.n, spec.K
    lam, phi = O.socs_kernels(spec, spec.focus_nm[0], K=K)
    b = (phi.shape[-1] - 1) // 2
    idx = np.r_[0:b + 1, n - b:n]
    band = np.ix_(idx, idx)
    order = np.r_[b:2 * b + 1, 0:b]                     # centred band -> FFT order
    kern = np.zeros((K, 2 * b + 1, 2 * b + 1), np.complex64)
    for k in range(K):
        kern[k] = (np.sqrt(lam[k]) * phi[k])[np.ix_(order, order)]
    t0 = time.perf_counter()
    for m, T in zip(masks, targets):
        m = m.astype(np.float32)
        T = T.astype(np.float32)
        Mh = sf.fft2(m, workers=workers)[band]
        full = np.zeros((n, n), np.complex64)
        E = np.empty((K, n, n), np.complex64)
        I = np.zeros((n, n), np.float32)
        for k in range(K):
            full[band] = kern[k] * Mh
            E[k] = sf.ifft2(full, workers=workers)
            I += (E[k].real ** 2 + E[k].imag ** 2)
        Z = 1.0 / (1.0 + np.exp(-50.0 * (I - 0.3)))
        G = (2.0 * (Z - T) * 50.0 * Z * (1.0 - Z)).astype(np.float32)
        acc = np.zeros_like(Mh)
        for k in range(K):
            acc += np.conj(kern[k]) * sf.fft2(G * E[k], workers=workers)[band]
        full[:] = 0
        full[band] = acc
        sf.ifft2(full, workers=workers).real * 2.0
    dt = time.perf_counter() - t0
    pk = len(masks) * spec.n * spec.n * K
    return {"value": pk / dt / 1e6, "unit": UNIT, "cores": workers, "kind": "scipy.fft FP32, baseline only",
            "seconds": dt, "sample": f"{label}: {len(masks)} clip(s) {n}x{n}, K={K}, forward+adjoint, {dt:.1f} s"}


# ------------------------------------------------------------------ served stream

def served_stream(L, n_requests, rho=0.8, seed=3000, device=False, prec="fp32", pool_per=8):
    """Served stream: clip sides log-uniform over {256, 512, 1024, 2048},
    Manhattan/curvilinear 50/50, forward or forward+gradient 50/50, K uniform in
    16..32 from resident K_max = 32 banks.  A closed-loop burst measures the
    saturated request rate; then Poisson arrivals at rho times that rate give
    the p50/p99 latency (submit -> device work done).  device=False: host
    arrays in and out (copies included); device=True: inputs resident in HBM
    and results written to device buffers (no host copies).  Masks come from a
    pool of `pool_per` seeded clips per side and kind."""
    import threading

    import numpy as np

    import workloads as W
    sizes = (256, 512, 1024, 2048)
    banks = [L.Bank.from_spec(W.serve_optics(n)) for n in sizes]
    pool = {}
    for bi, n in enumerate(sizes):
        for kind in ("manhattan", "curvilinear"):
            for j in range(pool_per):
                spec = W.ServeRequestSpec(n=n, kind=kind, mode=0, K_use=16, arrival_s=0.0,
                                          seed=seed + 97 * bi + j)
                pool[(bi, kind, j)] = W.as_f32_exact(W.request_mask(spec)).astype(np.float32)
        pool[(bi, "target")] = W.manhattan_target(n, seed + 7 + bi).astype(np.float32)
    reqs = W.served_stream(n_requests, seed, rate_hz=0.0, sizes=sizes)
    srv = L.Server(banks, hbm_budget=16 << 30, max_slots=8, max_queue=n_requests + 8)
    if device:
        import torch
        dpool = {k: torch.from_numpy(v).cuda() for k, v in pool.items()}
        outs = []
        for r in reqs:
            o = {"image": torch.empty((1, r.n, r.n), device="cuda")}
            if r.mode:
                o["grad"] = torch.empty((r.n, r.n), device="cuda")
                o["loss"] = torch.empty((1,), device="cuda", dtype=torch.float64)
            outs.append(o)
        torch.cuda.synchronize()

    def submit(i, r):
        bi = sizes.index(r.n)
        j = i % pool_per
        if not device:
            return srv.submit(bi, pool[(bi, r.kind, j)], K_use=r.K_use,
                              target=pool[(bi, "target")] if r.mode else None, prec=prec)
        o = outs[i]
        return srv.submit_device(bi, dpool[(bi, r.kind, j)], o["image"], K_use=r.K_use,
                                 target=dpool[(bi, "target")] if r.mode else None, grad=o.get("grad"),
                                 loss=o.get("loss"), prec=prec)

    tickets_ref = [None]

    def collect(i, r):
        if device:
            return srv.poll_info(tickets_ref[0][i])
        return srv.poll(tickets_ref[0][i], r.n, 1, bool(r.mode))

    def run(arrivals):
        t0 = time.perf_counter()
        tickets = [None] * len(reqs)
        tickets_ref[0] = tickets

        def producer():
            for i, r in enumerate(reqs):
                if arrivals is not None:
                    dt = arrivals[i] - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                tickets[i] = submit(i, r)
        th = threading.Thread(target=producer)
        th.start()
        lat, pk = [], 0.0
        for i, r in enumerate(reqs):
            while tickets[i] is None:
                time.sleep(1e-4)
            res = collect(i, r)
            lat.append((res["t_done_us"] - res["t_submit_us"]) * 1e-3)
            pk += r.n * r.n * r.K_use
        th.join()
        return time.perf_counter() - t0, np.array(lat), pk

    run(None)                                   # warm banks, workspaces, slot buffers
    wall, _, pk = run(None)                     # closed loop: saturated rate
    mu = len(reqs) / wall
    rng = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / (rho * mu), size=len(reqs)))
    wall2, lat, pk2 = run(list(arrivals))
    srv.close()
    for b in banks:
        b.close()
    return {"requests": len(reqs), "sizes": list(sizes), "K_range": [16, 32], "grad_fraction": 0.5,
            "mask_pool": f"{pool_per} seeded clips per side and kind",
            "saturated_req_per_s": mu, "saturated_Mpk_per_s": pk / wall / 1e6,
            "offered_load": rho, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "open_loop_Mpk_per_s": pk2 / wall2 / 1e6, "precision": prec,
            "io": "device-resident" if device else "host arrays (PCIe copies included)"}


# ------------------------------------------------------------------ main

def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 (no multi-GPU path is built)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    legs = set(args.only.split(",")) if args.only else {"headline", "mp", "large", "serve", "cpu"}
    import numpy as np
    import torch

    import workloads as W
    from paper_2602_15036_amd import litho as L

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration << 18                  # float32 elements
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return

    spec = W.CONFIG2
    batch = args.batch
    masks = np.stack([W.as_f32_exact(W.curvilinear_mask(spec.n, 1000 + i)) for i in range(batch)])
    targets = np.stack([W.manhattan_target(spec.n, 1100 + i) for i in range(batch)])
    leg = IltLeg(L, torch, spec, masks, targets)
    head = ilt_leg(L, torch, leg, args.steps, args.warmup,
                   SPLIT_MODES if ("mp" in legs and args.mp_steps > 0) else (),
                   traffic_lookup=measured_traffic)
    print(json.dumps({"kernels": head["kernels"]}), file=sys.stderr, flush=True)
    n, K, P = spec.n, spec.K, len(spec.focus_nm)
    out = {
        "metric": METRIC, "value": head["value"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ILT step (image + sigmoid resist + L2 loss + mask gradient), {batch} curvilinear "
                               f"clips {n}x{n} at 2 nm, NA 0.55 x-dipole 0.3-0.9, K={K}, 1 focus plane, FP32",
                   "clips": batch, "n": n, "K": K, "planes": P, "inner_grid": leg.bank.inner_grid,
                   "band": leg.bank.B},
        "forward_only": head["forward_only"],
        "settle": head["settle"],
        "roofline": head["roofline"],
    }
    if "split_precision" in head:
        out["mixed_precision"] = head["split_precision"]
    fp32_value = head["value"]
    del leg
    torch.cuda.empty_cache()

    if "large" in legs and args.large_steps > 0:
        large = {}
        for name, sp, seeds in (("ilt_2048x2048_3planes_K24", W.CONFIG3, (2000, 2001)),
                                ("tile_4096x4096_3planes_K32", W.CONFIG5, (4000, 4001))):
            m = W.as_f32_exact(W.curvilinear_mask(sp.n, seeds[0]))[None]
            t = W.manhattan_target(sp.n, seeds[1])[None]
            lg = IltLeg(L, torch, sp, m, t)
            r = ilt_leg(L, torch, lg, args.large_steps, 2, SPLIT_MODES if args.mp_steps > 0 else ())
            r["config"] = {"clips": 1, "n": sp.n, "K": sp.K, "planes": 3, "focus_nm": list(sp.focus_nm),
                           "inner_grid": lg.bank.inner_grid, "band": lg.bank.B}
            large[name] = r
            del lg
            torch.cuda.empty_cache()
            print(f"[bench] {name}: {r['value']:.4g} {UNIT}", file=sys.stderr, flush=True)
        out["large_tiles"] = large

    if "serve" in legs and args.serve_requests > 0:
        out["serve"] = served_stream(L, args.serve_requests)
        out["serve_device_io"] = served_stream(L, args.serve_requests, device=True)
        split = {}
        for mode in ("f16x3", "bf16"):
            s = served_stream(L, args.serve_requests, device=True, prec=mode)
            s["saturated_vs_fp32_batched_step"] = s["saturated_Mpk_per_s"] / fp32_value
            split[mode] = s
        out["serve_device_io_split"] = split
        out["serve_device_io"]["saturated_vs_fp32_batched_step"] = \
            out["serve_device_io"]["saturated_Mpk_per_s"] / fp32_value
        print("[bench] serve legs done", file=sys.stderr, flush=True)

    if "cpu" in legs and not args.no_cpu_baseline:
        nc = args.cpu_clips
        out["cpu_baseline"] = cpu_oracle(spec, masks[:nc], targets[:nc], 1, K, "bench workload")
        out["cpu_scipy_fp32"] = cpu_scipy_fp32(spec, masks[:2], targets[:2], "bench workload")
        if "large" in legs and args.large_steps > 0:
            m3 = W.as_f32_exact(W.curvilinear_mask(2048, 2000))[None]
            t3 = W.manhattan_target(2048, 2001)[None]
            out["large_tiles"]["ilt_2048x2048_3planes_K24"]["cpu_baseline"] = \
                cpu_oracle(W.CONFIG3, m3, t3, 1, 24, "2048^2 three-plane ILT step")
            m5 = W.as_f32_exact(W.curvilinear_mask(4096, 4000))[None]
            t5 = W.manhattan_target(4096, 4001)[None]
            out["large_tiles"]["tile_4096x4096_3planes_K32"]["cpu_baseline"] = \
                cpu_oracle(W.CONFIG5, m5, t5, 1, 4, "4096^2 three-plane tile")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
