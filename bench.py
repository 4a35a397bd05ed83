"""Throughput of the SOCS aerial image + ILT adjoint on one MI355X.

One step = one pass of the whole hot path over a batch of synthetic clips:
mask spectrum, per-kernel column/row transforms, |E_k|^2 accumulation,
sigmoid resist, L2 loss against a target, and the adjoint (mask gradient).
The batch is 16 curvilinear 1024 x 1024 clips at 2 nm (NA 0.55, x-dipole
0.3-0.9, K = 24 SOCS kernels, FP32), resident in HBM before timing starts.

Prints one JSON line (rank 0).  The metric counts clips x planes x N^2 x K
pixel-kernels per second; forward and adjoint work is counted once.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "aerial-image Mpixel·kernel/s (fwd+adjoint) vs plain FP32; p50/p99 clip latency"
UNIT = "Mpixel·kernel/s"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3


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
    ap.add_argument("--serve-requests", type=int, default=768,
                    help="requests in the served-stream latency sample (0: skip)")
    return ap.parse_args()


def kernel_model(name, n, Q, B, K, P, clips):
    """Algorithmic (bytes, flops) of one launch of a pass."""
    import math
    lg = math.log2(Q)
    fft = 5.0 * Q * lg                      # nominal complex FFT flops, length Q
    if name == "pass_x_fwd":
        # reads K band rows of Y per row (B complex), writes image + G, reads target
        by = clips * P * (K * Q * B * 8 + 3 * n * n * 4)
        fl = clips * P * K * Q * (fft + 3 * Q)
    elif name == "pass_x_adj":
        # reads and rewrites K band rows per row, reads G
        by = clips * P * (2 * K * Q * B * 8 + n * n * 4)
        fl = clips * P * K * Q * (2 * fft + 2 * Q)
    elif name == "pass_y_fwd":
        by = clips * P * K * (2 * B * B * 8 + Q * B * 8)
        fl = clips * P * K * B * (fft + 6 * B)
    elif name == "pass_y_adj":
        by = clips * P * K * (Q * B * 8 + B * B * 8)
        fl = clips * P * K * B * (fft + 8 * B)
    else:
        return None
    return by, fl


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None when the kernel sources have
    changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_ilt_step_1024x16_K24.txt")
    if not os.path.exists(path):
        return None
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
        return None
    v = vals.get(f"{kernel}.hbm_bytes_calibrated")
    return float(v) if v is not None else None


def cpu_baseline(n_clips: int):
    """Oracle (FP64, direct DFT) on the first n_clips clips of the workload."""
    import numpy as np
    import oracle as O
    import workloads as W
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        blas_threads = os.cpu_count()
    spec = W.CONFIG2
    banks = [O.socs_kernels(spec, 0.0, K=spec.K)]
    dt = 0.0
    for i in range(n_clips):
        m = W.as_f32_exact(W.curvilinear_mask(spec.n, 1000 + i))
        T = W.manhattan_target(spec.n, 1100 + i)
        t0 = time.perf_counter()
        O.gradient(m, T, banks, 50.0, 0.3, method="direct")
        dt += time.perf_counter() - t0
    pk = n_clips * spec.n * spec.n * spec.K
    return {"value": pk / dt / 1e6, "unit": UNIT, "cores": int(blas_threads), "kind": "oracle",
            "sample": f"{n_clips} of the 16 clips ({spec.n}x{spec.n}, K={spec.K}), forward+adjoint, "
                      f"FP64 direct-DFT oracle, {dt:.1f} s (host has {os.cpu_count()} CPUs)"}


def served_stream(L, n_requests: int, rho: float = 0.8, seed: int = 3000, device: bool = False):
    """Served stream: clip sides log-uniform over {256, 512, 1024, 2048},
    Manhattan/curvilinear 50/50, forward or forward+gradient 50/50, K uniform in
    16..32 from resident K_max = 32 banks.  First a closed-loop burst measures
    the saturated request rate; then Poisson arrivals at rho times that rate
    give the p50/p99 latency (submit -> device work done).  device=False: host
    arrays in and out (copies included); device=True: inputs resident in HBM
    and results written to device buffers (no host copies)."""
    import threading

    import numpy as np

    import workloads as W
    sizes = (256, 512, 1024, 2048)
    banks = [L.Bank.from_spec(W.serve_optics(n)) for n in sizes]
    # a small pool of seeded clips per size and kind, reused across requests
    pool = {}
    for bi, n in enumerate(sizes):
        for kind in ("manhattan", "curvilinear"):
            for j in range(2):
                spec = W.ServeRequestSpec(n=n, kind=kind, mode=0, K_use=16, arrival_s=0.0, seed=seed + 97 * bi + j)
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

    def args_of(r, i):
        bi = sizes.index(r.n)
        m = pool[(bi, r.kind, i % 2)]
        return bi, m, r.K_use, (pool[(bi, "target")] if r.mode else None)

    def submit(i, r):
        bi, m, k, tgt = args_of(r, i)
        if not device:
            return srv.submit(bi, m, K_use=k, target=tgt)
        o = outs[i]
        return srv.submit_device(bi, dpool[(bi, r.kind, i % 2)], o["image"], K_use=k,
                                 target=dpool[(bi, "target")] if r.mode else None, grad=o.get("grad"),
                                 loss=o.get("loss"))

    def collect(i, r):
        if device:
            return srv.poll_info(tickets_ref[0][i])
        return srv.poll(tickets_ref[0][i], r.n, 1, bool(r.mode))

    tickets_ref = [None]

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
            "saturated_req_per_s": mu, "saturated_Mpk_per_s": pk / wall / 1e6,
            "offered_load": rho, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "open_loop_Mpk_per_s": pk2 / wall2 / 1e6, "precision": "fp32",
            "io": "device-resident" if device else "host arrays (PCIe copies included)"}


def mixed_precision(L, torch, step, fwd, img, grad, steps, pk, fp32_value, fp32_fwd_value):
    """Each split-precision mode on the same batch: throughput, speed-up over
    FP32 and relative L2 error of the image and the gradient against the FP32
    path (the FP32 path itself is held to 1e-5 of the FP64 oracle by the tests)."""
    step()
    torch.cuda.synchronize()
    img32, grad32 = img.clone(), grad.clone()
    g2 = torch.empty_like(grad)
    res = {}
    for name in ("f16x3", "bf16x3", "f16", "bf16"):
        code = L.prec_code(name)
        step(code, g2)
        torch.cuda.synchronize()
        e_img = float(torch.linalg.vector_norm((img - img32).double()) / torch.linalg.vector_norm(img32.double()))
        e_grad = float(torch.linalg.vector_norm((g2 - grad32).double()) / torch.linalg.vector_norm(grad32.double()))
        L.profile_read()
        L.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step(code, g2)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        L.profile_enable(False)
        prof = L.profile_read()
        t0 = time.perf_counter()
        for _ in range(steps):
            fwd(name)
        torch.cuda.synchronize()
        dtf = (time.perf_counter() - t0) / steps
        res[name] = {"value": pk / dt / 1e6, "ms_per_step": dt * 1e3, "speedup_vs_fp32": pk / dt / 1e6 / fp32_value,
                     "forward_value": pk / dtf / 1e6, "forward_speedup_vs_fp32": pk / dtf / 1e6 / fp32_fwd_value,
                     "rel_l2_image_vs_fp32": e_img, "rel_l2_grad_vs_fp32": e_grad,
                     "kernels_avg_ms": {k: round(v[1] / max(v[0], 1), 5) for k, v in prof.items()}}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
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
    bank = L.Bank.from_spec(spec)
    masks = np.stack([W.as_f32_exact(W.curvilinear_mask(spec.n, 1000 + i)) for i in range(batch)])
    targets = np.stack([W.manhattan_target(spec.n, 1100 + i) for i in range(batch)])
    d_mask = torch.from_numpy(masks.astype(np.float32)).cuda()
    d_target = torch.from_numpy(targets.astype(np.float32)).cuda()
    n, K, P = spec.n, spec.K, len(spec.focus_nm)
    img = torch.empty((batch, P, n, n), device="cuda")
    grad = torch.empty((batch, n, n), device="cuda")
    loss = torch.empty((batch,), device="cuda", dtype=torch.float64)

    def step(prec=L.A.LITHO_PREC_FP32, g=grad):
        L._check(L._lib.litho_image_grad(
            bank.handle, L._dev_ptr(d_mask, "mask"), batch, K, L._dev_ptr(d_target, "target"),
            L.C.byref(L.A.Resist(slope=50.0, threshold=0.3)), None, L._dev_ptr(img, "image"),
            L._dev_ptr(loss, "loss", torch.float64), L._dev_ptr(g, "grad"), prec,
            L.C.c_void_p(L._stream_handle())), "litho_image_grad")

    def fwd(prec="fp32", out=img):
        L.image(bank, d_mask, out=out, prec=prec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    L.profile_read()
    L.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.profile_enable(False)
    prof = L.profile_read()

    # forward-only throughput (same batch), for reference
    for _ in range(2):
        fwd()
    torch.cuda.synchronize()
    tf0 = time.perf_counter()
    for _ in range(args.steps):
        fwd()
    torch.cuda.synchronize()
    dtf = time.perf_counter() - tf0

    pk = batch * P * n * n * K
    ms = dt / args.steps * 1e3
    value = pk / (dt / args.steps) / 1e6
    fwd_value = pk / (dtf / args.steps) / 1e6

    info = bank
    kern = {}
    for name, (cnt, tot) in prof.items():
        avg = tot / max(cnt, 1)
        rec = {"launches": cnt, "avg_ms": avg, "share": tot / (dt * 1e3)}
        mod = kernel_model(name, n, info.inner_grid, info.B, K, P, batch)
        if mod:
            by, fl = mod
            rec["GBps"] = by / (avg * 1e-3) / 1e9
            rec["TFLOPs"] = fl / (avg * 1e-3) / 1e12
        kern[name] = rec
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    by, fl = kernel_model(dom, n, info.inner_grid, info.B, K, P, batch)
    avg = kern[dom]["avg_ms"] * 1e-3
    traffic = measured_traffic(dom)
    roof = {"kernel": dom, "bound": "alu", "achieved": fl / avg / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": fl / avg / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3, copy-calibrated)",
            "algorithmic_bytes": by,
            "nonpacked_fp32_peak": 78.6, "frac_of_nonpacked": fl / avg / 1e12 / 78.6,
            "hbm_view": {"achieved_GBps": by / avg / 1e9, "peak_GBps": HBM_PEAK_GBS,
                         "frac": by / avg / 1e9 / HBM_PEAK_GBS}}
    print(json.dumps({"kernels": kern}), file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ILT step (image + sigmoid resist + L2 loss + mask gradient), {batch} curvilinear "
                               f"clips {n}x{n} at 2 nm, NA 0.55 x-dipole 0.3-0.9, K={K}, 1 focus plane, FP32",
                   "clips": batch, "n": n, "K": K, "planes": P, "inner_grid": info.inner_grid, "band": info.B},
        "forward_only": {"value": fwd_value, "unit": UNIT, "ms_per_batch": dtf / args.steps * 1e3},
        "roofline": roof,
    }
    if args.mp_steps > 0:
        out["mixed_precision"] = mixed_precision(L, torch, step, fwd, img, grad, args.mp_steps, pk,
                                                 value, fwd_value)
    if args.serve_requests > 0:
        out["serve"] = served_stream(L, args.serve_requests)
        out["serve_device_io"] = served_stream(L, args.serve_requests, device=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_clips)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
