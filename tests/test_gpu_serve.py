"""Served stream on the GPU: results are the same alone and in a mixed batch,
match the oracle, and the serve ABI reports its errors."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2602_15036_amd import litho
    return litho


@pytest.fixture(scope="module")
def banks(L):
    out = []
    for n in (256, 512):
        out.append(L.Bank.from_spec(W.serve_optics(n).with_(K=20)))
    return out


def _requests():
    reqs = []
    rng = np.random.default_rng(3000)
    for i in range(24):
        bi = int(rng.integers(0, 2))
        n = (256, 512)[bi]
        kind = "manhattan" if i % 2 else "curvilinear"
        m = W.manhattan_mask(n, 50 + i, n_rects=max(1, 20 * n * n // 16384)) if kind == "manhattan" \
            else W.curvilinear_mask(n, 50 + i)
        mode = int(rng.integers(0, 2))
        K = int(rng.integers(12, 21))
        T = W.manhattan_target(n, 80 + i) if mode else None
        reqs.append((bi, n, W.as_f32_exact(m), K, T))
    return reqs


def test_alone_equals_mixed_and_matches_oracle(L, banks):
    reqs = _requests()
    srv = L.Server(banks, hbm_budget=2 << 30, max_slots=6)
    # mixed: submit everything, then collect
    tickets = [srv.submit(bi, m, K_use=K, target=T) for (bi, n, m, K, T) in reqs]
    mixed = [srv.poll(t, n, 1, T is not None) for t, (bi, n, m, K, T) in zip(tickets, reqs)]
    # overlap: some request started before another finished
    spans = sorted((r["t_start_us"], r["t_done_us"]) for r in mixed)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    # alone: one at a time
    for (bi, n, m, K, T), mix in zip(reqs, mixed):
        t = srv.submit(bi, m, K_use=K, target=T)
        alone = srv.poll(t, n, 1, T is not None)
        assert np.array_equal(alone["image"], mix["image"])
        if T is not None:
            assert np.array_equal(alone["grad"], mix["grad"])
            assert alone["loss"] == mix["loss"]
    srv.close()
    # oracle parity on two of them
    for idx in (0, 1):
        bi, n, m, K, T = reqs[idx]
        lam, phi = O.socs_kernels(W.serve_optics(n), 0.0, K=K)
        ref = O.image(m, lam, phi, method="fft")
        err = np.linalg.norm(mixed[idx]["image"][0] - ref) / np.linalg.norm(ref)
        assert err < 1e-5


def test_serve_errors(L, banks):
    srv = L.Server(banks, hbm_budget=1 << 20, max_slots=2, max_queue=2)   # 1 MiB: nothing fits
    m = np.zeros((256, 256), np.float32)
    with pytest.raises(L.LithoError) as e:
        srv.submit(0, m, K_use=8)
    assert "NOMEM" in str(e.value)
    srv.close()
    srv = L.Server(banks, hbm_budget=4 << 30, max_slots=1, max_queue=2)
    with pytest.raises(L.LithoError):
        srv.submit(0, m, K_use=99)
    with pytest.raises(L.LithoError) as e:
        srv.poll(424242, 256, 1, False, timeout_us=0)
    assert "NOTFOUND" in str(e.value)
    # a full queue: device-resident submits (no host copy) outpace one slot
    import torch
    dm = torch.zeros((512, 512), device="cuda")
    outs = [torch.empty((1, 512, 512), device="cuda") for _ in range(8)]
    torch.cuda.synchronize()
    tickets = []
    busy = False
    for i in range(500):
        try:
            tickets.append(srv.submit_device(1, dm, outs[i % 8], K_use=20))
        except L.LithoError as err:
            assert "BUSY" in str(err)
            busy = True
            break
    assert busy
    for t in tickets:
        assert srv.poll_info(t) is not None
    srv.close()


def test_device_resident_requests_match_host_requests(L, banks):
    # the same requests with device-resident I/O: bit-identical to the host
    # path, mixed with host requests in flight, and one split-precision request
    import torch
    reqs = _requests()[:12]
    srv = L.Server(banks, hbm_budget=2 << 30, max_slots=6)
    host = [srv.poll(srv.submit(bi, m, K_use=K, target=T), n, 1, T is not None) for (bi, n, m, K, T) in reqs]
    dev_bufs, tickets = [], []
    for i, (bi, n, m, K, T) in enumerate(reqs):
        d = {"mask": torch.from_numpy(m.astype(np.float32)).cuda(), "image": torch.empty((1, n, n), device="cuda")}
        if T is not None:
            d.update(target=torch.from_numpy(T.astype(np.float32)).cuda(),
                     grad=torch.empty((n, n), device="cuda"),
                     loss=torch.empty((1,), device="cuda", dtype=torch.float64))
        torch.cuda.synchronize()
        dev_bufs.append(d)
        tickets.append(srv.submit_device(bi, d["mask"], d["image"], K_use=K, target=d.get("target"),
                                         grad=d.get("grad"), loss=d.get("loss")))
        if i % 3 == 0:   # host requests in between
            srv.poll(srv.submit(bi, m, K_use=K, target=T), n, 1, T is not None)
    for t in tickets:
        info = srv.poll_info(t)
        assert info["t_done_us"] >= info["t_start_us"] >= info["t_submit_us"]
    for d, h, (bi, n, m, K, T) in zip(dev_bufs, host, reqs):
        assert np.array_equal(d["image"].cpu().numpy(), h["image"])
        if T is not None:
            assert np.array_equal(d["grad"].cpu().numpy(), h["grad"])
            assert d["loss"].item() == h["loss"]
    # split precision through the served form: same as the direct call
    bi, n, m, K, T = reqs[0]
    img = torch.empty((1, n, n), device="cuda")
    srv.poll_info(srv.submit_device(bi, dev_bufs[0]["mask"], img, K_use=K, prec="f16x3"))
    ref = L.image(banks[bi], dev_bufs[0]["mask"][None], K_use=K, prec="f16x3")
    assert torch.equal(img, ref[0])
    with pytest.raises(L.LithoError):      # device request without an output buffer
        req = L.A.Request(bank=0, K_use=8, mode=0, d_mask=dev_bufs[0]["mask"].data_ptr())
        L._check(L._lib.litho_serve_submit(srv._h, L.C.byref(req), L.C.byref(L.C.c_uint64())), "litho_serve_submit")
    srv.close()


def test_large_clips_and_split_modes_alone_equal_mixed(L):
    # 1024 and 2048 clips, FP32 and split-precision requests in one mix: each
    # result equals the same request run alone, bit for bit
    banks = [L.Bank.from_spec(W.serve_optics(n).with_(K=16)) for n in (1024, 2048)]
    rng = np.random.default_rng(3100)
    reqs = []
    for i in range(10):
        bi = i % 2
        n = (1024, 2048)[bi]
        m = W.as_f32_exact(W.curvilinear_mask(n, 500 + i))
        T = W.manhattan_target(n, 600 + i) if i % 3 else None
        prec = ("fp32", "f16x3", "bf16")[i % 3]
        reqs.append((bi, n, m, int(rng.integers(8, 17)), T, prec))
    srv = L.Server(banks, hbm_budget=24 << 30, max_slots=4)
    tickets = [srv.submit(bi, m, K_use=K, target=T, prec=p) for (bi, n, m, K, T, p) in reqs]
    mixed = [srv.poll(t, n, 1, T is not None) for t, (bi, n, m, K, T, p) in zip(tickets, reqs)]
    spans = sorted((r["t_start_us"], r["t_done_us"]) for r in mixed)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    for (bi, n, m, K, T, p), mix in zip(reqs, mixed):
        alone = srv.poll(srv.submit(bi, m, K_use=K, target=T, prec=p), n, 1, T is not None)
        assert np.array_equal(alone["image"], mix["image"]), (n, p)
        if T is not None:
            assert np.array_equal(alone["grad"], mix["grad"]) and alone["loss"] == mix["loss"]
    srv.close()
    for b in banks:
        b.close()


def test_device_memory_stays_within_the_budget(L):
    # mixed sizes and modes through 8 slots under a 1.5 GiB budget: the
    # device memory the server holds (slot arenas with workspaces and I/O
    # buffers), read with hipMemGetInfo while the stream runs, stays within it
    import threading
    import time

    import torch
    banks = [L.Bank.from_spec(W.serve_optics(n).with_(K=20)) for n in (256, 512, 1024, 2048)]
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    budget = 3 << 29
    srv = L.Server(banks, hbm_budget=budget, max_slots=8)
    rng = np.random.default_rng(3200)
    masks = {n: W.as_f32_exact(W.curvilinear_mask(n, 700 + n)) for n in (256, 512, 1024, 2048)}
    tgts = {n: W.manhattan_target(n, 800 + n) for n in (256, 512, 1024, 2048)}
    used, stop = [], [False]

    def watch():
        while not stop[0]:
            used.append(free0 - torch.cuda.mem_get_info()[0])
            time.sleep(0.002)
    th = threading.Thread(target=watch)
    th.start()
    tickets = []
    for i in range(48):
        bi = int(rng.integers(0, 4))
        n = (256, 512, 1024, 2048)[bi]
        tickets.append((srv.submit(bi, masks[n], K_use=int(rng.integers(10, 21)),
                                   target=tgts[n] if i % 2 else None), n, bool(i % 2)))
    for t, n, g in tickets:
        assert srv.poll(t, n, 1, g) is not None
    used.append(free0 - torch.cuda.mem_get_info()[0])
    stop[0] = True
    th.join()
    srv.close()
    slack = 64 << 20      # streams, events and allocator granularity
    print(f"served under a {budget >> 20} MiB budget: peak device use {max(used) >> 20} MiB")
    assert max(used) <= budget + slack
    for b in banks:
        b.close()
