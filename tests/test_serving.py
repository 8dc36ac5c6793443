"""The serving loop: continuous batching, captured graphs, budget admission, waits.

The key property: per-event arithmetic does not depend on batch composition, so every
served request's |M|^2 equals, bit for bit, hme_compute on that request alone.  The
graphs are replayed many times, with the program's own eager GPU work and
synchronisations between rounds, and every replay is checked.
"""
import threading

import numpy as np
import pytest

import paper_2507_21039_amd as hme
from workloads import configs

AS = 0.118


def test_server_argument_errors_without_gpu():
    import ctypes
    import os
    if not os.path.exists(hme.LIB_PATH):
        pytest.skip("libhme.so is not built (python -m paper_2507_21039_amd.build)")
    L = hme.lib()
    s = ctypes.c_void_p()
    card = hme.card_struct(configs.card_array())
    assert L.hme_server_create(None, 0, 0, 1 << 30, 2, ctypes.byref(s)) == hme.HME_E_ARG
    assert L.hme_server_create(ctypes.byref(card), 0, 0, 1 << 30, 0, ctypes.byref(s)) == hme.HME_E_ARG
    assert L.hme_server_create(ctypes.byref(card), 0, 0, 1 << 10, 2, ctypes.byref(s)) == hme.HME_E_BUDGET
    rid = ctypes.c_uint64()
    assert L.hme_submit(None, 0, AS, 1, None, None, ctypes.byref(rid)) == hme.HME_E_ARG
    assert L.hme_wait(None, 1, 0.0) == hme.HME_E_ARG
    assert L.hme_server_destroy(None) == hme.HME_OK


@pytest.fixture(scope="module")
def gpu_setup():
    torch = pytest.importorskip("torch")
    card = configs.card_array()
    pools = {}
    for key, proc in (("ggtt", hme.GGTT), ("ggttg", hme.GGTTG), ("ggttgg", hme.GGTTGG)):
        pools[proc] = torch.from_numpy(configs.WORKLOADS[key].momenta(6000)).cuda()
    return torch, card, pools


def _requests(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        proc = [hme.GGTT, hme.GGTTG, hme.GGTTGG][rng.integers(0, 3)]
        nevt = int(np.exp(rng.uniform(0, np.log(3000))))
        start = int(rng.integers(0, 6000 - nevt))
        alpha = [0.118, 0.12][rng.integers(0, 2)]
        out.append((proc, start, nevt, alpha))
    return out


@pytest.mark.gpu
def test_served_equals_alone(gpu_setup):
    torch, card, pools = gpu_setup
    reqs = _requests(1, 48)
    alone = []
    handles = {p: hme.Handle(p, card, hme.FP64) for p in pools}
    for proc, start, nevt, alpha in reqs:
        alone.append(handles[proc].compute(pools[proc][start:start + nevt].contiguous(), alpha_s=alpha))
    torch.cuda.synchronize()
    alone = [a.cpu().numpy() for a in alone]
    for h in handles.values():
        h.close()
    print("[gpu] served vs alone", flush=True)
    with hme.Server(card, hme.FP64, hbm_budget_bytes=64 << 20, nstreams=3) as srv:
        for rnd in range(4):
            outs, ids = [], []
            for proc, start, nevt, alpha in reqs:
                o = torch.full((nevt,), -1.0, dtype=torch.float64, device="cuda")
                outs.append(o)
                ids.append(srv.submit(proc, pools[proc][start:start + nevt], o, alpha))
            # the program's own GPU work while the server runs
            junk = torch.randn(1 << 20, device="cuda").sum().item()
            for rid in ids:
                assert srv.wait(rid) is not None
            torch.cuda.synchronize()
            for k, o in enumerate(outs):
                assert np.array_equal(o.cpu().numpy(), alone[k]), f"round {rnd} request {k}"
        st = srv.stats()
        print(" ", st)
        assert st["completed"] == 4 * len(reqs)
        assert st["batches"] < 4 * len(reqs)  # requests were batched together
        assert st["graphs"] >= 1


@pytest.mark.gpu
def test_concurrent_clients(gpu_setup):
    torch, card, pools = gpu_setup
    reqs = _requests(2, 32)
    with hme.Handle(hme.GGTTG, card, hme.MIXED_FAST) as h:
        ref = h.compute(pools[hme.GGTTG][:2000].contiguous()).cpu().numpy()
    errors = []
    with hme.Server(card, hme.MIXED_FAST, hbm_budget_bytes=32 << 20, nstreams=2) as srv:
        def client(k):
            try:
                for j in range(8):
                    o = torch.empty(2000, dtype=torch.float64, device="cuda")
                    rid = srv.submit(hme.GGTTG, pools[hme.GGTTG][:2000], o)
                    srv.wait(rid)
                    torch.cuda.synchronize()
                    if not np.array_equal(o.cpu().numpy(), ref):
                        errors.append((k, j))
            except Exception as e:  # pragma: no cover - reported below
                errors.append(repr(e))
        ts = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    assert errors == []


@pytest.mark.gpu
def test_request_larger_than_a_slot_runs_in_parts(gpu_setup):
    """A request of more events than one slot holds is split into parts (each its own batch on
    any slot); the result is bitwise that of hme_compute on the whole request."""
    torch, card, pools = gpu_setup
    p = pools[hme.GGTTGG][:6000].contiguous()
    with hme.Handle(hme.GGTTGG, card, hme.FP64) as h:
        alone = h.compute(p)
    torch.cuda.synchronize()
    with hme.Server(card, hme.FP64, hbm_budget_bytes=2 << 20, nstreams=2) as srv:
        cap = (srv.stats()["slot_capacity_bytes"] - 256) // (6 * 32 + 8)
        assert cap < 6000
        o = torch.full((6000,), -1.0, dtype=torch.float64, device="cuda")
        rid = srv.submit(hme.GGTTGG, p, o)
        assert srv.wait(rid) is not None
        torch.cuda.synchronize()
        assert torch.equal(o, alone)
        assert srv.stats()["batches"] >= (6000 + cap - 1) // cap


@pytest.mark.gpu
def test_budget_and_wait_errors(gpu_setup):
    torch, card, pools = gpu_setup
    with hme.Server(card, hme.FP64, hbm_budget_bytes=2 << 20, nstreams=2) as srv:
        cap = (srv.stats()["slot_capacity_bytes"] - 256) // (6 * 32 + 8)
        big = torch.zeros((cap + 1, 6, 4), dtype=torch.float64, device="cuda")
        o = torch.zeros(cap + 1, dtype=torch.float64, device="cuda")
        with pytest.raises(hme.HmeError) as e:
            srv.wait(123456)
        assert e.value.code == hme.HME_E_ARG
        rid = srv.submit(hme.GGTTGG, big[:0], o[:0])
        assert srv.wait(rid, 0.0) == 0.0
        # a full-slot request: wait(0) either times out or is already done; a blocking wait finishes
        p = pools[hme.GGTTGG][:min(cap, 6000)]
        rid = srv.submit(hme.GGTTGG, p, o)
        first = srv.wait(rid, 0.0)
        if first is None:
            assert srv.wait(rid, -1.0) is not None


@pytest.mark.gpu
def test_served_ggttggg_equals_alone(gpu_setup):
    """The process evaluated in pieces, served beside another: bitwise equal to hme_compute alone
    (the server's sub-batches are smaller than the handle's; per-event values do not depend on it)."""
    torch, card, pools = gpu_setup
    p7 = torch.from_numpy(configs.WORKLOADS["ggttggg"].momenta(9000)).cuda()
    rng = np.random.default_rng(3)
    reqs = [(hme.GGTTGGG, 0, 9000)]  # more than one 8192-event part
    for i in range(12):
        proc = [hme.GGTTGG, hme.GGTTGGG][i % 2]
        nevt = int(rng.integers(1, 3000)) if proc == hme.GGTTGG else int(rng.integers(1, 9000 // 2))
        start = int(rng.integers(0, (6000 if proc == hme.GGTTGG else 9000) - nevt))
        reqs.append((proc, start, nevt))
    src = {hme.GGTTGG: pools[hme.GGTTGG], hme.GGTTGGG: p7}
    alone = []
    hs = {p: hme.Handle(p, card, hme.MIXED_FAST) for p in src}
    for proc, start, nevt in reqs:
        alone.append(hs[proc].compute(src[proc][start:start + nevt].contiguous()))
    torch.cuda.synchronize()
    alone = [a.cpu().numpy() for a in alone]
    for h in hs.values():
        h.close()
    print("[gpu] served ggttggg vs alone", flush=True)
    with hme.Server(card, hme.MIXED_FAST, hbm_budget_bytes=1 << 30, nstreams=2) as srv:
        for rnd in range(2):
            outs, ids = [], []
            for proc, start, nevt in reqs:
                o = torch.full((nevt,), -1.0, dtype=torch.float64, device="cuda")
                outs.append(o)
                ids.append(srv.submit(proc, src[proc][start:start + nevt], o))
            for rid in ids:
                assert srv.wait(rid) is not None
            torch.cuda.synchronize()
            for k, o in enumerate(outs):
                assert np.array_equal(o.cpu().numpy(), alone[k]), f"round {rnd} request {k} {reqs[k]}"


@pytest.mark.gpu
def test_ggttggg_workspace_must_fit_a_slot(gpu_setup):
    """An 8 MiB slot cannot hold one 64-event group of gg -> ttbar ggg's double-precision
    workspace (1.6 MB per event): its requests are refused for the budget, others are served."""
    torch, card, pools = gpu_setup
    with hme.Server(card, hme.FP64, hbm_budget_bytes=8 << 20, nstreams=1) as srv:
        p = torch.zeros((4, 7, 4), dtype=torch.float64, device="cuda")
        o = torch.zeros(4, dtype=torch.float64, device="cuda")
        with pytest.raises(hme.HmeError) as e:
            srv.submit(hme.GGTTGGG, p, o)
        assert e.value.code == hme.HME_E_BUDGET
