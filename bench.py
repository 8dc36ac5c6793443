"""Benchmark: |M|^2 events/s for g g -> t tbar g g on one MI355X, FP64 and mixed precision.

One step is one hme_compute call over the whole batch (1,048,576 RAMBO events at
sqrt(s) = 2 TeV with dR(g,g) > 0.4, seed 4), momenta already resident in HBM:
external wavefunctions, propagator denominators, the 123-diagram sequence for
every good helicity, jamps, colour sum, helicity sum and normalisation, all in
one kernel launch.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "|M|^2 events/s on 1 MI355X (gg→tt̄gg, FP64 vs mixed); p50/p99 served latency"
PEAK_FP64_VALU = 78.6e12  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP32_VALU = 157.3e12  # published FP32 vector peak (twice the FP64 rate)
PEAK_HBM = 8.0e12

# HBM traffic of one FP64 gg -> ttbar gg launch (1,048,576 events) from rocprofv3 counters
# (profiles/me2_ggttgg_1M_traffic.md): L2-to-memory read requests by size (TCC_EA0_RDREQ_32B/64B/
# 128B) and WRITE_SIZE.  Calibrated on kernels of known traffic: a 256 MiB copy and a 256 MiB
# read-only sum issue 2,097,152 requests of 128 B (exactly 256 MiB, factor 1.000; FETCH_SIZE, which
# counts a 128 B request as 64 B on this part, reads half); a 256 MiB fill writes WRITE_SIZE =
# 262,144 KiB (factor 1.000).  Valid only for the kernel sources it was taken on (sha256 prefix of
# me2_kernels.h + colour_mfma.h + helas.h + procs/ggttgg.h); otherwise traffic is null.
TRAFFIC = {"source_sha": "3e458153565a38e9", "nevt": 1048576,
           "rdreq_32b": 0, "rdreq_64b": 3166233, "rdreq_128b": 104, "fetch_size_kib": 197895.875,
           "write_kib": 8192.0, "write_factor": 1.0}

# VALU and MFMA instruction counters of the same launches (profiles/me2_ggttgg_1M_valu_counters.md),
# wave instructions summed over the device: FLOPs = 64 lanes x (2 FMA + ADD + MUL + TRANS) plus
# 512 per MFMA "MOPS" unit (the counter's own scale).
COUNTERS = {
    "source_sha": "3e458153565a38e9", "nevt": 1048576,
    "fp64": {"FMA_F64": 12253654936, "ADD_F64": 2386559326, "MUL_F64": 3064986948, "TRANS_F64": 45088068,
             "VALU": 18407744330},
    "mixed_fast": {"FMA_F32": 11243880448, "ADD_F32": 1732247552, "MUL_F32": 2757754880, "TRANS_F32": 0,
                   "FMA_F64": 351272960, "ADD_F64": 694157312, "MUL_F64": 223346688, "TRANS_F64": 45088768,
                   "MFMA_MOPS_BF16": 2684354560, "VALU": 18330157056},
}


def counter_flops(mode: str, nevt: int):
    """Vector-ALU FLOPs per launch from the counters, or None if they were taken on other sources."""
    if kernel_source_sha() != COUNTERS["source_sha"] or nevt != COUNTERS["nevt"]:
        return None
    c = COUNTERS[mode]
    return 64.0 * sum(2 * v if k.startswith("FMA") else v for k, v in c.items() if k[:4] in ("FMA_", "ADD_", "MUL_", "TRAN"))


def counter_mfma_flops(mode: str, nevt: int):
    """Matrix-core FLOPs per launch from the MFMA counters (bf16 operand splits included), or None."""
    if kernel_source_sha() != COUNTERS["source_sha"] or nevt != COUNTERS["nevt"]:
        return None
    return 512.0 * sum(v for k, v in COUNTERS[mode].items() if k.startswith("MFMA"))


def kernel_source_sha() -> str:
    import hashlib
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2507_21039_amd", "csrc")
    h = hashlib.sha256()
    for f in ("me2_kernels.h", "colour_mfma.h", "helas.h", "procs/ggttgg.h"):
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(nevt: int):
    """HBM bytes per launch (read requests by size + calibrated WRITE_SIZE), or None."""
    if kernel_source_sha() != TRAFFIC["source_sha"] or nevt != TRAFFIC["nevt"]:
        return None
    read = 32 * TRAFFIC["rdreq_32b"] + 64 * TRAFFIC["rdreq_64b"] + 128 * TRAFFIC["rdreq_128b"]
    return read + 1024 * TRAFFIC["write_kib"] * TRAFFIC["write_factor"]


def colour_dense_excess(key: str) -> float:
    """Flops per helicity by which the dense colour count (4 ncol^2) exceeds the symmetric form
    the vector-ALU kernels execute (from the generator's process table)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2507_21039_amd", "csrc", "procs",
                        "processes.json")
    with open(path) as fh:
        p = json.load(fh)[key]
    return p["flops_colour"] - p["flops_colour_symmetric"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_steps(h, mom, out, steps, warmup, alpha_s=0.118):
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        h.compute(mom, out, alpha_s, stream)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        h.compute(mom, out, alpha_s, stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall


def cpu_baseline(proc, p, gpu_out, card, target_s=12.0):
    """The FP64 oracle on the host cores over a bounded sample of the same events."""
    import oracle
    threads = oracle.default_threads()
    n = 256
    oracle.me2(proc, p[:64], card)  # warm the library and its colour matrix
    while True:
        t0 = time.perf_counter()
        ref = oracle.me2(proc, p[:n], card, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= target_s or n >= len(p):
            break
        n = min(len(p), int(n * max(2.0, min(8.0, target_s / max(dt, 1e-3)))))
    rel = np.abs(gpu_out[:n] / ref - 1)
    return dict(value=n / dt, unit="events/s", cores=threads, kind="oracle",
                sample=f"first {n} events of the same batch, colour-ordered FP64 oracle, {dt:.1f} s",
                max_rel_diff_vs_gpu=float(rel.max()))


def ggttggg_leg(card, steps=3, warmup=1):
    """gg -> ttbar ggg alone (the served mix's largest process): 65536 RAMBO events at 2 TeV, seed 5,
    in its three precisions (the paper's FP64 against mixed contrast is about this process), timed
    like the main workload; MIXED_FAST is the headline of this leg."""
    import torch

    import oracle
    import paper_2507_21039_amd as hme
    from workloads import configs
    w = configs.WORKLOADS["ggttggg"]
    p = w.momenta()
    mom = torch.from_numpy(p).cuda()
    out = torch.empty(w.nevt, dtype=torch.float64, device="cuda")
    res, outs = {}, {}
    for prec in (hme.MIXED_FAST, hme.FP64, hme.MIXED_PAPER):
        name = hme.PRECISION_NAMES[prec]
        with hme.Handle(hme.GGTTGGG, card, prec) as h:
            info = h.query()
            gpu_s, _ = time_steps(h, mom, out, steps, warmup)
        per = gpu_s / steps
        tflops = info["flops_per_event"] * w.nevt / per / 1e12
        peak = PEAK_FP32_VALU if prec == hme.MIXED_FAST else PEAK_FP64_VALU
        outs[name] = out.cpu().numpy().copy()
        res[name] = {"value": w.nevt / per, "ms_per_step": per * 1e3, "achieved_tflops": tflops,
                     "frac_of_valu_peak": tflops * 1e12 / peak, "valu_peak_tflops": peak / 1e12,
                     "workspace_bytes_per_event": info["workspace_bytes_per_event"]}
        log(f"[bench] gg->ttbar ggg {name}: {w.nevt / per:.4g} events/s, {per * 1e3:.2f} ms")
    for name in ("mixed_fast", "mixed_paper"):
        rel = np.abs(outs[name] / outs["fp64"] - 1)
        res[name].update(max_rel_diff_vs_fp64=float(rel.max()), p99_rel_diff_vs_fp64=float(np.quantile(rel, 0.99)))
    idx = np.linspace(0, w.nevt - 1, 384).astype(int)  # about 10 s of the oracle on 16 cores
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    ref = oracle.me2(configs.GGTTGGG, p[idx], card, nthreads=threads)
    dt = time.perf_counter() - t0
    fast = res["mixed_fast"]
    return {"value": fast["value"], "unit": "events/s", "ms_per_step": fast["ms_per_step"], "steps": steps,
            "workload": f"gg->ttbar ggg, {w.nevt} RAMBO events at sqrt(s)=2 TeV, no cuts, seed 5",
            "dtype": "f32 vertices/propagators/jamps, bf16x3-split MFMA colour sum with f32 accumulation, "
                     "f64 externals and sums",
            "diagrams": 1240, "helicities": 128, "good_helicities": info["ngoodhel"], "colour_flows": 120,
            "achieved_tflops": fast["achieved_tflops"], "frac_of_valu_peak": fast["frac_of_valu_peak"],
            "precisions": res,
            "max_rel_diff_vs_oracle_sample": {k: float(np.max(np.abs(v[idx] / ref - 1))) for k, v in outs.items()},
            "workspace_bytes_per_event": fast["workspace_bytes_per_event"],
            "cpu_baseline": {"value": len(idx) / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
                             "sample": f"{len(idx)} evenly spaced events of the same batch, FP64 oracle, {dt:.1f} s"}}


def e2e_leg(card, steps=5, warmup=2):
    """Flat Monte Carlo on the device for gg -> ttbar gg at 2^20 points per step: RAMBO points
    (Delta R cut as zero weight), FP64 |M|^2, weighted sum; each stage timed with events on the
    stream it runs on."""
    import torch

    import paper_2507_21039_amd as hme
    from workloads import configs
    w = configs.WORKLOADS["ggttgg"]
    kind, value = configs.CUT_CODES[w.cut_text]
    n = w.nevt
    stream = torch.cuda.current_stream()
    mom = torch.empty((n, hme.NPAR[w.process], 4), dtype=torch.float64, device="cuda")
    wt = torch.empty(n, dtype=torch.float64, device="cuda")
    me = torch.empty(n, dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t = np.zeros(3)
    sums = []
    with hme.Handle(w.process, card, hme.FP64) as h:
        for step in range(warmup + steps):
            first = step * n
            ev[0].record(stream)
            hme.rambo(w.process, card, w.sqrt_s, w.seed, n, first, kind | hme.CUT_NO_RETRY, value, out=mom,
                      weights=wt, stream=stream)
            ev[1].record(stream)
            h.compute(mom, me, 0.118, stream)
            ev[2].record(stream)
            sums.append(hme.weighted_sum(me, wt, stream))
            ev[3].record(stream)
            torch.cuda.synchronize()
            if step >= warmup:
                t += [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(3)]
    tot = np.sum([x.cpu().numpy() for x in sums], axis=0)
    sigma, err = hme.cross_section_pb(tot, n * (warmup + steps), w.sqrt_s)
    per = t / steps
    rambo_bytes = n * (hme.NPAR[w.process] * 4 + 1) * 8
    return {"value": n / per.sum(), "unit": "events/s", "steps": steps, "nevt_per_step": n,
            "workload": f"gg->ttbar gg flat Monte Carlo at sqrt(s)=2 TeV, dR(g,g)>0.4 as zero weight, seed 4, "
                        f"event numbers 0..{n * (warmup + steps) - 1}",
            "ms_rambo": per[0] * 1e3, "ms_me2": per[1] * 1e3, "ms_sum": per[2] * 1e3,
            "rambo_written_gbps": rambo_bytes / per[0] / 1e9,
            "sigma_pb": sigma, "sigma_err_pb": err, "points": n * (warmup + steps)}


def pcie_leg(card, p, steps=5, warmup=2):
    """gg -> ttbar gg FP64 with the batch handed over in host memory (pinned): momenta copied to
    the device, |M|^2, |M|^2 copied back, all on one stream and timed there.  The library's
    boundary takes device pointers; this is the rate a caller holding host buffers sees."""
    import torch

    import paper_2507_21039_amd as hme
    from workloads import configs
    n = p.shape[0]
    host_in = torch.empty(p.shape, dtype=torch.float64, pin_memory=True)
    host_in.numpy()[...] = p
    host_out = torch.empty(n, dtype=torch.float64, pin_memory=True)
    mom = torch.empty(p.shape, dtype=torch.float64, device="cuda")
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t = np.zeros(3)
    with hme.Handle(configs.GGTTGG, card, hme.FP64) as h:
        for step in range(warmup + steps):
            ev[0].record(stream)
            mom.copy_(host_in, non_blocking=True)
            ev[1].record(stream)
            h.compute(mom, out, 0.118, stream)
            ev[2].record(stream)
            host_out.copy_(out, non_blocking=True)
            ev[3].record(stream)
            torch.cuda.synchronize()
            if step >= warmup:
                t += [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(3)]
    per = t / steps
    return {"value": n / per.sum(), "unit": "events/s", "nevt": n, "steps": steps,
            "ms_h2d": per[0] * 1e3, "ms_me2": per[1] * 1e3, "ms_d2h": per[2] * 1e3,
            "h2d_gbps": p.nbytes / per[0] / 1e9, "d2h_gbps": n * 8 / per[2] / 1e9,
            "note": "not the headline value: the headline times |M|^2 on momenta already in HBM"}


def select_leg(card, steps=3, warmup=1):
    """Cost of the per-event helicity and colour-flow choice (hme_compute_select) and of a
    strong coupling per event (hme_compute_alphas) against hme_compute on the same resident batch (gg -> ttbar gg FP64 at 2^20 events and
    gg -> ttbar ggg single precision at 65536), each timed with events on the launch stream."""
    import torch

    import paper_2507_21039_amd as hme
    from workloads import configs
    res = {}
    for key, prec in (("ggttgg", hme.FP64), ("ggttggg", hme.MIXED_FAST)):
        w = configs.WORKLOADS[key]
        kind, value = configs.CUT_CODES[w.cut_text]
        mom = hme.rambo(w.process, card, w.sqrt_s, w.seed, w.nevt, 0, kind, value)
        gen = torch.Generator(device="cuda").manual_seed(1)
        rh = torch.rand(w.nevt, dtype=torch.float64, device="cuda", generator=gen)
        rc = torch.rand(w.nevt, dtype=torch.float64, device="cuda", generator=gen)
        stream = torch.cuda.current_stream()
        out = torch.empty(w.nevt, dtype=torch.float64, device="cuda")
        t = {}
        with hme.Handle(w.process, card, prec) as h:
            alphas = 0.1 + 0.05 * rh  # one strong coupling per event
            legs = [("compute", lambda: h.compute(mom, out, 0.118, stream)),
                    ("select", lambda: h.compute_select(mom, rh, rc, 0.118, stream)),
                    ("alphas", lambda: h.compute_alphas(mom, alphas, out, stream))]
            if w.process != hme.GGTTGGG:
                legs.append(("channels", lambda: h.compute_channels(mom, 0.118, stream)))
            for name, fn in legs:
                for _ in range(warmup):
                    fn()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(steps):
                    fn()
                b.record(stream)
                torch.cuda.synchronize()
                t[name] = a.elapsed_time(b) / steps
        res[key] = {"nevt": w.nevt, "precision": hme.PRECISION_NAMES[prec], "ms_compute": t["compute"],
                    "ms_select": t["select"], "overhead": t["select"] / t["compute"] - 1,
                    "ms_per_event_alpha_s": t["alphas"], "overhead_per_event_alpha_s": t["alphas"] / t["compute"] - 1,
                    "events_per_s_select": w.nevt / t["select"] * 1e3}
        if "channels" in t:
            res[key].update(ms_channels=t["channels"], overhead_channels=t["channels"] / t["compute"] - 1)
    return res


# The other configurations, each timed like the main workload on momenta made on the device
# (hme_rambo: the workload's energy, seed and cuts), in every precision the library builds,
# with the mixed-precision error distributions against the FP64 output and the oracle timed
# on the host cores: all events of e+e- -> mu+mu-, gg -> ttbar and gg -> ttbar g, a bounded
# leading sample of the Drell-Yan processes.
CONFIG_LEGS = (  # key, label, cpu-baseline sample (None: every event)
    ("eemumu", "C1 e+e- -> mu+mu- (photon + Z), 16384 events at 500 GeV, seed 1", None),
    ("ggtt", "C2 gg -> ttbar, 524288 events at 1 TeV, seed 2", None),
    ("ggttg", "C3 gg -> ttbar g, 1048576 events at 1.5 TeV, pT(g) > 20 GeV, seed 3", None),
    ("uuee", "Drell-Yan u u~ -> e+ e-, 1048576 events at 1 TeV, seed 6", 262144),
    ("uueeg", "Drell-Yan u u~ -> e+ e- g, 1048576 events at 1 TeV, pT(g) > 20 GeV, seed 6", 131072),
    ("uueegg", "Drell-Yan u u~ -> e+ e- g g, 1048576 events at 1 TeV, dR(g,g) > 0.4, seed 6", 32768),
    ("uueeggg", "Drell-Yan u u~ -> e+ e- g g g, 1048576 events at 1 TeV, dR(g,g) > 0.4, seed 6", 8192),
)


def configs_leg(card, steps=10, warmup=3, cpu=True):
    import torch

    import oracle
    import paper_2507_21039_amd as hme
    from workloads import configs
    res = {}
    for key, label, sample in CONFIG_LEGS:
        w = configs.WORKLOADS[key]
        kind, value = configs.CUT_CODES[w.cut_text]
        mom = hme.rambo(w.process, card, w.sqrt_s, w.seed, w.nevt, 0, kind, value)
        out = torch.empty(w.nevt, dtype=torch.float64, device="cuda")
        precs = (hme.FP64,) if w.process == hme.EEMUMU else (hme.FP64, hme.MIXED_FAST, hme.MIXED_PAPER)
        entry, outs = {"workload": label, "nevt": w.nevt}, {}
        for prec in precs:
            name = hme.PRECISION_NAMES[prec]
            with hme.Handle(w.process, card, prec) as h:
                info = h.query()
                gpu_s, _ = time_steps(h, mom, out, steps, warmup)
            per = gpu_s / steps
            peak = PEAK_FP32_VALU if prec == hme.MIXED_FAST else PEAK_FP64_VALU
            tflops = info["flops_per_event"] * w.nevt / per / 1e12
            outs[name] = out.cpu().numpy().copy()
            entry[name] = {"value": w.nevt / per, "unit": "events/s", "ms_per_step": per * 1e3,
                           "achieved_tflops": tflops, "frac_of_valu_peak": tflops * 1e12 / peak}
            entry.update(diagrams=info["ndiag"], helicities=info["nhel"], good_helicities=info["ngoodhel"],
                         colour_flows=info["ncol"], flops_per_event=info["flops_per_event"])
            log(f"[bench] {key} {name}: {w.nevt / per:.4g} events/s, {per * 1e3:.3f} ms/step")
        for name in outs:
            if name != "fp64":
                rel = np.abs(outs[name] / outs["fp64"] - 1)
                entry[name].update(max_rel_diff_vs_fp64=float(rel.max()),
                                   p99_rel_diff_vs_fp64=float(np.quantile(rel, 0.99)),
                                   median_rel_diff_vs_fp64=float(np.median(rel)))
        if cpu:
            n = w.nevt if sample is None else sample
            p = mom[:n].cpu().numpy()
            threads = oracle.default_threads()
            t0 = time.perf_counter()
            ref = oracle.me2(w.process, p, card, nthreads=threads)
            dt = time.perf_counter() - t0
            entry["cpu_baseline"] = {
                "value": n / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
                "sample": f"{'all' if sample is None else 'first'} {n} events of the same batch, FP64 oracle, "
                          f"{dt:.1f} s",
                "max_rel_diff_vs_gpu_fp64": float(np.max(np.abs(outs["fp64"][:n] / ref - 1)))}
            log(f"[bench] {key} oracle: {n / dt:.4g} events/s on {threads} threads")
        res[key] = entry
        del mom, out
    return res


def served_leg(card, precision, nwarm=200, ntimed=3000, budget=32 << 30, nstreams=4):
    """Poisson request stream (200 requests/s, sizes log-uniform in 256..65536) through the server.

    Latency is measured inside the library from hme_submit to the end of the request's batch
    on the device.  Momenta come from per-process pools resident in HBM.
    """
    import threading

    import torch

    import paper_2507_21039_amd as hme
    from workloads import configs
    procs_avail = [configs.GGTT, configs.GGTTG, configs.GGTTGG, configs.GGTTGGG]
    arrival, procs, nevt, _ = configs.served_requests(nwarm + ntimed, processes=procs_avail)
    w = configs.WORKLOADS["served"]
    pools = {}
    for p in procs_avail:
        wl = configs.Workload("pool", p, 65536, w.sqrt_s, w.seed)
        pools[p] = torch.from_numpy(wl.momenta()).cuda()
    out = torch.empty(int(nevt.sum()), dtype=torch.float64, device="cuda")
    offs = np.concatenate([[0], np.cumsum(nevt)[:-1]])
    ids = [None] * len(nevt)
    lat = np.zeros(len(nevt))
    srv = hme.Server(card, precision, hbm_budget_bytes=budget, nstreams=nstreams)
    try:
        t0 = time.perf_counter()

        def submitter():
            for k in range(len(nevt)):
                delay = t0 + arrival[k] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                ids[k] = srv.submit_ptr(int(procs[k]), 0.118, int(nevt[k]), pools[int(procs[k])].data_ptr(),
                                        out.data_ptr() + 8 * int(offs[k]))

        th = threading.Thread(target=submitter)
        th.start()
        for k in range(len(nevt)):
            while ids[k] is None:
                time.sleep(0.0002)
            lat[k] = srv.wait(ids[k])
        th.join()
        wall = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    timed = lat[nwarm:]
    span = arrival[-1] - arrival[nwarm]
    by_proc = {}
    for p in procs_avail:
        sel = procs[nwarm:] == p
        if sel.any():
            by_proc[hme.PROCESS_NAMES[p]] = {"requests": int(sel.sum()),
                                             "p50_ms": float(np.median(timed[sel]) * 1e3),
                                             "p99_ms": float(np.quantile(timed[sel], 0.99) * 1e3),
                                             "max_ms": float(timed[sel].max() * 1e3)}
    return {"p50_ms": float(np.median(timed) * 1e3), "p99_ms": float(np.quantile(timed, 0.99) * 1e3),
            "by_process": by_proc,
            "mean_ms": float(timed.mean() * 1e3), "max_ms": float(timed.max() * 1e3),
            "requests": int(ntimed), "warmup_requests": int(nwarm),
            "offered_events_per_s": float(nevt[nwarm:].sum() / span), "offered_requests_per_s": float(ntimed / span),
            "wall_s": wall, "batches": int(st["batches"]), "graphs": int(st["graphs"]),
            "precision": hme.PRECISION_NAMES[precision], "hbm_budget_bytes": budget, "streams": nstreams,
            "processes": "gg->ttbar, gg->ttbar g, gg->ttbar gg, gg->ttbar ggg (uniform)",
            "offered_events_per_s_by_process": {
                hme.PROCESS_NAMES[q]: float(nevt[nwarm:][procs[nwarm:] == q].sum() / span) for q in procs_avail}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nevt", type=int, default=None, help="override the batch size (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-ggttggg", action="store_true")
    ap.add_argument("--no-e2e", action="store_true")
    ap.add_argument("--no-select", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the C1-C3 and Drell-Yan legs")
    ap.add_argument("--pmc", action="store_true",
                    help="counter-collection mode: one FP64 and one MIXED_FAST gg->ttbar gg launch, one "
                         "8192-event gg->ttbar ggg call, then a plain 256 MiB device copy and a 256 MiB "
                         "read-only sum (known traffic, for calibrating FETCH_SIZE / WRITE_SIZE); no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); events are independent and "
              "shard without communication, see the design notes.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2507_21039_amd as hme
    from workloads import configs

    w = configs.WORKLOADS["ggttgg"]
    nevt = args.nevt or w.nevt
    card = configs.card_array()
    log(f"[bench] generating {nevt} RAMBO events ({w.name})")
    p = w.momenta(nevt)
    mom = torch.from_numpy(p).cuda()
    out = torch.empty(nevt, dtype=torch.float64, device="cuda")
    if args.pmc:
        # one launch of each kernel whose counters are quoted, then a copy of known size
        with hme.Handle(hme.GGTTGG, card, hme.FP64) as h:
            h.compute(mom, out)
        with hme.Handle(hme.GGTTGG, card, hme.MIXED_FAST) as h:
            h.compute(mom, out)
        w7 = configs.WORKLOADS["ggttggg"]
        mom7 = torch.from_numpy(w7.momenta(8192)).cuda()
        with hme.Handle(hme.GGTTGGG, card, hme.MIXED_FAST) as h:
            h.compute(mom7)
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        # read-only calibration: a reduction reads the 256 MiB once and writes a few bytes
        total = src.sum()
        torch.cuda.synchronize()
        log(f"[bench] pmc mode: FP64 and MIXED_FAST gg->ttbar gg launches, one 8192-event gg->ttbar ggg "
            f"call, 256 MiB copy, 256 MiB read-only sum ({float(total):.0f}) done")
        return
    results = {}
    for prec, name in ((hme.FP64, "fp64"), (hme.MIXED_FAST, "mixed_fast"), (hme.MIXED_PAPER, "mixed_paper")):
        log(f"[bench] {name}: create")
        h = hme.Handle(hme.GGTTGG, card, prec)
        info = h.query()
        log(f"[bench] {name}: {args.warmup} warmup + {args.steps} timed steps")
        gpu_s, wall_s = time_steps(h, mom, out, args.steps, args.warmup)
        per_launch = gpu_s / args.steps
        flops = info["flops_per_event"] * nevt
        results[name] = dict(value=nevt * args.steps / gpu_s, ms_per_step=per_launch * 1e3, wall_s=wall_s,
                             flops_per_event=info["flops_per_event"], ngoodhel=info["ngoodhel"],
                             achieved_tflops=flops / per_launch / 1e12, out=out.cpu().numpy().copy())
        h.close()
        log(f"[bench] {name}: {results[name]['value']:.4g} events/s, {per_launch * 1e3:.3f} ms/step")

    # the Feynman-diagram gauge variant of the same workload (gauge invariant |M|^2, fewer
    # cancellations between diagrams in single precision)
    fd = {}
    for prec, name in ((hme.FP64, "fp64"), (hme.MIXED_FAST, "mixed_fast")):
        with hme.Handle(hme.GGTTGG, card, prec | hme.GAUGE_FD) as h:
            gpu_s, _ = time_steps(h, mom, out, args.steps, args.warmup)
        per = gpu_s / args.steps
        rel = np.abs(out.cpu().numpy() / results["fp64"]["out"] - 1)
        fd[name] = {"value": nevt / per, "ms_per_step": per * 1e3, "max_rel_diff_vs_fp64": float(rel.max()),
                    "p99_rel_diff_vs_fp64": float(np.quantile(rel, 0.99)),
                    "median_rel_diff_vs_fp64": float(np.median(rel))}
        log(f"[bench] fd gauge {name}: {nevt / per:.4g} events/s, max rel diff vs fp64 {rel.max():.3g}")

    f64 = results["fp64"]
    achieved = f64["flops_per_event"] * nevt / (f64["ms_per_step"] / 1e3)
    cf = counter_flops("fp64", nevt)
    counter_achieved = cf / (f64["ms_per_step"] / 1e3) if cf else None
    cf_fast = counter_flops("mixed_fast", nevt)
    mf_fast = counter_mfma_flops("mixed_fast", nevt)
    line = {
        "metric": METRIC,
        "value": f64["value"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"gg->ttbar gg, {nevt} RAMBO events at sqrt(s)=2 TeV, dR(g,g)>0.4, seed 4, "
                               f"alpha_s=0.118, mt=173 GeV",
                   "process": "gg->ttbar gg", "nevt": nevt, "diagrams": 123, "helicities": 64,
                   "good_helicities": f64["ngoodhel"], "colour_flows": 24},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": measured_traffic(nevt),
                     "traffic_unit": "bytes per launch (HBM: L2 read requests by size + WRITE_SIZE)",
                     "algorithmic_bytes": 200 * nevt, "flops_per_event": f64["flops_per_event"],
                     "flops_note": "generator's static count: every call once, jamp additions, colour sum as "
                                   "4 ncol^2 (dense), per-event table",
                     "frac_symmetric_colour": (f64["flops_per_event"] - f64["ngoodhel"] * colour_dense_excess("ggttgg"))
                                              * nevt / (f64["ms_per_step"] / 1e3) / PEAK_FP64_VALU,
                     "counter_achieved": counter_achieved / 1e12 if counter_achieved else None,
                     "counter_frac": counter_achieved / PEAK_FP64_VALU if counter_achieved else None,
                     "counter_note": "executed FLOPs from SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64, recomputed "
                                     "wavefunctions included"},
        "mixed": {
            name: {"value": results[name]["value"], "ms_per_step": results[name]["ms_per_step"], "dtype": dt,
                   "achieved_tflops": results[name]["achieved_tflops"],
                   "frac_of_valu_peak": results[name]["achieved_tflops"] * 1e12 / peak,
                   "valu_peak_tflops": peak / 1e12,
                   "counter_achieved_tflops": (cf_fast / (results[name]["ms_per_step"] / 1e3) / 1e12
                                               if name == "mixed_fast" and cf_fast else None),
                   "counter_mfma_tflops": (mf_fast / (results[name]["ms_per_step"] / 1e3) / 1e12
                                           if name == "mixed_fast" and mf_fast else None),
                   "max_rel_diff_vs_fp64": float(np.max(np.abs(results[name]["out"] / f64["out"] - 1))),
                   "p99_rel_diff_vs_fp64": float(np.quantile(np.abs(results[name]["out"] / f64["out"] - 1), 0.99))}
            for name, dt, peak in (
                ("mixed_fast", "f32 vertices/propagators/jamps, bf16x3-split MFMA colour sum with f32 accumulation, "
                           "f64 externals and sums", PEAK_FP32_VALU),
                ("mixed_paper", "f64 amplitudes and jamps, f32 colour algebra, f64 sums", PEAK_FP64_VALU))},
        "fd_gauge": fd,
        "configs": None,
        "ggttggg": None,
        "e2e": None,
        "select": None,
        "served": None,
    }
    if not args.no_configs:
        log("[bench] other configurations (C1-C3, Drell-Yan)")
        line["configs"] = configs_leg(card, cpu=not args.no_cpu_baseline)
    if not args.no_ggttggg:
        log("[bench] gg->ttbar ggg (mixed fast)")
        line["ggttggg"] = ggttggg_leg(card)
        log(f"[bench] gg->ttbar ggg: {line['ggttggg']['value']:.4g} events/s")
    if not args.no_e2e:
        log("[bench] end-to-end flat Monte Carlo (device RAMBO + FP64 |M|^2 + sum)")
        line["e2e"] = e2e_leg(card)
        log(f"[bench] e2e: {line['e2e']['value']:.4g} events/s, rambo {line['e2e']['ms_rambo']:.3f} ms")
        log("[bench] host buffers (pinned H2D, FP64 |M|^2, D2H)")
        line["e2e"]["host_buffers"] = pcie_leg(card, p)
        log(f"[bench] host buffers: {line['e2e']['host_buffers']['value']:.4g} events/s, "
            f"H2D {line['e2e']['host_buffers']['h2d_gbps']:.1f} GB/s")
    if not args.no_select:
        log("[bench] helicity and colour-flow choice")
        line["select"] = select_leg(card)
        log(f"[bench] select overhead: " + ", ".join(f"{k} {v['overhead'] * 100:.2f}%"
                                                     for k, v in line["select"].items()))
        log(f"[bench] channel weights overhead (gg->ttbar gg): {line['select']['ggttgg']['overhead_channels'] * 100:.2f}%")
    if not args.no_served:
        log("[bench] served mix (Poisson, 200 requests/s)")
        line["served"] = served_leg(card, hme.MIXED_FAST)
        log(f"[bench] served p50 {line['served']['p50_ms']:.3f} ms p99 {line['served']['p99_ms']:.3f} ms")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(configs.GGTTGG, p, f64["out"], card)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
