"""Benchmark: likelihood evaluations per second at 1023^2 interior nodes.

One step = the whole hot path over one batch of parameter samples resident in
HBM: Leaves to Root for every sample (leaf assembly, extend-add, interface
factorization, matrix-core Schur updates), Root to Leaves, float64
refinement of the float32 factors against the assembled operator, and the
measurements of the 1023^2 workload (64 point values, the root midline
interface, the mean over [0.25,0.5]^2) with the Gaussian log-likelihood of
the 64 observations.  value = batch * steps / timed seconds.

Prints one JSON line (see the keys below).  --gpus N > 1 exits: this build
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma": 157.3, "fp64_mfma": 78.6, "hbm_gbs": 8000.0}
# HBM traffic per launch of the roofline kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes, each scaled by what the counter reads for a 1 GiB device copy
# (profiles/k_syrk128_f32_c2_1023_b128.md), keyed (kernel, config, batch).
# An entry is removed whenever its kernel changes.
TRAFFIC = {("k_syrk128_f32", "c2_1023", 128): 4.592e9}
KIND = {"syrk32": 0, "factor": 1, "extend": 2, "block_build": 3, "topdown": 4, "forward": 5, "residual": 6,
        "syrk64": 7, "syrk128": 8, "merge": 9, "eliminate": 12}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--config", default="c2_1023")
    ap.add_argument("--precision", default="fp32_refine", choices=["fp32_refine", "fp64"])
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile-steps", type=int, default=1, help="extra steps with per-kernel event timing")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-mix measurement")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the float64 batched full / partial top-down steps reported beside the headline")
    ap.add_argument("--serve-requests", type=int, default=96, help="requests per arrival rate in the serving mix")
    ap.add_argument("--no-graph", action="store_true", help="issue every launch eagerly (no captured HIP graphs)")
    ap.add_argument("--no-autotune", action="store_true", help="built-in tile rule instead of the autotuner")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the 255^2 x 256 and 2047^2 workloads reported beside the headline")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run 3 device-to-device copies of BYTES (calibrates HBM byte counters) and exit")
    return ap.parse_args()


def copy_probe(nbytes: int):
    """Three plain device-to-device copies of nbytes: the reference dispatch
    for scaling the FETCH_SIZE / WRITE_SIZE counters (reads nbytes, writes
    nbytes per copy)."""
    import torch

    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "copies": 3}), flush=True)


def cpu_baseline(w, seconds: float):
    """The oracle on the host, one core (it is single-threaded):
    - at 1023^2 (the headline workload, sample 0), its banded-Cholesky
      factorization of the first columns of the operator, scaled to the full
      factorization by column count (every column away from the end costs the
      same); triangular solves and refinement are not included, so the figure
      favours the CPU;
    - complete oracle solves (factorization, solves, 2 extended-precision
      refinement sweeps) at 255^2 and 511^2 on the same statistics.
    value = 1023^2 evaluations/s on one core; all_cores_value = nproc x value
    (samples are independent)."""
    from oracle import oracle as O
    from workload import make_workload

    n = w.n
    ncols_total = n * n
    probe = 2000
    t = O.factor_prefix_seconds(n, w.kappa[0], probe)
    ncols = int(min(ncols_total, max(probe, probe * seconds / max(t, 1e-6))))
    t = O.factor_prefix_seconds(n, w.kappa[0], ncols)
    t_full = t * ncols_total / ncols
    full = {}
    for name in ("s_255", "s_511"):
        ws = make_workload(name, n_samples=1)
        t0 = time.perf_counter()
        O.solve(ws.n, ws.kappa[0], ws.f)
        full[f"{ws.n}^2"] = time.perf_counter() - t0
    nproc = os.cpu_count() or 1
    return {"value": 1.0 / t_full, "unit": "likelihood evals/s", "cores": 1, "kind": "oracle",
            "sample": f"banded Cholesky of the first {ncols} of {ncols_total} columns of the 1023^2 operator "
                      f"(sample 0), {t:.1f} s, scaled by column count to {t_full:.0f} s per solve; "
                      f"triangular solves and refinement (O(N^3)) not included",
            "full_solve_seconds_1core": full,
            "all_cores_value": nproc / t_full, "nproc": nproc,
            "host": platform.processor() or platform.machine()}


def serving_mix(H, n_req: int, seed: int = 7):
    """Serving mix: each request draws its mesh uniformly from 127^2, 255^2 and
    511^2 interior nodes (16x16 leaves, 20-mode log-normal kappa, corr 0.1,
    var 1) and 1-32 uniform observation sites; arrivals are Poisson at 0.5,
    0.8 and 1.0 times the saturated throughput measured first with a burst.
    Latency is submit-to-result as measured by the server.  Parameter
    samples come from a pre-drawn pool per mesh so the client stays off the
    critical path."""
    import threading

    from workload import make_workload

    names = ["s_127", "s_255", "s_511"]
    pool = {m: make_workload(m, n_samples=16) for m in names}
    srv = H.Server([pool[m].n for m in names], H.HDD_FP32_REFINE, slots=32,
                   leaves=[pool[m].leaf for m in names], f=[pool[m].f for m in names])
    rng = np.random.default_rng(seed)

    def draw():
        m = int(rng.integers(0, 3))
        w = pool[names[m]]
        xy = rng.uniform(size=(int(rng.integers(1, 33)), 2))
        return m, w.kappa[int(rng.integers(0, 16))], xy

    def run(rate):
        reqs = [draw() for _ in range(n_req)]
        # Poisson arrivals on an absolute schedule (no drift from the client)
        at = np.cumsum(rng.exponential(1.0 / rate, size=n_req)) if rate else np.zeros(n_req)
        ids = []
        t0 = time.perf_counter()
        for k, (m, kap, xy) in enumerate(reqs):
            wait = t0 + at[k] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            ids.append((srv.submit(m, kap, xy), len(xy)))
        t_sub = time.perf_counter() - t0
        lat = []
        for i, n in ids:
            _, _, tm = srv.result(i, n)
            lat.append(tm[2])
        dt = time.perf_counter() - t0
        lat = np.array(lat) * 1e3
        return {"target_rps": rate, "offered_rps": n_req / t_sub if t_sub > 0 else None,
                "throughput_rps": n_req / dt, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "requests": n_req}

    run(0)  # warm up every mesh
    burst = run(0)
    sat = burst["throughput_rps"]
    out = {"mix": "127^2/255^2/511^2 uniform, 1-32 sites, FP32+refinement", "slots_per_mesh": srv.slots,
           "saturated_rps": sat, "rates": [run(f * sat) for f in (0.5, 0.8, 1.0)], "stats": srv.stats()}
    srv.close()
    out["serve_1023"] = serving_1023(H, n_req, seed)
    return out


def serving_1023(H, n_req: int, seed: int):
    """Requests of the headline workload served one by one: each a fresh
    parameter sample at 1023^2 (32 x 32 leaves) with the 64 observation
    sites and observations; Poisson arrivals at 0.5 and 0.8 of the
    saturated rate; per-request latency is submit-to-result."""
    from workload import make_workload

    w = make_workload("c2_1023", n_samples=16)
    srv = H.Server([w.n], H.HDD_FP32_REFINE, slots=32, leaves=[w.leaf], f=[w.f])
    rng = np.random.default_rng(seed + 1)
    y = np.zeros(len(w.points))

    def run(rate, n):
        at = np.cumsum(rng.exponential(1.0 / rate, size=n)) if rate else np.zeros(n)
        ids = []
        t0 = time.perf_counter()
        for k in range(n):
            wait = t0 + at[k] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            ids.append(srv.submit(0, w.kappa[int(rng.integers(0, 16))], w.points, y, w.sigma_y))
        lat = np.array([srv.result(i, len(w.points))[2][2] for i in ids]) * 1e3
        dt = time.perf_counter() - t0
        return {"target_rps": rate, "throughput_rps": n / dt, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "requests": n}

    run(0, 32)
    sat = run(0, n_req)["throughput_rps"]
    out = {"workload": "c2_1023 requests, 64 sites each", "slots": srv.slots, "saturated_rps": sat,
           "rates": [run(f * sat, n_req) for f in (0.5, 0.8)]}
    srv.close()
    return out


def other_workloads(H, stream, steps: int):
    """Throughput of the batched 255^2 workload (256 samples, 16 points and
    the log-likelihood per sample) and of the 2047^2 high-contrast workload
    (8 samples, 128 points and the root interface per sample), float32 +
    refinement against float64, with the refined error against the float64
    path of the same batch."""
    import torch

    from workload import make_workload

    out = {}
    for name, ns in (("c1_255", 256), ("c4_2047", 8)):
        w = make_workload(name, n_samples=ns)
        dev = torch.device("cuda:0")
        kd = torch.from_numpy(w.kappa).to(dev)
        fd = torch.from_numpy(w.f).to(dev)
        yd = torch.zeros(len(w.points), dtype=torch.float64, device=dev)
        pts = torch.empty(ns * len(w.points), dtype=torch.float64, device=dev)
        ll = torch.empty(ns, dtype=torch.float64, device=dev)
        res, vals = {}, {}
        for prec, key in ((H.HDD_FP32_REFINE, "fp32_refine"), (H.HDD_FP64, "fp64")):
            t = H.HDD(H.hdd_default_opts(w.n, prec, leaf=w.leaf), ns, stream=stream)

            def step():
                t.build(kd, fd)
                t.query_points(w.points, out=pts)
                t.loglik(w.points, yd, w.sigma_y, False, out=ll)
                if w.spec["interface"]:
                    t.query_interface(0, 0)

            step()
            if prec == H.HDD_FP32_REFINE:
                t.autotune(1)
            step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            _, sw = t.error_estimate()
            vals[key] = pts.cpu().numpy().reshape(ns, -1)
            res[key] = {"value": ns / dt, "ms_per_step": 1e3 * dt, "refine_sweeps": int(np.max(sw))}
            t.close()
        ref = vals["fp64"]
        res["fp32_refine"]["max_rel_err_vs_fp64"] = float(
            max(np.abs(vals["fp32_refine"][s] - ref[s]).max() / np.abs(ref[s]).max() for s in range(ns)))
        out[name] = {"samples": ns, "unit": "likelihood evals/s", **res}
    return out


def main():
    a = parse()
    if a.copy_probe > 0:
        copy_probe(a.copy_probe)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1708_02207_amd import hdd as H
    from workload import make_workload, rhs_nodal

    w = make_workload(a.config, n_samples=a.batch)
    gold_path = os.path.join(ROOT, "tests", "golden", f"{a.config}.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None
    y = np.array(gold["y"]) if gold else np.zeros(len(w.points))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    kd = torch.from_numpy(w.kappa).to(dev)
    fd = torch.from_numpy(w.f).to(dev)
    yd = torch.from_numpy(y).to(dev)
    prec = H.HDD_FP32_REFINE if a.precision == "fp32_refine" else H.HDD_FP64
    opts = H.hdd_default_opts(w.n, prec, leaf=w.leaf, flags=H.HDD_FLAG_NO_GRAPH if a.no_graph else 0)
    t = H.HDD(opts, a.batch, stream=stream)
    B = a.batch
    ll = torch.empty(B, dtype=torch.float64, device=dev)
    pts = torch.empty(B * len(w.points), dtype=torch.float64, device=dev)
    iface = torch.empty(B * w.n, dtype=torch.float64, device=dev)
    mean = torch.empty(B, dtype=torch.float64, device=dev)
    rect = np.array(w.mean_rect if w.mean_rect else (0.25, 0.5, 0.25, 0.5))

    def step():
        t.build(kd, fd)
        t.loglik(w.points, yd, w.sigma_y, False, out=ll)
        t.query_points(w.points, out=pts)
        H._check(H._lib.hdd_query_interface(t.h, 0, 0, H.ctypes.c_void_p(iface.data_ptr()), None, H.HDD_MEM_DEVICE),
                 "hdd_query_interface")
        H._check(H._lib.hdd_query_mean(t.h, H._np_ptr(rect), H.ctypes.c_void_p(mean.data_ptr()), H.HDD_MEM_DEVICE),
                 "hdd_query_mean")

    step()
    # per-level tile choices of the Schur updates, timed on this GPU
    tiles = None if a.no_autotune else t.autotune(1).tolist()
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    code = t.sync()
    est, sweeps = t.error_estimate()
    graphs = t.graph_info()

    # accuracy of this run's outputs against the stored oracle values
    err = None
    if gold:
        P = pts.cpu().numpy().reshape(B, -1)
        I = iface.cpu().numpy().reshape(B, -1)
        M = mean.cpu().numpy()
        errs = []
        for g in gold["samples"]:
            s = g["sample"]
            if s >= B:
                continue
            r = lambda v, ref: float(np.abs(np.asarray(v) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())
            errs.append(r(P[s], g["points"]))
            if "interface" in g:
                errs.append(r(I[s], g["interface"]))
            if "mean" in g:
                errs.append(r([M[s]], [g["mean"]]))
        err = max(errs) if errs else None

    # per-kernel event timing over extra profiled steps
    t.timing_enable(sum(1 << k for k in KIND.values()))
    for _ in range(a.profile_steps):
        step()
    kern = {}
    for name, k in KIND.items():
        ms, n, fl, by = t.timing_get(k, with_bytes=True)
        ps = max(a.profile_steps, 1)
        kern[name] = {"ms": ms / ps, "launches": n // ps, "flops": fl / ps, "bytes": by / ps,
                      "tflops": (fl / (ms * 1e-3) / 1e12) if ms > 0 and fl > 0 else None}
    t.timing_enable(0)
    # dominant kernel: the 128 x 128-tile float32 Schur update (FP32 path) or
    # the float64 Schur update (FP64 path); algorithmic flops = 2 K per
    # lower-triangle output element of every launch
    syrk_key = "syrk128" if prec == H.HDD_FP32_REFINE else "syrk64"
    kname = "k_syrk128_f32" if syrk_key == "syrk128" else "k_syrk_mfma_f64"
    peak = PEAK["fp32_mfma"] if syrk_key == "syrk128" else PEAK["fp64_mfma"]
    ach = kern[syrk_key]["tflops"] or 0.0
    nl = max(kern[syrk_key]["launches"], 1)
    roofline = {"bound": "mfma", "kernel": kname, "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": TRAFFIC.get((kname, a.config, a.batch)),
                "launches_per_step": kern[syrk_key]["launches"],
                "avg_launch_ms": kern[syrk_key]["ms"] / nl,
                "algorithmic_flops_per_launch": kern[syrk_key]["flops"] / nl,
                "algorithmic_bytes_per_launch": kern[syrk_key]["bytes"] / nl}
    # Further right-hand sides on the headline handle's operators: a bump load
    # with boundary data u = x + y, through the forward pass, a full top-down
    # and the refinement sweeps (hdd_solve_rhs), against the full step.
    multi_rhs = None
    if not a.no_ablation:
        nc1 = w.n + 2
        xg = np.arange(nc1) / (w.n + 1)
        fb = torch.from_numpy(rhs_nodal(w.n, "bump")).to(dev)
        gb = torch.from_numpy(np.add.outer(xg, xg)).to(dev)
        t.build(kd, fd)
        torch.cuda.synchronize()
        reps, tot = 3, 0.0
        for r in range(reps + 1):
            t0 = time.perf_counter()
            t.solve_rhs(fb, gb)
            torch.cuda.synchronize()
            if r > 0:
                tot += time.perf_counter() - t0
        _, rhs_sweeps = t.error_estimate()
        multi_rhs = {"samples": B, "ms_per_rhs": 1e3 * tot / reps, "sweeps": rhs_sweeps,
                     "build_and_queries_ms": 1e3 * dt / a.steps,
                     "note": "full field of every sample for a new load and Dirichlet data on the built operators"}

    # Two batches in flight: a second handle on its own stream, each driven
    # by a host thread (the library calls release the interpreter), so one
    # batch's latency-bound top levels and host-side stopping tests overlap
    # the other batch's work.  Throughput of the pair; latency per batch.
    concurrent = None
    if not a.no_ablation and prec == H.HDD_FP32_REFINE:
        import threading

        s2 = torch.cuda.Stream()
        t2 = H.HDD(opts, a.batch, stream=s2)
        ll2 = torch.empty(B, dtype=torch.float64, device=dev)
        pts2 = torch.empty(B * len(w.points), dtype=torch.float64, device=dev)
        iface2 = torch.empty(B * w.n, dtype=torch.float64, device=dev)
        mean2 = torch.empty(B, dtype=torch.float64, device=dev)

        def step2():
            t2.build(kd, fd)
            t2.loglik(w.points, yd, w.sigma_y, False, out=ll2)
            t2.query_points(w.points, out=pts2)
            H._check(H._lib.hdd_query_interface(t2.h, 0, 0, H.ctypes.c_void_p(iface2.data_ptr()), None,
                                                H.HDD_MEM_DEVICE), "hdd_query_interface")
            H._check(H._lib.hdd_query_mean(t2.h, H._np_ptr(rect), H.ctypes.c_void_p(mean2.data_ptr()),
                                           H.HDD_MEM_DEVICE), "hdd_query_mean")

        step2()
        if tiles is not None:
            t2.autotune(1)
        step2()
        t.build(kd, fd)
        torch.cuda.synchronize()
        nc = max(2, a.steps // 2)
        lat2 = {0: [], 1: []}

        def drive(k, fn):
            for _ in range(nc):
                s0 = time.perf_counter()
                fn()
                (stream if k == 0 else s2).synchronize()
                lat2[k].append(time.perf_counter() - s0)

        c0 = time.perf_counter()
        th = [threading.Thread(target=drive, args=(0, step)), threading.Thread(target=drive, args=(1, step2))]
        for x in th:
            x.start()
        for x in th:
            x.join()
        torch.cuda.synchronize()
        cdt = time.perf_counter() - c0
        _, sw2 = t2.error_estimate()
        P2 = pts2.cpu().numpy().reshape(B, -1)
        err2 = None
        if gold:
            err2 = max(float(np.abs(P2[g["sample"]] - np.array(g["points"])).max() / np.abs(np.array(g["points"])).max())
                       for g in gold["samples"] if g["sample"] < B)
        allat = sorted(1e3 * x for x in lat2[0] + lat2[1])
        concurrent = {"batches_in_flight": 2, "value": 2 * nc * B / cdt, "unit": "likelihood evals/s",
                      "batch_latency_ms": {"p50": float(np.percentile(allat, 50)),
                                           "p99": float(np.percentile(allat, 99))},
                      "refine_sweeps": int(np.max(sw2)), "max_rel_err_vs_oracle": err2,
                      "note": "two handles of the headline batch on two streams, one host thread each"}
        t2.close()
        del t2

    t.close()
    del t

    # The same step with block low-rank copies of the wide levels' maps P
    # (H-matrix style, float32 accuracy 1e-5) applied by the refinement
    lowrank = None
    if not a.no_ablation and prec == H.HDD_FP32_REFINE:
        o_lr = H.hdd_default_opts(w.n, prec, leaf=w.leaf, flags=H.HDD_FLAG_LOWRANK)
        t = H.HDD(o_lr, a.batch, stream=stream)
        step()
        t.autotune(1)
        step()
        torch.cuda.synchronize()
        ns_lr = max(2, a.steps // 2)
        l0 = time.perf_counter()
        for _ in range(ns_lr):
            step()
        torch.cuda.synchronize()
        ldt = time.perf_counter() - l0
        info = t.lowrank_info()
        _, lr_sweeps = t.error_estimate()
        lr_err = None
        if gold:
            P = pts.cpu().numpy().reshape(B, -1)
            lr_err = max(float(np.abs(P[g["sample"]] - np.array(g["points"])).max() / np.abs(np.array(g["points"])).max())
                         for g in gold["samples"] if g["sample"] < B)
        lowrank = {"value": B * ns_lr / ldt, "ms_per_step": 1e3 * ldt / ns_lr, "refine_sweeps": lr_sweeps,
                   "max_rel_err_vs_oracle": lr_err,
                   "maps_dense_MB_per_sample": info["dense_bytes"] / 1e6,
                   "block_store_MB_per_sample": info["store_bytes"] / 1e6,
                   "rank_MB_per_sample": info["rank_bytes"] / 1e6,
                   "lowrank_blocks": info["lowrank_blocks"], "dense_blocks": info["dense_blocks"],
                   "mean_rank": info["mean_rank"]}
        t.close()
        del t

    # The same step with every level in float32 (fp64_top_levels = 0)
    all_f32 = None
    if not a.no_ablation and prec == H.HDD_FP32_REFINE:
        o32 = H.hdd_default_opts(w.n, prec, leaf=w.leaf)
        o32.fp64_top_levels = 0
        t = H.HDD(o32, a.batch, stream=stream)
        step()
        t.autotune(1)
        step()
        torch.cuda.synchronize()
        n32 = max(2, a.steps // 2)
        l0 = time.perf_counter()
        for _ in range(n32):
            step()
        torch.cuda.synchronize()
        d32 = time.perf_counter() - l0
        _, sw32 = t.error_estimate()
        err32 = None
        if gold:
            P = pts.cpu().numpy().reshape(B, -1)
            err32 = max(float(np.abs(P[g["sample"]] - np.array(g["points"])).max() / np.abs(np.array(g["points"])).max())
                        for g in gold["samples"] if g["sample"] < B)
        all_f32 = {"fp64_top_levels": 0, "value": B * n32 / d32, "ms_per_step": 1e3 * d32 / n32,
                   "refine_sweeps": int(np.max(sw32)), "max_rel_err_vs_oracle": err32}
        t.close()
        del t

    others = None if (a.no_other or a.no_ablation) else other_workloads(H, stream, max(2, a.steps // 2))

    comparator = None
    if not a.no_comparator:
        o64 = H.hdd_default_opts(w.n, H.HDD_FP64, leaf=w.leaf)
        c = H.HDD(o64, 1, stream=stream)
        k1 = kd[:1].contiguous()
        ll1 = torch.empty(1, dtype=torch.float64, device=dev)

        def cstep():
            c.build(k1, fd)
            c.solve_full()
            c.loglik(w.points, yd, w.sigma_y, False, out=ll1)

        cstep()
        torch.cuda.synchronize()
        cs = max(2, a.steps // 2)
        c0 = time.perf_counter()
        for _ in range(cs):
            cstep()
        torch.cuda.synchronize()
        cdt = time.perf_counter() - c0
        comparator = {"name": "FP64 HDD full solve, one sample at a time (build + full Root to Leaves)",
                      "value": cs / cdt, "unit": "likelihood evals/s", "ms_per_eval": 1e3 * cdt / cs}
        c.close()

    # Ablation at the same batch and outputs: float64 factors with a full
    # Root to Leaves, float64 with the partial one, and the headline step
    ablation = None
    if not a.no_ablation and prec == H.HDD_FP32_REFINE:
        ablation = []
        o64 = H.hdd_default_opts(w.n, H.HDD_FP64, leaf=w.leaf)
        for name, full in (("fp64 batched, full Root to Leaves", True), ("fp64 batched, partial Root to Leaves", False)):
            c = H.HDD(o64, B, stream=stream)

            def astep():
                c.build(kd, fd)
                if full:
                    c.solve_full()
                c.loglik(w.points, yd, w.sigma_y, False, out=ll)
                c.query_points(w.points, out=pts)
                H._check(H._lib.hdd_query_interface(c.h, 0, 0, H.ctypes.c_void_p(iface.data_ptr()), None,
                                                    H.HDD_MEM_DEVICE), "hdd_query_interface")
                H._check(H._lib.hdd_query_mean(c.h, H._np_ptr(rect), H.ctypes.c_void_p(mean.data_ptr()),
                                               H.HDD_MEM_DEVICE), "hdd_query_mean")

            astep()
            torch.cuda.synchronize()
            ns = max(2, a.steps // 2)
            a0 = time.perf_counter()
            for _ in range(ns):
                astep()
            torch.cuda.synchronize()
            adt = time.perf_counter() - a0
            ablation.append({"name": name, "value": B * ns / adt, "unit": "likelihood evals/s",
                             "ms_per_step": 1e3 * adt / ns})
            c.close()
        ablation.append({"name": "fp32 + float64 refinement batched (headline)", "value": B * a.steps / dt,
                         "unit": "likelihood evals/s", "ms_per_step": 1e3 * dt / a.steps})

    # Means over all 2 nb - 1 subdomains of the tree on the float64 batch:
    # functional propagation (bottom-up functional pass, interfaces above the
    # blocks only) against the full Root to Leaves plus the direct sum.
    node_means = None
    coarse = None
    if not a.no_ablation and prec == H.HDD_FP32_REFINE:
        o64 = H.hdd_default_opts(w.n, H.HDD_FP64, leaf=w.leaf)
        summ = H.hdd_plan_summary(o64)
        c = H.HDD(o64, B, stream=stream)
        nm = torch.empty((B, summ["nodes"]), dtype=torch.float64, device="cuda")
        route_ms = {}
        for route in ("functional", "full_field"):
            reps, tot = 3, 0.0
            for r in range(reps + 1):
                c.build(kd, fd)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if route == "full_field":
                    c.solve_full()
                c.query_node_means(out=nm)
                torch.cuda.synchronize()
                if r > 0:
                    tot += time.perf_counter() - t0
            route_ms[route] = 1e3 * tot / reps
        # u on the coarse mesh of interfaces above depth 4 (cells of 256 x 256)
        # with Root to Leaves stopped there, against the full Root to Leaves
        skel_len = sum(H.hdd_plan_level(o64, d)["nodes"] * H.hdd_plan_level(o64, d)["gam"] for d in range(4))
        skel = torch.empty((B, skel_len), dtype=torch.float64, device=dev)
        coarse = {}
        for what in ("skeleton", "full"):
            reps, tot = 3, 0.0
            for r in range(reps + 1):
                c.build(kd, fd)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if what == "full":
                    c.solve_full()
                else:
                    c.query_skeleton(4, out=skel)
                torch.cuda.synchronize()
                if r > 0:
                    tot += time.perf_counter() - t0
            coarse[what] = 1e3 * tot / reps
        c.close()
        coarse = {"depth": 4, "skeleton_nodes": int(skel.shape[1]), "skeleton_ms": coarse["skeleton"],
                  "full_root_to_leaves_ms": coarse["full"], "dtype": "f64", "samples": B,
                  "note": "u on every interface above depth 4 (Root to Leaves stopped there) against the "
                          "full Root to Leaves, float64 batch"}
        node_means = {"nodes": summ["nodes"], "samples": B, "dtype": "f64",
                      "functional_ms": route_ms["functional"], "full_field_ms": route_ms["full_field"],
                      "means_per_s": summ["nodes"] * B / (1e-3 * route_ms["functional"]),
                      "note": "ms per batch after the build; full_field = full Root to Leaves + direct sums"}

    serving = None if a.no_serve else serving_mix(H, a.serve_requests)
    cpu = None if a.no_cpu_baseline else cpu_baseline(w, a.cpu_seconds)

    lat_ms = sorted(1e3 * x for x in lat)
    out = {
        "metric": "likelihood evals/s at 1023^2 (HDD vs full GPU solve) at 1e-8 rel err; p50/p99 ms",
        "value": B * a.steps / dt,
        "unit": "likelihood evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == H.HDD_FP32_REFINE else "f64",
        "data": "synthetic (seeded log-normal kappa, no dataset)",
        "config": {"workload": f"{a.config}: {w.n}^2 interior nodes, {w.leaf}x{w.leaf} leaves, log-normal kappa "
                               f"(var {w.spec['var']}, corr {w.spec['corr']}, {w.spec['n_z']} modes), f=1; "
                               f"64 points + midline + mean[0.25,0.5]^2 + loglik",
                   "global_batch": B, "precision": a.precision, "fp64_top_levels": int(opts.fp64_top_levels),
                   "parallelism": "1 GPU"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "note": "per step (a batch of evaluations)"},
        "accuracy": {"max_rel_err_vs_oracle": err, "refine_sweeps": sweeps,
                     "max_refine_estimate": float(np.max(est)) if len(est) else None, "status": H.strerror(code)},
        "roofline": roofline,
        "launches": {"build_graph_nodes": graphs["build_nodes"], "solve_graph_nodes": graphs["solve_nodes"],
                     "sweep_graph_nodes": graphs["sweep_nodes"], "graph_launches_per_step":
                         graphs["launches"] / max(1, a.steps + a.warmup + 1),
                     "note": "kernel launches per step = build + solve + sweeps x sweep graph nodes, "
                             "replayed from captured HIP graphs"},
        "autotune_tiles": tiles,
        "lowrank": lowrank,
        "all_float32": all_f32,
        "concurrent_batches": concurrent,
        "other_workloads": others,
        "ablation": ablation,
        "node_means": node_means,
        "coarse_mesh": coarse,
        "multi_rhs": multi_rhs,
        "kernels_ms_per_step": {k: v["ms"] for k, v in kern.items()},
        "kernels_tflops": {k: v["tflops"] for k, v in kern.items() if v["tflops"]},
        "comparator": comparator,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
