"""Benchmark: PARAFAC2-ALS iterations per second on one MI355X.

One step is one full ALS iteration (Procrustes step, three MTTKRPs with the
H, V and W updates, fit) over the whole synthetic input, with the input and
the state resident in HBM.  Default workload: K = 1,000,000 subjects,
J = 5000, R = 10, I_k in [10, 100], 1 + Poisson(0.145) nonzeros per row at
Zipf(1.1) columns (about 63M nonzeros), float32 values.

Prints one JSON line.  The dominant kernel's roofline is computed from HIP
events recorded inside the library around each launch during the timed
region; the CPU baseline is the FP64 oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4, 5],
                   help="1-3 one decomposition; 4 the 64-problem batch; 5 the serving trace")
    p.add_argument("--k-limit", type=int, default=None, help="only the first K subjects")
    p.add_argument("--cpu-subjects", type=int, default=-1,
                   help="subjects in the oracle's timed sample (0 = skip; default: about 12 s "
                        "of oracle work, 60,000 subjects at R=10 and 6,000 at R=40)")
    p.add_argument("--profile-only", action="store_true",
                   help="skip the CPU baseline (for profiler runs)")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the default launch schedule instead of autotuning it")
    p.add_argument("--serve-seconds", type=float, default=10.0,
                   help="measured seconds of the serving trace (after 1 s of warm-up)")
    p.add_argument("--copy-bytes", type=int, default=0,
                   help="only run a plain device-to-device copy of this many bytes (calibrates "
                        "the profiler's FETCH_SIZE / WRITE_SIZE counters) and exit")
    return p.parse_args()


def copy_rate_gbps(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Achievable HBM rate on this device: a plain device-to-device copy of
    nbytes, timed with events (read + write bytes over the best launch)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (best * 1e-3) / 1e9


def copy_calibration(nbytes: int):
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "launches": 3}), flush=True)


KERNEL_SOURCES = ("paper_1703_04219_amd/csrc/p2_kernels.hip", "paper_1703_04219_amd/csrc/p2_device.h",
                  "paper_1703_04219_amd/csrc/p2_batch.h")


def kernel_source_hash() -> str:
    """Hash of the kernel sources: counter readings taken on other sources
    no longer describe the kernels that run."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stream_bytes(X, R: int) -> dict:
    """Algorithmic HBM bytes of one pass over the re-encoded slices and the
    per-subject state, as used by the per-iteration kernels."""
    K, n_rows, nnz = X.K, X.n_rows, X.nnz
    x = nnz * (2 + 4) + n_rows * 2 + (K + 1) * 16  # col16 + val, row starts, offsets
    f = K * R * R * 8                              # F_k (float64 R x R)
    w = K * R * 4
    return {"x": x, "f": f, "w": w}


def algorithmic_bytes(X, R: int) -> dict:
    """Algorithmic HBM bytes of one launch of each per-iteration kernel."""
    sb = stream_bytes(X, R)
    LDV = (R + 3) & ~3
    v_bytes = X.J * LDV * 4
    return {
        # k_gamma: X once, F read + F write (next Procrustes step), W and M3 written, V_t, V_{t+1}
        "gamma": sb["x"] + 2 * sb["f"] + 2 * sb["w"] + 2 * v_bytes,
        # k_mode2: X once, F and W read, V_t, M2 written
        "mode2": sb["x"] + sb["f"] + sb["w"] + 2 * v_bytes,
        "alpha": sb["x"] + sb["f"] + sb["w"] + v_bytes,
    }


def cpu_baseline(cfg: int, n_subjects: int):
    from threadpoolctl import threadpool_limits

    from datagen import gen_config, gen_init
    from oracle import parafac2_oracle as O
    X, R = gen_config(cfg, k_limit=n_subjects)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, cfg, 1])
    Xs = O.slices_to_list(X.subj_ptr, X.row_ptr, X.col, X.val, X.J)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.iterate(Xs, H0, V0, W0, dense_loss=False)
        dt = time.perf_counter() - t0
    return {"value": X.nnz / dt, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"first {X.K} subjects of the workload ({X.nnz} nnz), one ALS iteration, "
                      f"FP64 NumPy/LAPACK, one thread, {dt:.1f} s"}


def _request(X, k):
    r0, r1 = int(X.subj_ptr[k]), int(X.subj_ptr[k + 1])
    rp = X.row_ptr[r0:r1 + 1]
    z0, z1 = int(rp[0]), int(rp[-1])
    return (np.ascontiguousarray(rp - rp[0]), np.ascontiguousarray(X.col[z0:z1]),
            np.ascontiguousarray(X.val[z0:z1]))


def replay(server, t, reqs, stop_after: float):
    """Replay arrival times t (seconds) against the server in real time;
    returns each request's completion time (nan if not done by stop_after)."""
    n = len(t)
    done = np.full(n, np.nan)
    i, ndone = 0, 0
    t0 = time.perf_counter()
    while ndone < n:
        now = time.perf_counter() - t0
        if now > stop_after:
            break
        while i < n and t[i] <= now:
            if server.submit(i, *reqs[i]) != 0:
                break  # queue full: the request waits on the client side
            i += 1
        ids, _, _ = server.poll()
        if len(ids):
            done[ids] = time.perf_counter() - t0
            ndone += len(ids)
    return done


def serving(a) -> dict:
    import torch

    from datagen.synth import gen_serving_model, gen_serving_requests
    from paper_1703_04219_amd import binding as B
    warm, dur, rate = 1.0, a.serve_seconds, 2000.0
    V, H = gen_serving_model()
    t, X = gen_serving_requests(int((warm + dur) * rate))
    reqs = [_request(X, k) for k in range(X.K)]
    nnz_req = X.nnz / X.K
    torch.cuda.set_device(0)
    model = B.Model(V, H)
    out = {}
    for name, kw in (("continuous", dict(slots=4, max_requests=512)),
                     ("one_at_a_time", dict(slots=1, max_requests=1))):
        server = B.Server(model, **kw)
        for k in range(64):  # warm the kernels and the staging buffers
            server.submit(k, *reqs[k])
        server.drain()
        server.poll()
        # idle latency: one request at a time on an empty server
        idle = []
        for k in range(20):
            t1 = time.perf_counter()
            server.submit(k, *reqs[k])
            server.drain()
            server.poll()
            idle.append((time.perf_counter() - t1) * 1e3)
        # saturation: a backlog of 1000 requests (500 for the plain path) drained
        nb = 1000 if kw["max_requests"] > 1 else 200
        t1 = time.perf_counter()
        for k in range(nb):
            server.submit(k, *reqs[k])
        server.drain()
        server.poll()
        sat = nb / (time.perf_counter() - t1)
        # the Poisson trace: 1 s of warm-up arrivals, then the measured window
        span = dur if kw["max_requests"] > 1 else min(dur, 2.0)
        m = int(np.searchsorted(t, warm + span))
        done = replay(server, t[:m], reqs[:m], stop_after=warm + span + 5.0)
        server.drain()
        lat = done - t[:m]
        sel = t[:m] >= warm
        ok = np.isfinite(lat) & sel
        lat_ms = lat[ok] * 1e3
        span_s = float(np.nanmax(done[sel]) - warm) if ok.any() else float("nan")
        out[name] = {"p50_ms": float(np.percentile(lat_ms, 50)) if ok.any() else None,
                     "p99_ms": float(np.percentile(lat_ms, 99)) if ok.any() else None,
                     "completed": int(ok.sum()), "offered": int(sel.sum()),
                     "throughput_req_s": float(ok.sum() / span_s) if ok.any() else 0.0,
                     "measured_s": span,
                     "idle_latency_ms_p50": float(np.median(idle)),
                     "saturation_req_s": float(sat), "server": kw}
        print(f"[bench] serving {name}: {out[name]}", file=sys.stderr, flush=True)
        server.close()
    out["rate_req_s"] = rate
    out["nnz_per_request"] = round(nnz_req, 1)
    out["R"] = int(V.shape[1])
    return out


def batched(a):
    import concurrent.futures as cf
    import multiprocessing as mp

    from datagen.synth import gen_batched_problem, gen_batched_specs
    from datagen import gen_init
    specs = gen_batched_specs()
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1),
                                mp_context=mp.get_context("fork")) as ex:
        Xs = list(ex.map(gen_batched_problem, specs))
    nnz = sum(X.nnz for X in Xs)
    print(f"[bench] generated 64 problems, {nnz} nnz, in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    import torch

    from paper_1703_04219_amd import binding as B
    torch.cuda.set_device(0)
    ctxs = []
    for i, (sp, X) in enumerate(zip(specs, Xs)):
        H0, V0, W0 = gen_init(X.J, X.K, sp["R"], [170304219, 4, 1, i])
        ctxs.append(B.Context(B.DeviceSlices.from_slices(X), sp["R"], H0, V0, W0))
    del Xs
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # one problem at a time (each context runs its own launches)
    for c in ctxs:
        c.iterate(a.warmup, with_fit=False)
    torch.cuda.synchronize()
    e0.record()
    for c in ctxs:
        c.iterate(a.steps, with_fit=False)
    e1.record()
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / a.steps
    # the batch: one launch per rank class and kernel, autotuned schedule
    batch = B.Batch(ctxs, B.make_sched(graph=1))
    chosen, tuned_ms = (None, None) if a.no_autotune else batch.autotune(2)
    batch.iterate(a.warmup, with_fit=False)
    torch.cuda.synchronize()
    e0.record()
    batch.iterate(a.steps, with_fit=False)
    e1.record()
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1) / a.steps
    fits = batch.iterate(1)[0]
    print(f"[bench] batched {ms_batch:.3f} ms/iteration vs one problem at a time "
          f"{ms_single:.3f} ms; schedule {chosen.as_dict() if chosen else 'default'}",
          file=sys.stderr, flush=True)
    out = {
        "metric": "ALS-iteration nnz/s & % HBM roofline at R=10/40; p50/p99 projection latency",
        "value": nnz / (ms_batch * 1e-3), "unit": "nnz/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_batch, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 sparse products, f64 RxR", "data": "synthetic",
        "config": {"workload": "c4_batched_64_problems", "problems": len(ctxs), "nnz": nnz,
                   "K_total": int(sum(c.X.K for c in ctxs)),
                   "ranks": {str(r): sum(1 for sp in specs if sp["R"] == r) for r in (5, 10, 20)},
                   "one_problem_at_a_time_ms": ms_single,
                   "one_problem_at_a_time_nnz_s": nnz / (ms_single * 1e-3),
                   "speedup_vs_one_at_a_time": ms_single / ms_batch,
                   "schedule": chosen.as_dict() if chosen else None,
                   "autotune_ms_per_iteration": tuned_ms,
                   "min_fit_after": float(np.min(fits))},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.copy_bytes:
        copy_calibration(a.copy_bytes)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU "
              "subject-sharded design is described but not built.", file=sys.stderr)
        sys.exit(2)
    if a.config == 4:
        batched(a)
        return
    if a.config == 5:
        res = serving(a)
        c = res["continuous"]
        print(json.dumps({
            "metric": "ALS-iteration nnz/s & % HBM roofline at R=10/40; p50/p99 projection latency",
            "value": c["p99_ms"], "unit": "ms (p99 latency)", "n_gpus": 1, "steps": c["completed"],
            "warmup": 1, "ms_per_step": c["p50_ms"], "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32 gather, f64 RxR",
            "data": "synthetic", "config": {"workload": "c5_serving_2000req_s", **res},
            "roofline": None, "cpu_baseline": None}), flush=True)
        return
    import torch

    from datagen import CONFIGS, gen_config, gen_init
    from paper_1703_04219_amd import binding as B

    # draw the input before the GPU runtime starts (the generator forks workers)
    t0 = time.perf_counter()
    X, R = gen_config(a.config, k_limit=a.k_limit)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, a.config, 1])
    print(f"[bench] generated K={X.K} J={X.J} R={R} rows={X.n_rows} nnz={X.nnz} "
          f"in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    dX = B.DeviceSlices.from_slices(X)
    ctx = B.Context(dX, R, H0, V0, W0)
    del dX  # the context re-encoded the input into its workspace
    torch.cuda.synchronize()
    # device memory held from here on: the workspace (re-encoded X, per-subject
    # state, partial sums) and the factors; the peak includes the input copy
    # that init reads
    footprint = {"steady_bytes": int(torch.cuda.memory_allocated()),
                 "peak_bytes": int(torch.cuda.max_memory_allocated()),
                 "workspace_bytes": int(ctx.ws_bytes)}
    print(f"[bench] init done, workspace {ctx.ws_bytes / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    chosen, tuned_ms = None, None
    if not a.no_autotune:
        chosen, tuned_ms = ctx.autotune(2)
        print(f"[bench] autotuned schedule {chosen.as_dict()} ({tuned_ms:.3f} ms/iteration)",
              file=sys.stderr, flush=True)
    if a.warmup:
        ctx.iterate(a.warmup, with_fit=False)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    ctx.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    ctx.iterate(a.steps, with_fit=False)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    prof = ctx.profile()
    ctx.set_profiling(False)
    ms_step = ms_total / a.steps
    fit = float(ctx.iterate(1)[0])
    torch.cuda.synchronize()
    print(f"[bench] {ms_step:.3f} ms/iteration, fit {fit:.6f}, phases "
          + ", ".join(f"{k}={v[0] / max(v[1], 1):.3f}ms x{v[1]}" for k, v in prof.items()),
          file=sys.stderr, flush=True)

    # dominant kernel: the per-iteration phase with the most device time
    per_launch_bytes = algorithmic_bytes(X, R)
    cand = {k: prof[k] for k in ("gamma", "mode2") if prof[k][1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    avg_ms = cand[dom][0] / cand[dom][1]
    achieved = per_launch_bytes[dom] / (avg_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_k_{dom}_c{a.config}.json")
    if os.path.exists(tfile) and a.k_limit is None:
        with open(tfile) as f:
            rec = json.load(f)
        if rec.get("source_sha256") == kernel_source_hash():
            traffic = rec.get("bytes_per_launch")
    copy_gbps = copy_rate_gbps()
    roof = {"bound": "hbm", "kernel": f"k_{dom}", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": per_launch_bytes[dom],
            "copy_GBps_measured": round(copy_gbps, 1),
            "frac_of_measured_copy": round(achieved / copy_gbps, 4)}

    cpu = None
    if a.cpu_subjects and not a.profile_only:
        print("[bench] timing the oracle on a sample ...", file=sys.stderr, flush=True)
        n_cpu = a.cpu_subjects if a.cpu_subjects > 0 else {1: X.K, 2: 60000, 3: 6000}[a.config]
        cpu = cpu_baseline(a.config, min(n_cpu, X.K))

    name = CONFIGS[a.config]["name"] + ("" if a.k_limit is None else f"_first{X.K}")
    out = {
        "metric": "ALS-iteration nnz/s & % HBM roofline at R=10/40; p50/p99 projection latency",
        "value": X.nnz / (ms_step * 1e-3),
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 sparse products, f64 RxR",
        "data": "synthetic",
        "config": {"workload": name, "K": X.K, "J": X.J, "R": R, "n_rows": X.n_rows,
                   "nnz": X.nnz, "fit_after": fit,
                   "phase_ms_per_launch": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()},
                   "schedule": chosen.as_dict() if chosen else None,
                   "hbm_footprint": footprint,
                   "paper_context": "SPARTan: 7.4 min/iteration at 63M nnz, R=10 (4x Xeon E5-4620 v4, "
                                    "NNLS-constrained, uniform sparsity)"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
