"""Benchmark: batched TabNet inference on one MI355X (libtabnet, HIP/gfx950).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload adult108]

One step is one tabnet_forward over the whole batch of the workload: every decision step
of the hot path (input BN, feature-transformer passes, attentive transformer with the
prior, sparsemax, prior update, decision and mask aggregation, final map), with logits,
the aggregate mask and all per-step masks written to HBM.  Inputs are seeded synthetic
rows shaped like the paper's Adult table (Sec. IV-A), resident in HBM before timing.

The JSON line reports BF16 rows/s as `value`, the plain FP32 path and the reduced-precision
paths (FP8, INT8, MX) on the same GPU beside it, the roofline of the fused kernel
(algorithmic bytes per launch over the event-timed launch duration), the 200-feature model
at 1,048,576 rows in FP32, BF16 and FP8, the serving legs (step masks returned, a stated
p99 bound, per-model figures for the mixed load), and the FP64 CPU oracle timed on a
bounded sample on the host's cores (one process per core).

Before the W warm-up launches the GPU is brought to its steady clock by repeating the same
forward for a fixed time (the first launches on an idle GPU run several percent slower);
the ramp is reported in the line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
BF16_PEAK_TFLOPS = 2500.0      # dense
FP8_PEAK_TFLOPS = 5000.0       # dense
FP32_MFMA_PEAK_TFLOPS = 157.3
SERVE_P99_BOUND_MS = 10.0      # stated p99 bound of the single-model serving load (step masks on)
CLOCK_RAMP_S = 0.3
# The paper's own figures (Tables I and II): end-to-end serverless invocations of a small
# TabNet (n_d = n_a = 8, 3 steps) through an HTTP gateway, on the hardware it names.  They
# count invocation overhead, not kernel work: context beside the line, never vs_baseline.
PAPER_CONTEXT = {
    "source": "arXiv 2510.19689, Tables I and II",
    "gpu": {"hardware": "NVIDIA T4 16 GB", "batch_rows": 1000, "throughput_samples_per_s": 4565.8,
            "p99_latency_ms": 11.4, "what": "serverless invocations (PyTorch on OpenFaaS)"},
    "cpu": {"hardware": "8 CPU cores", "batch_rows": 1000, "throughput_samples_per_s": 387.2,
            "latency_ms": 258.4},
}


KERNEL_SOURCES = ("paper_2510_19689_amd/csrc/tabnet_kernel.hip", "paper_2510_19689_amd/csrc/tabnet_kernel.hpp")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(name: str):
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE + WRITE_SIZE, each scaled by
    its reading for a plain device copy), from the committed profile summary; None when
    the summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"tabnet_forward_bf16_{name}_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.strip().strip("-* `")
            if ":" in line and line.startswith(("kernel_source_sha256", "traffic_bytes_per_launch")):
                k, v = line.split(":", 1)
                vals[k.strip("` ")] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic(cfg, rows: int, with_steps: bool = True):
    """Bytes and FLOPs of one forward: X read once; logits, masks_agg and (optionally) the
    per-step masks written once (FP32).  FLOPs are 2 x MACs of the unpadded GEMMs."""
    D, N, n_d, n_a, S = cfg.D, cfg.n_d + cfg.n_a, cfg.n_d, cfg.n_a, cfg.n_steps
    byt = 4 * (D + cfg.n_out + D + (S * D if with_steps else 0))
    k_first = D
    macs_pass = k_first * 2 * N + (cfg.n_shared + cfg.n_indep - 1) * N * 2 * N
    macs = (S + 1) * macs_pass + S * n_a * D + n_d * cfg.n_out
    return byt * rows, 2 * macs * rows


def clock_ramp(model, X, outs, seconds: float) -> int:
    """Repeat the forward for `seconds` (untimed) so that the GPU runs at its steady clock;
    returns the number of launches."""
    import torch
    lo, ag, ms = outs
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            model.forward_into(X, lo, ag, ms)
        n += 10
        torch.cuda.synchronize()
    return n


def time_forward(model, X, outs, steps: int, warmup: int):
    import torch
    lo, ag, ms = outs
    for _ in range(warmup):
        model.forward_into(X, lo, ag, ms)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        model.forward_into(X, lo, ag, ms)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def forward_detail(model, X, outs, n: int = 200, per_graph: int = 20):
    """Per-launch spread and two variants of the same BF16 forward: p10/p50/p90 of the
    interval between events recorded around each of n back-to-back launches; the time per
    launch without step masks; and the time per launch when per_graph launches are
    captured in one HIP graph and replayed (no per-launch host work)."""
    import numpy as np
    import torch
    lo, ag, ms = outs
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    ev[0].record(stream)
    for i in range(n):
        model.forward_into(X, lo, ag, ms)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    dts = np.array([ev[i].elapsed_time(ev[i + 1]) * 1e3 for i in range(n)])
    t_nomask, _ = time_forward(model, X, (lo, ag, None), n, 10)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        model.forward_into(X, lo, ag, ms)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            model.forward_into(X, lo, ag, ms)
    g.replay()
    torch.cuda.synchronize()
    reps = max(1, n // per_graph)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    t_graph = e0.elapsed_time(e1) / 1e3 / (reps * per_graph)
    return {"p10_us": float(np.percentile(dts, 10)), "p50_us": float(np.percentile(dts, 50)),
            "p90_us": float(np.percentile(dts, 90)), "no_step_masks_us": t_nomask / n * 1e6,
            "graph_replay_us": t_graph * 1e6}


def time_forward_raw(model, X_raw, outs, steps: int, warmup: int) -> float:
    """Seconds per tabnet_forward_raw launch (HIP events on the launch stream)."""
    import torch
    lo, ag, ms = outs
    for _ in range(warmup):
        model.forward_raw_into(X_raw, lo, ag, ms)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        model.forward_raw_into(X_raw, lo, ag, ms)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def time_mask_stats(masks, steps: int, warmup: int, per_graph: int = 20):
    """Seconds per tabnet_mask_stats call over a device [B, D] mask matrix.  A call is two
    short kernels, shorter than a Python-level launch, so `per_graph` calls are captured in
    one HIP graph and the graph is replayed; HIP events on the replay stream time it."""
    import torch
    from paper_2510_19689_amd import tabnet
    B, D = int(masks.shape[0]), int(masks.shape[1])
    mean = torch.empty(D, dtype=torch.float64, device=masks.device)
    var = torch.empty_like(mean)
    ws = torch.empty(tabnet.mask_stats_workspace_bytes(B, D), dtype=torch.uint8, device=masks.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        tabnet.mask_stats_into(masks, mean, var, ws)      # warm the code object outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            tabnet.mask_stats_into(masks, mean, var, ws)
    reps = max(1, steps // per_graph)
    for _ in range(max(1, warmup // per_graph)):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / (reps * per_graph)


def _oracle_rows(params, X, payload):
    from oracle import tabnet as oracle
    oracle.forward(params, X)
    return X.shape[0]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(params, X, budget_s: float = 30.0):
    """The FP64 oracle on the host's cores over a bounded sample of the same rows: one
    single-threaded worker process per core (oracle.parallel), 8,192-row chunks.  A first
    pass over the batch sizes the sample to about budget_s; the rate counts the whole pool
    run (worker start-up included)."""
    import numpy as np
    from oracle import parallel
    workers = parallel.default_workers()
    t0 = time.perf_counter()
    done = sum(r for _, r in parallel.map_rows(_oracle_rows, params, X, chunk=8192, workers=workers))
    t1 = time.perf_counter() - t0
    passes = max(1, int(budget_s / max(t1, 1e-3)))
    Xs = np.tile(X, (passes, 1)) if passes > 1 else X
    t0 = time.perf_counter()
    done = sum(r for _, r in parallel.map_rows(_oracle_rows, params, Xs, chunk=8192, workers=workers))
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "rows/s", "cores": workers, "kind": "oracle",
            "cpu": cpu_model(), "affinity_cores": len(os.sched_getaffinity(0)),
            "sample": f"{done} rows ({passes} passes over the {X.shape[0]} benchmark rows), FP64 numpy oracle, "
                      f"one single-threaded process per core ({workers}, OPENBLAS_NUM_THREADS=1), 8192-row "
                      f"chunks, {dt:.1f} s including worker start-up"}


def _ring_alloc(spans, head: int, need: int, size: int):
    """First-in-first-out ring of output space: spans holds (start, end, id) of the live
    allocations in order; returns the start of a free contiguous run or None."""
    if need > size:
        raise ValueError("request larger than the output ring")
    if not spans:
        return 0
    tail = spans[0][0]
    if head > tail or (head == tail and not spans):   # live region [tail, head) does not wrap
        if head + need <= size:
            return head
        return 0 if need <= tail else None
    return head if head + need <= tail else None      # wrapped: free run is [head, tail)


def serve_bench(models, Xpools, rates, warm_s: float, dur_s: float, step_masks: bool = False,
                max_rows: int = 4096, mix_seed=None):
    """Open-loop Poisson load against the continuous-batching server.

    Request sizes are log-uniform over 1..max_rows; arrivals and sizes come from the
    seeded request stream.  With several models each request goes to one of them, drawn
    uniformly from a seeded generator (mix_seed).  Latency is measured by the library
    from each request's scheduled arrival to the completion of its copy-out, so a late
    submission counts against the server (no coordinated omission)."""
    import collections
    import threading

    import numpy as np
    from paper_2510_19689_amd import synth, tabnet

    cfgs = [m.config for m in models]
    per_row = [c.n_out + c.D + (c.n_steps * c.D if step_masks else 0) for c in cfgs]
    RING = 1 << 26                      # floats of output space in flight (256 MiB)
    out = []
    for lam in rates:
        t_arr, rows = synth.request_stream(lam, warm_s + dur_s, seed=synth.REQUEST_SEED, max_rows=max_rows)
        pick = (np.random.default_rng(mix_seed).integers(0, len(models), size=t_arr.size)
                if len(models) > 1 else np.zeros(t_arr.size, np.int64))
        ring = np.empty(RING, np.float32)
        spans = collections.deque()      # (start, end, req_id) in submission order
        lock = threading.Condition()
        head = [0]
        done_sub = [False]
        with tabnet.Server(models, max_rows_per_launch=65536, slots=3, with_step_masks=step_masks) as srv:
            def waiter():
                while True:
                    with lock:
                        while not spans and not done_sub[0]:
                            lock.wait()
                        if not spans:
                            return
                        rid = spans[0][2]
                    srv.wait(rid)
                    with lock:
                        spans.popleft()
                        lock.notify_all()
            th = threading.Thread(target=waiter)
            th.start()
            start = srv.now_ns() + 2_000_000
            measured_from = int(np.searchsorted(t_arr, warm_s))
            rows_meas = 0
            for i, (ta, r) in enumerate(zip(t_arr, rows)):
                r = int(r)
                mi = int(pick[i])
                c = cfgs[mi]
                if i == measured_from:
                    srv.reset_stats()
                need = r * per_row[mi]
                with lock:
                    while (base := _ring_alloc(spans, head[0], need, RING)) is None:
                        lock.wait()
                lo = ring[base:base + r * c.n_out].reshape(r, c.n_out)
                ag = ring[base + r * c.n_out:base + r * (c.n_out + c.D)].reshape(r, c.D)
                ms = (ring[base + r * (c.n_out + c.D):base + need].reshape(c.n_steps, r, c.D)
                      if step_masks else None)
                pool = Xpools[mi]
                off = (i * 7919) % (pool.shape[0] - r)
                target = start + int(ta * 1e9)
                while srv.now_ns() < target:
                    pass
                rid = srv.submit(mi, pool[off:off + r], lo, ag, ms, arrival_ns=target)
                if i >= measured_from:
                    rows_meas += r
                with lock:
                    spans.append((base, base + need, rid))
                    head[0] = base + need
                    lock.notify_all()
            with lock:
                done_sub[0] = True
                lock.notify_all()
            th.join()
            st = srv.stats()
            per = [srv.model_stats(k) for k in range(len(models))] if len(models) > 1 else []
        pt = {"rate_req_s": lam, "requests": int(st["completed"]), "offered_rows_per_s": rows_meas / dur_s,
              "rows_per_s": st["rows_per_s"], "p50_ms": st["p50_us"] / 1e3, "p99_ms": st["p99_us"] / 1e3,
              "p999_ms": st["p999_us"] / 1e3, "mean_rows_per_launch": st["mean_rows_per_launch"],
              "launches": int(st["launches"])}
        if per:
            pt["per_model"] = [{"requests": int(q["completed"]), "rows_per_s": q["rows_per_s"],
                                "p50_ms": q["p50_us"] / 1e3, "p99_ms": q["p99_us"] / 1e3,
                                "mean_rows_per_launch": q["mean_rows_per_launch"], "launches": int(q["launches"])}
                               for q in per]
        out.append(pt)
        print(f"[bench] serve{' mix' if len(models) > 1 else ''} {lam} req/s: p50 {st['p50_us']/1e3:.3f} ms "
              f"p99 {st['p99_us']/1e3:.3f} ms {st['rows_per_s']/1e6:.2f} M rows/s, "
              f"{st['mean_rows_per_launch']:.0f} rows/launch", file=sys.stderr, flush=True)
    return out


def wide_leg(precs, steps: int, tmpdir: str):
    """The 200-feature model at its full batch (1,048,576 rows, D = 200, n_d = n_a = 64,
    7 steps, step masks on) in each precision: time per launch (HIP events on the launch
    stream, after a clock ramp and two untimed launches), rows/s, and the fractions of the
    matrix-core roof of the precision and of the HBM roof."""
    import torch
    from paper_2510_19689_amd import synth, tabnet
    cfg = synth.WORKLOADS["wide200"]["cfg"]
    params, Xh = synth.workload("wide200")
    rows = Xh.shape[0]
    path = os.path.join(tmpdir, "wide200.tnw")
    synth.write_weights(params, path)
    X = torch.from_numpy(Xh).cuda()
    byt, flops = algorithmic(cfg, rows, with_steps=True)
    peaks = {"fp32": FP32_MFMA_PEAK_TFLOPS, "bf16": BF16_PEAK_TFLOPS, "fp8": FP8_PEAK_TFLOPS,
             "fp8w": BF16_PEAK_TFLOPS}
    n = max(3, steps // 5)
    out = {"rows": rows, "D": cfg.D, "n_d": cfg.n_d, "n_a": cfg.n_a, "n_steps": cfg.n_steps,
           "n_shared": cfg.n_shared, "n_indep": cfg.n_indep, "n_out": cfg.n_out, "masks_step": True,
           "algorithmic_bytes_per_launch": byt, "algorithmic_flops_per_launch": flops, "launches_timed": n}
    for prec in precs:
        with tabnet.Model(path, prec) as m:
            outs = m.outputs(rows, with_steps=True)
            clock_ramp(m, X, outs, 0.1)
            t, _ = time_forward(m, X, outs, n, 2)
            per = t / n
            out[prec] = {"ms_per_forward": per * 1e3, "rows_per_s": rows / per,
                         "mfma_tflops": flops / per / 1e12, "mfma_frac": flops / per / 1e12 / peaks[prec],
                         "hbm_GB_s": byt / per / 1e9, "hbm_frac": byt / per / 1e9 / HBM_PEAK_GBS}
            print(f"[bench] wide200 {prec}: {per * 1e3:.2f} ms/forward, {rows / per / 1e6:.1f} M rows/s, "
                  f"{out[prec]['mfma_frac'] * 100:.1f}% of the {prec} matrix roof", file=sys.stderr, flush=True)
            del outs
    if "bf16" in out and "fp32" in out:
        out["bf16_over_fp32"] = out["fp32"]["ms_per_forward"] / out["bf16"]["ms_per_forward"]
    for q in ("fp8", "fp8w"):
        if "bf16" in out and q in out:
            out[q + "_over_bf16"] = out["bf16"]["ms_per_forward"] / out[q]["ms_per_forward"]
    del X
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=2000,
                    help="untimed launches first (~0.2 s at the default workload: the GPU reaches its "
                         "steady clock within that)")
    ap.add_argument("--workload", default="adult108")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--quant", default="fp8,fp8w,int8,mxfp8,mxfp8_e5m2,mxfp6,mxfp6_e3m2,mxfp4",
                    help="reduced-precision paths timed beside BF16 and FP32 (fp8: E4M3 weights and GEMM "
                         "inputs; int8: INT8 weights and GEMM inputs; mxfp8, mxfp8_e5m2, mxfp6, mxfp6_e3m2, "
                         "mxfp4: OCP MX on both GEMM operands); "
                         "empty to skip")
    ap.add_argument("--serve-rates", default="2000,5000,10000,20000",
                    help="request rates (req/s) of the serving leg; empty to skip")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-step-masks", type=int, default=1,
                    help="serving requests also return the per-step masks (1) or only logits and the "
                         "aggregate mask (0)")
    ap.add_argument("--serve-mix-step-masks", type=int, default=0,
                    help="mixed-load requests also return the per-step masks (1; up to 168 MB per "
                         "8,192-row request of the 512-feature model) or not (0)")
    ap.add_argument("--wide", default="fp32,bf16,fp8,fp8w",
                    help="precisions of the 200-feature leg (1,048,576 rows, 7 steps); empty to skip")
    ap.add_argument("--serve-mix-rates", default="2000,5000,10000",
                    help="request rates of a mixed load over four resident models (HR-, Adult-, "
                         "200- and 512-feature models, requests of 1..8192 rows); empty to skip")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of TabNet, time a plain device-to-device copy of this many "
                         "bytes (the reference for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (rows are "
              "independent, so the path shards by rows with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2510_19689_amd import synth, tabnet

    if args.copy_bytes:
        n = args.copy_bytes // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.warmup):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"copy_bytes": n * 4, "s_per_copy": dt, "GB_s": 2 * n * 4 / dt / 1e9}))
        return

    name = args.workload
    w = synth.WORKLOADS[name]
    cfg, rows = w["cfg"], w["rows"]
    params, Xh = synth.workload(name)
    print(f"[bench] workload {name}: rows={rows} D={cfg.D} n_d=n_a={cfg.n_d} steps={cfg.n_steps}",
          file=sys.stderr, flush=True)
    X = torch.from_numpy(Xh).cuda()
    res = {}
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, f"{name}.tnw")
        synth.write_weights(params, path)
        precs = ["bf16"] + ([] if args.skip_fp32 else ["fp32"]) + [p for p in args.quant.split(",") if p]
        for prec in precs:
            try:
                m = tabnet.Model(path, prec)
            except tabnet.TabNetError as err:
                if err.status != tabnet.E_UNSUPPORTED or prec in ("bf16", "fp32"):
                    raise
                print(f"[bench] {prec}: no kernel for this shape", file=sys.stderr, flush=True)
                continue
            with m:
                outs = m.outputs(rows, with_steps=True)
                ramp = clock_ramp(m, X, outs, CLOCK_RAMP_S if prec == "bf16" else 0.05)
                if prec == "bf16":
                    res["ramp"] = ramp
                t, wall = time_forward(m, X, outs, args.steps, args.warmup)
                res[prec] = (t, wall)
                print(f"[bench] {prec}: {t / args.steps * 1e6:.1f} us/forward, "
                      f"{rows * args.steps / t / 1e6:.1f} M rows/s", file=sys.stderr, flush=True)
                if prec == "bf16":
                    res["detail"] = forward_detail(m, X, outs)
                    dd = res["detail"]
                    print(f"[bench] bf16 per launch p10/p50/p90 {dd['p10_us']:.1f}/{dd['p50_us']:.1f}/"
                          f"{dd['p90_us']:.1f} us; without step masks {dd['no_step_masks_us']:.1f} us; "
                          f"graph replay {dd['graph_replay_us']:.1f} us", file=sys.stderr, flush=True)
                    t_ms = time_mask_stats(outs[1], args.steps, args.warmup)
                    res["mask_stats"] = t_ms
                    print(f"[bench] mask_stats of masks_agg: {t_ms * 1e6:.2f} us, "
                          f"{rows * cfg.D * 4 / t_ms / 1e9:.0f} GB/s", file=sys.stderr, flush=True)
                    if w["data"] in ("adult", "hr"):
                        # the same rows before embedding: gather in the kernel, masks per raw column
                        X_raw, cards, dims, tables = synth.make_raw_inputs(w["data"], rows, synth.DATA_SEED[name])
                        m.set_embeddings(cards, dims, tables)
                        Xr = torch.from_numpy(X_raw).cuda()
                        C = X_raw.shape[1]
                        routs = (torch.empty((rows, cfg.n_out), dtype=torch.float32, device="cuda"),
                                 torch.empty((rows, C), dtype=torch.float32, device="cuda"),
                                 torch.empty((cfg.n_steps, rows, C), dtype=torch.float32, device="cuda"))
                        t_raw = time_forward_raw(m, Xr, routs, args.steps, args.warmup)
                        res["raw"] = (t_raw, C)
                        print(f"[bench] bf16 raw rows (C={C}): {t_raw * 1e6:.1f} us/forward, "
                              f"{rows / t_raw / 1e6:.1f} M rows/s", file=sys.stderr, flush=True)
                        del routs, Xr
                del outs
        wide = None
        if args.wide and name == "adult108":
            wide = wide_leg([p for p in args.wide.split(",") if p], args.steps, d)
        serving = None
        sm = bool(args.serve_step_masks)
        if args.serve_rates:
            rates = [int(r) for r in args.serve_rates.split(",") if r]
            with tabnet.Model(path, "bf16") as m:
                serving = serve_bench([m], [Xh], rates, warm_s=0.5, dur_s=args.serve_seconds, step_masks=sm)
        serving_mix = None
        if args.serve_mix_rates:
            rates = [int(r) for r in args.serve_mix_rates.split(",") if r]
            names = ["hr35", "adult108", "wide200", "wide512"]
            models, pools = [], []
            for nm in names:
                p_nm = os.path.join(d, f"{nm}.tnw")
                synth.write_weights(synth.make_params(synth.WORKLOADS[nm]["cfg"], synth.WEIGHT_SEED[nm]), p_nm)
                models.append(tabnet.Model(p_nm, "bf16"))
                pools.append(synth.make_inputs(synth.WORKLOADS[nm]["data"], 20000, synth.DATA_SEED[nm]))
            try:
                smx = bool(args.serve_mix_step_masks)
                serving_mix = {"models": names, "precision": "bf16",
                               "masks": "logits + masks_agg" + (" + masks_step" if smx else ""),
                               "request_rows": "log-uniform 1..8192", "model_choice": "uniform, seeded",
                               "arrivals": "Poisson, open loop", "seconds_per_rate": args.serve_seconds,
                               "points": serve_bench(models, pools, rates, warm_s=0.5, dur_s=args.serve_seconds,
                                                     step_masks=smx, max_rows=8192, mix_seed=4000)}
            finally:
                for m in models:
                    m.close()
    t_bf16, wall_bf16 = res["bf16"]
    per_launch = t_bf16 / args.steps
    value = rows * args.steps / t_bf16
    byt, flops = algorithmic(cfg, rows, with_steps=True)
    achieved_gbs = byt / per_launch / 1e9
    out = {
        "metric": "TabNet rows/sec (BF16/FP8 vs FP32 plain, same GPU) + p50/p99 ms at fixed QPS",
        "value": value,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_launch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded " + {"hr": "HR-shaped", "adult": "Adult-shaped", "wide": "200-feature",
                                        "wide512": "512-feature N(0,1)"}[w["data"]]
                + " rows and Xavier-uniform weights; no dataset)",
        "config": {"workload": name, "rows": rows, "D": cfg.D, "n_d": cfg.n_d, "n_a": cfg.n_a,
                   "n_steps": cfg.n_steps, "n_shared": cfg.n_shared, "n_indep": cfg.n_indep,
                   "n_out": cfg.n_out, "gamma": cfg.gamma, "masks_step": True,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": profiled_traffic(name),
                     "kernel": "tabnet_forward_kernel<bf16>",
                     "algorithmic_bytes_per_launch": byt,
                     "mfma_tflops": flops / per_launch / 1e12},
    }
    if "fp32" in res:
        t32 = res["fp32"][0]
        out["fp32_rows_per_s"] = rows * args.steps / t32
        out["bf16_over_fp32"] = t32 / t_bf16
        out["fp32_mfma_frac"] = flops / (t32 / args.steps) / 1e12 / FP32_MFMA_PEAK_TFLOPS
    quant = {}
    for prec, what in (("fp8", "E4M3 weights (one scale per output channel) and GEMM inputs (one scale per "
                                "row), FP8 MFMA"),
                       ("fp8w", "E4M3 weights (one scale per output channel), BF16 GEMM inputs, codes widened "
                                 "to BF16 for the BF16 MFMA"),
                       ("int8", "INT8 weights (one scale per output channel) and GEMM inputs (one step "
                                "per row), INT32 products"),
                       ("mxfp8", "OCP MXFP8 (E4M3 elements, E8M0 scale per 32) on both GEMM operands, "
                                 "scaled MFMA"),
                       ("mxfp8_e5m2", "OCP MXFP8 with E5M2 elements (E8M0 scale per 32) on both GEMM "
                                      "operands, scaled MFMA"),
                       ("mxfp6", "OCP MXFP6 (E2M3 elements, E8M0 scale per 32) on both GEMM operands, "
                                 "scaled MFMA"),
                       ("mxfp6_e3m2", "OCP MXFP6 with E3M2 elements (E8M0 scale per 32) on both GEMM "
                                      "operands, scaled MFMA"),
                       ("mxfp4", "OCP MXFP4 (E2M1 elements, E8M0 scale per 32) on both GEMM operands, "
                                 "scaled MFMA")):
        if prec in res:
            tq = res[prec][0]
            quant[prec] = {"what": what, "us_per_forward": tq / args.steps * 1e6,
                           "rows_per_s": rows * args.steps / tq, "over_bf16": t_bf16 / tq}
    if quant:
        out["quantised"] = quant
    out["paper_context"] = PAPER_CONTEXT
    out["wall_s_bf16"] = wall_bf16
    out["clock_ramp"] = {"seconds": CLOCK_RAMP_S, "launches": res.get("ramp", 0),
                         "what": "untimed launches of the same forward before the warm-up"}
    if "detail" in res:
        out["bf16_forward_detail"] = res["detail"]
    if "raw" in res:
        t_raw, C = res["raw"]
        rb = 4 * (C + cfg.n_out + C + cfg.n_steps * C)
        out["raw_rows"] = {"what": "BF16 forward on raw rows: embedding gathered in the kernel, masks per raw column",
                           "columns": C, "rows_per_s": rows / t_raw, "us_per_forward": t_raw * 1e6,
                           "algorithmic_bytes_per_row": rb, "GB_s": rb * rows / t_raw / 1e9}
    if "mask_stats" in res:
        t_ms = res["mask_stats"]
        gbs = rows * cfg.D * 4 / t_ms / 1e9
        out["mask_stats"] = {"what": "per-feature mean and variance of masks_agg", "rows": rows, "D": cfg.D,
                             "us_per_call": t_ms * 1e6, "GB_s": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    if serving is not None:
        worst = max(pt["p99_ms"] for pt in serving)
        out["serving"] = {"model": name, "precision": "bf16",
                          "masks": "logits + masks_agg" + (" + masks_step" if sm else ""),
                          "request_rows": "log-uniform 1..4096", "arrivals": "Poisson, open loop",
                          "seconds_per_rate": args.serve_seconds,
                          "p99_bound_ms": SERVE_P99_BOUND_MS, "p99_worst_ms": worst,
                          "p99_within_bound": bool(worst <= SERVE_P99_BOUND_MS), "points": serving}
    if wide is not None:
        out["wide200"] = wide
    if serving_mix is not None:
        out["serving_mix"] = serving_mix
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(params, Xh)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
