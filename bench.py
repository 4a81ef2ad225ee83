#!/usr/bin/env python3
"""SpAMM benchmark on one MI355X.

One step = the whole hot path over one input matrix already resident in HBM:
build the quadtree (leaf norms + pack + norm pyramid), then the product
C = A A under the SpAMM condition (tier-by-tier cull + MFMA leaf GEMM).

    python bench.py [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  `value` is kept-leaf TFLOP/s over the whole step
(2 n_b^3 K / step time).  `roofline` rates the leaf GEMM kernel (the dominant
kernel) against the FP32 MFMA peak, with its duration from HIP events recorded
around its launch on the stream it runs on.  `cpu_baseline` times the FP64
oracle on a seeded sample of output leaves of the same matrix.  `serving`
then drives a stream of 2000 products and squaring chains of uneven size
through the continuous-batching server: saturation throughput, and p50/p99
latency under Poisson arrivals at 0.5x and 0.8x of it (`--serve` runs only
that, `--no-serve` skips it).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_FP32_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E peak
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "leaf_gemm_cluster1310-n32750_traffic.json")


# The paper's single-core CPU figures (Sec. V.B, numeric multiply against
# SGEMM; platforms in Sec. IV.A).  Context for the GPU numbers only.
PAPER_CONTEXT = {
    "note": "the paper's own FP32 CPU figures, one core, context only (other hardware, other matrices)",
    "spamm_numeric_gflops_dense_16x16_blocks": {"AMD Opteron 6168 (1.8 GHz)": 8.1,
                                                 "Intel Xeon X5650 (2.66 GHz)": 13.7},
    "sgemm_gflops_large_n": {"AMD Opteron 6168, ACML or MKL": 12.6,
                             "Intel Xeon X5650, ACML": 12.7, "Intel Xeon X5650, MKL": 19.8},
    "source": "Sec. V.B (numeric multiply vs. SGEMM), Sec. IV.A (platforms)",
}

GEMM_SOURCES = ("paper_1203_1692_amd/csrc/gemm.hip", "paper_1203_1692_amd/csrc/common.hpp",
                "paper_1203_1692_amd/_build.py")


def kernel_source_digest() -> str:
    """SHA-256 over the leaf GEMM's source, its layout header and build flags."""
    h = hashlib.sha256()
    for rel in GEMM_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per leaf-GEMM launch from the committed rocprofv3 counter runs,
    or None when absent, for another workload, or taken on other kernel code."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("gemm_sources_sha256") != kernel_source_digest():
        return None
    return rec.get("bytes_per_launch")


def measured_split_traffic(workload: str, tau: float, low_tol: float, fmt: str = "bf16"):
    """HBM bytes per launch of the split kernel (LOW operands in `fmt`) at
    (tau, low_tol) from the committed counter runs, or None when the kernel
    sources changed since."""
    kind = "leaf_gemm_split" if fmt == "bf16" else "leaf_gemm_split_fp16"
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if (t.get("gemm_sources_sha256") != kernel_source_digest() or
            abs(t.get("tau", -1.0) - tau) > 1e-12 * tau or
            abs(t.get("low_tol", -1.0) - low_tol) > 1e-12 * low_tol):
        return None
    return t["bytes_per_launch"]


def measured_sub_traffic(workload: str, tau: float):
    """HBM bytes per launch of the sub-leaf culling kernel at tau from the
    committed counter runs, or None when the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"leaf_gemm_sub_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if (t.get("gemm_sources_sha256") != kernel_source_digest() or
            abs(t.get("tau", -1.0) - tau) > 1e-12 * tau):
        return None
    return t["bytes_per_launch"]


def sample_tiles(N: int, count: int, seed: int = 0):
    import numpy as np
    rng = np.random.default_rng(seed)
    flat = rng.choice(N * N, size=min(count, N * N), replace=False)
    return [(int(f) // N, int(f) % N) for f in np.sort(flat)]


def matched_error(sp, wl, A, dA, C, tau, leaf, n, N, reps=2):
    import numpy as np
    rng = np.random.default_rng(7)
    tiles = [(int(i), int(j)) for i, j in rng.integers(0, N, size=(24, 2))]
    tiles += [(int(i), int(i)) for i in rng.integers(0, N, size=12)]
    tiles = sorted({(I, J) for I, J in tiles if I * leaf < n and J * leaf < n})
    exact = {}
    for (I, J) in tiles:
        r0, r1 = I * leaf, min((I + 1) * leaf, n)
        c0, c1 = J * leaf, min((J + 1) * leaf, n)
        exact[(I, J)] = A[r0:r1].astype(np.float64) @ A[:, c0:c1].astype(np.float64)

    def max_err():
        # only the sampled leaves come back to the host
        e = 0.0
        for (I, J), ex in exact.items():
            r0, c0 = I * leaf, J * leaf
            blk = C[r0:r0 + ex.shape[0], c0:c0 + ex.shape[1]].cpu().numpy()
            e = max(e, float(np.abs(blk - ex).max()))
        return e

    taus = [tau * 10.0 ** (h / 2) for h in range(11)]       # tau x 10^{0, 0.5, ..., 5}

    tree = sp.build_tree(dA, leaf, bf16=True)
    points = []
    for t_ in taus:
        for lmul in (0, 256, 512, 1024, 2048, 4096, 8192, 16384):
            prec = sp.PREC_SPLIT_BF16 if lmul else sp.PREC_FP32
            best = None
            for _ in range(reps):
                st = sp.multiply_ex(tree, tree, t_, C, precision=prec, low_tol=lmul * t_)
                ms = st["symbolic_ms"] + st["numeric_ms"]
                best = ms if best is None else min(best, ms)
            points.append({"precision": "split-bf16" if lmul else "fp32", "tau": t_,
                           "low_tol": lmul * t_, "ms": round(best, 3), "err": max_err(),
                           "ms_leaf_gemm": round(st["numeric_ms"], 3),
                           "tasks": st["tasks"], "low_frac": round(st["tasks_low"] / max(1, st["tasks"]), 4)})
    tree.free()
    # FP16 LOW operands (8 times finer than BF16): the same tau grid, low_tol up to 64x higher
    tree = sp.build_tree(dA, leaf, fp16=True)
    for t_ in taus:
        for lmul in [1024 * 2 ** h for h in range(11)]:           # 1024 .. 1048576
            best = None
            for _ in range(reps):
                st = sp.multiply_ex(tree, tree, t_, C, precision=sp.PREC_SPLIT_FP16,
                                    low_tol=lmul * t_)
                ms = st["symbolic_ms"] + st["numeric_ms"]
                best = ms if best is None else min(best, ms)
            points.append({"precision": "split-fp16", "tau": t_, "low_tol": lmul * t_,
                           "ms": round(best, 3), "err": max_err(),
                           "ms_leaf_gemm": round(st["numeric_ms"], 3), "tasks": st["tasks"],
                           "low_frac": round(st["tasks_low"] / max(1, st["tasks"]), 4)})
    tree.free()
    target = next(p["err"] for p in points if p["precision"] == "fp32" and p["tau"] == tau)
    subleaf = None
    if leaf == 64:
        # sub-leaf culling: 32 x 32 sub-products tested inside each 64 x 64 one
        sub_tree = sp.build_tree(dA, leaf, subnorms=True)
        for h in range(-2, 10):                                # tau x 10^{-1, ..., 4.5}
            t_ = tau * 10.0 ** (h / 2)
            best = None
            for _ in range(reps):
                st = sp.multiply_ex(sub_tree, sub_tree, t_, C, sub_cull=True)
                ms = st["symbolic_ms"] + st["numeric_ms"]
                if best is None or ms < best[0]:
                    best = (ms, st["numeric_ms"])
            points.append({"precision": "fp32-subleaf", "tau": t_, "low_tol": 0.0,
                           "ms": round(best[0], 3), "ms_leaf_gemm": round(best[1], 3),
                           "err": max_err(), "tasks": st["tasks"],
                           "sub_products": st["subtasks"],
                           "sub_fraction": round(st["subtasks"] / max(1, 8 * st["tasks"]), 4)})
        sub_tree.free()
        at_tau = next(p for p in points if p["precision"] == "fp32-subleaf" and p["tau"] == tau)
        plain = next(p for p in points if p["precision"] == "fp32" and p["tau"] == tau)
        subleaf = {"tau": tau, "leaf_products": plain["tasks"],
                   "sub_products": at_tau["sub_products"], "sub_fraction": at_tau["sub_fraction"],
                   "ms_plain": plain["ms"], "ms_subleaf": at_tau["ms"],
                   "err_plain": plain["err"], "err_subleaf": at_tau["err"]}

    def fastest(kind):
        ok = [p for p in points if p["precision"] == kind and p["err"] <= target]
        return min(ok, key=lambda p: p["ms"]) if ok else None

    f32, spl, sub = fastest("fp32"), fastest("split-bf16"), fastest("fp32-subleaf")
    s16 = fastest("split-fp16")

    def split_roof(point, fmt, kernel):
        if point is None:
            return None
        tb = measured_split_traffic(wl.name, point["tau"], point["low_tol"], fmt)
        if tb is None:
            return None
        gbs = tb / (point["ms_leaf_gemm"] * 1e-3) / 1e9
        return {"kernel": kernel, "bound": "hbm", "achieved": round(gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": tb,
                "note": "measured HBM bytes per launch / leaf-GEMM time; the LOW phase runs "
                        "above this average, the HIGH tail below"}

    split_roofline = split_roof(spl, "bf16", "leaf_gemm_split<64, false>")
    split_fp16_roofline = split_roof(s16, "fp16", "leaf_gemm_split<64, true>")
    return {
        "target_err": target,
        "err_sample": f"{len(tiles)} seeded output leaves (incl. diagonal), dense FP64 reference",
        "fp32_at_target": f32, "split_at_target": spl, "split_fp16_at_target": s16,
        "subleaf_at_target": sub,
        "speedup_split_vs_fp32": round(f32["ms"] / spl["ms"], 3) if f32 and spl else None,
        "speedup_split_fp16_vs_fp32": round(f32["ms"] / s16["ms"], 3) if f32 and s16 else None,
        "speedup_subleaf_vs_fp32": round(f32["ms"] / sub["ms"], 3) if f32 and sub else None,
        "split_roofline": split_roofline,
        "split_fp16_roofline": split_fp16_roofline,
        "subleaf_same_tau": subleaf,
        "grid": "tau x 10^{0, 0.5, ..., 5}; low_tol = 0 (fp32), tau x {256, 512, ..., 16384} "
                "(bf16), tau x {1024, 2048, ..., 1048576} (fp16); "
                "sub-leaf culling: tau x 10^{-1, -0.5, ..., 4.5}",
    }


# ---------------------------------------------------------------------------
# Serving: continuous batching of a stream of products and squaring chains
# ---------------------------------------------------------------------------
def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def serve_inputs(torch, reqs, dev):
    """Every request's input, generated on the device before any timed run
    (so the runs measure the server, not the generator)."""
    from workloads import serve_matrix
    inputs = {req.index: serve_matrix(torch, req, dev) for req in reqs}
    torch.cuda.synchronize()
    return inputs


def serve_run(sp, torch, srv, reqs, inputs, qps=None, window=16, keep=()):
    """Drive `reqs` through the server: open loop with Poisson arrivals at
    `qps`, or closed loop with `window` requests outstanding (qps None).
    Returns per-request results, timing and the C of the requests in `keep`."""
    import numpy as np
    from workloads import SERVE_LEAF, SERVE_THETA
    out, kept = {}, {}
    pending = {}
    arrivals = None
    t0 = time.perf_counter()
    if qps is not None:
        arrivals = t0 + np.cumsum([r.gap for r in reqs]) / qps

    def sweep():
        got = False
        for t in list(pending):
            res = srv.poll(t)
            if res is not None:
                req, C = pending.pop(t)
                res["n"], res["chain"], res["split"] = req.n, req.chain_len, req.split
                out[req.index] = res
                if req.index in keep:
                    kept[req.index] = C
                got = True
        return got

    t_first = t_last = None
    info0 = srv.info()
    for k, req in enumerate(reqs):
        if arrivals is None:
            while len(pending) >= window:
                if not sweep():
                    time.sleep(50e-6)
        else:
            while time.perf_counter() < arrivals[k]:
                if not sweep():
                    time.sleep(50e-6)
        A = inputs[req.index]
        C = torch.empty_like(A)
        t_sub = time.perf_counter()
        t_first = t_first or t_sub
        t_last = t_sub
        tk = srv.submit(A, C, req.tau, SERVE_LEAF,
                        precision=sp.PREC_SPLIT_BF16 if req.split else sp.PREC_FP32,
                        low_rel=SERVE_THETA if req.split else 0.0, chain_len=req.chain_len,
                        sync=False)
        pending[tk] = (req, C)
    while pending:
        if not sweep():
            time.sleep(50e-6)
    t_end = time.perf_counter()
    info1 = srv.info()
    busy = ((info1["sched_cpu_ms"] - info0["sched_cpu_ms"]) /
            max(info1["sched_wall_ms"] - info0["sched_wall_ms"], 1e-9))
    return out, kept, dict(t0=t0, t_first=t_first, t_last=t_last, t_end=t_end, sched_busy=busy)


def serve_summary(reqs, res, tm, qps):
    lat = [res[r.index]["latency_ms"] for r in reqs]
    bad = sum(res[r.index]["status"] != 0 for r in reqs)
    span = tm["t_end"] - tm["t_first"]
    flops = sum(res[r.index]["flops"] for r in reqs)

    def pq(sel):
        v = [res[r.index]["latency_ms"] for r in reqs if sel(r)]
        return {"count": len(v), "p50_ms": percentile(v, 50), "p99_ms": percentile(v, 99)}

    d = {
        "offered_qps": qps,
        "arrival_qps": (len(reqs) - 1) / (tm["t_last"] - tm["t_first"]) if len(reqs) > 1 else None,
        "throughput_rps": len(reqs) / span,
        "kept_tile_tflops": flops / span / 1e12,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "queue_p50_ms": percentile([res[r.index]["queue_ms"] for r in reqs], 50),
        "queue_p99_ms": percentile([res[r.index]["queue_ms"] for r in reqs], 99),
        "failed": bad,
        "scheduler_cpu_fraction": tm.get("sched_busy"),
        "plain": pq(lambda r: r.chain_len == 0),
        "chains": pq(lambda r: r.chain_len > 0),
        "fp32": pq(lambda r: not r.split),
        "split_bf16": pq(lambda r: r.split),
        "by_n": {str(n): pq(lambda r, n=n: r.n == n) for n in sorted({r.n for r in reqs})},
    }
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}


def serve_verify(sp, torch, reqs, kept, inputs):
    """Requests kept from the mix, recomputed alone through the one-call API
    (tree build + multiply per step): the bits must agree.  Returns the
    number that agree and, per kept chain, its kept (and LOW) products per
    step."""
    from workloads import SERVE_LEAF, SERVE_THETA
    ok = 0
    per_step = {}
    for req in reqs:
        if req.index not in kept:
            continue
        X = inputs[req.index]
        prec = sp.PREC_SPLIT_BF16 if req.split else sp.PREC_FP32
        ks = []
        for _ in range(max(1, req.chain_len)):
            t = sp.build_tree(X, SERVE_LEAF, bf16=req.split)
            C = torch.empty_like(X)
            st = sp.multiply_ex(t, t, req.tau, C, precision=prec,
                                low_rel=SERVE_THETA if req.split else 0.0)
            ks.append([st["tasks"], st["tasks_low"]])
            t.free()
            X = C
        ok += int(torch.equal(X, kept[req.index]))
        if req.chain_len:
            per_step[f"request {req.index} (n={req.n}, rate={req.rate:.3f}, tau={req.tau:g}, "
                     f"{'split' if req.split else 'fp32'})"] = ks
    return ok, per_step


def serve_one_call(sp, torch, reqs, inputs):
    """The same requests through the one-call API, one after another (tree
    build + multiply per step, each synchronizing): the plain GPU form the
    server is compared with.  Results are those of the server bit for bit
    (serve_verify), so the errors match."""
    from workloads import SERVE_LEAF, SERVE_THETA
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for req in reqs:
        X = inputs[req.index]
        prec = sp.PREC_SPLIT_BF16 if req.split else sp.PREC_FP32
        for _ in range(max(1, req.chain_len)):
            t = sp.build_tree(X, SERVE_LEAF, bf16=req.split)
            C = torch.empty_like(X)
            sp.multiply_ex(t, t, req.tau, C, precision=prec,
                           low_rel=SERVE_THETA if req.split else 0.0)
            t.free()
            X = C
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"requests_per_s": round(len(reqs) / wall, 2), "wall_s": round(wall, 3),
            "note": "each request alone through spamm_build_tree + spamm_multiply_opts per "
                    "step, synchronizing; same results as served"}


def serve_bench(sp, torch, dev, count, slots, budget_gib):
    """Saturation (closed loop, 2 x slots outstanding), then Poisson arrivals
    at 0.5x and 0.8x of it; returns the summary dict."""
    import workloads
    reqs = workloads.serving_mix(count)
    t = time.perf_counter()
    inputs = serve_inputs(torch, reqs, dev)
    t_gen = time.perf_counter() - t
    print(f"serving inputs: {len(reqs)} matrices in {t_gen:.1f} s", file=sys.stderr, flush=True)
    srv = sp.Server(int(budget_gib * (1 << 30)), max_slots=slots)
    try:
        # warm-up outside the timed runs: every slot's arena grown to the largest
        # footprint (no device allocation inside the timed runs), every
        # size x precision x chain combination run once, torch's cache holding
        # output buffers for the outstanding requests
        big = max(workloads.SERVE_SIZES)
        warm = [workloads.ServeRequest(i, big, 0.05, 1e-8, 0, True, 900000 + i, 1.0)
                for i in range(slots)]
        warm += [workloads.ServeRequest(len(warm) + j, n_, 0.1, 1e-6, chain, split, 910000 + j, 1.0)
                 for j, (n_, chain, split) in enumerate(
                     (n_, c, sp_) for n_ in workloads.SERVE_SIZES for c in (0, 10)
                     for sp_ in (False, True))]
        serve_run(sp, torch, srv, warm, serve_inputs(torch, warm, dev), window=slots)
        spare = [torch.empty((n_, n_), device=dev) for n_ in workloads.SERVE_SIZES
                 for _ in range(2 * slots)]
        del spare
        res, _, tm = serve_run(sp, torch, srv, reqs, inputs, window=2 * slots)
        sat = serve_summary(reqs, res, tm, None)
        print(f"saturation: {sat['throughput_rps']:.2f} req/s, p50 {sat['p50_ms']} ms, "
              f"p99 {sat['p99_ms']} ms", file=sys.stderr, flush=True)
        loads = {}
        keep_idx = set()
        for want in (lambda r: r.chain_len > 0 and r.split, lambda r: r.chain_len > 0,
                     lambda r: r.split and r.n == 8192, lambda r: r.n == 512):
            keep_idx |= {next(r.index for r in reqs if want(r))}
        verified = None
        for frac in (0.5, 0.8):
            qps = frac * sat["throughput_rps"]
            i0 = srv.info()
            res, kept, tm = serve_run(sp, torch, srv, reqs, inputs, qps=qps,
                                      keep=keep_idx if frac == 0.8 else ())
            i1 = srv.info()
            s = serve_summary(reqs, res, tm, round(qps, 3))
            s["launches"] = i1["launches"] - i0["launches"]
            s["mean_products_per_launch"] = round(
                (i1["launched_products"] - i0["launched_products"]) / max(1, s["launches"]), 3)
            loads[f"{frac}x"] = s
            print(f"{frac}x load: {s['arrival_qps']} req/s offered, p50 {s['p50_ms']} ms, "
                  f"p99 {s['p99_ms']} ms", file=sys.stderr, flush=True)
            if frac == 0.8:
                verified, chain_steps = serve_verify(sp, torch, reqs, kept, inputs)
        info = srv.info()
    finally:
        srv.destroy()
    one = serve_one_call(sp, torch, reqs, inputs)
    print(f"one-call API, one request at a time: {one['requests_per_s']} req/s",
          file=sys.stderr, flush=True)
    del inputs
    torch.cuda.empty_cache()
    return {
        "workload": f"serve-mix{len(reqs)}",
        "requests": len(reqs), "sizes": list(workloads.SERVE_SIZES),
        "leaf": workloads.SERVE_LEAF, "taus": [1e-6, 1e-8], "chain_share": 0.3,
        "chain_len": 10, "split_share": 0.5, "split_theta": workloads.SERVE_THETA,
        "slots": slots, "budget_gib": budget_gib,
        "input": "device-generated per request (torch generator, seed 1000+r), resident "
                 "before the timed runs",
        "saturation": sat,
        "loads": loads,
        "verified_bitwise_vs_alone": f"{verified}/{len(keep_idx)}",
        "chain_kept_products_per_step": chain_steps,
        "one_call_sequential": one,
        "served_speedup_vs_one_call": round(sat["throughput_rps"] / one["requests_per_s"], 3),
        "server": {k: info[k] for k in ("max_batch", "peak_active", "peak_used", "budget")},
    }


def serve_main(args) -> int:
    import torch

    import paper_1203_1692_amd as sp

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sp.load()
    sv = serve_bench(sp, torch, dev, args.serve_requests, args.serve_slots, args.serve_budget_gib)
    out = {
        "metric": "serving: saturation throughput; p50/p99 latency at 0.5x and 0.8x of it",
        "value": round(sv["saturation"]["throughput_rps"], 3),
        "unit": "requests/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {k: v for k, v in sv.items() if k not in ("saturation", "loads")},
        "saturation": sv["saturation"],
        "loads": sv["loads"],
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cluster1310-n32750")
    ap.add_argument("--tau", type=float, default=None)
    ap.add_argument("--sample-tiles", type=int, default=96,
                    help="output leaves checked against the dense FP64 product")
    ap.add_argument("--oracle-tiles", type=int, default=3072,
                    help="output leaves computed by the FP64 oracle (CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--no-matched-error", action="store_true",
                    help="skip the FP32-vs-split comparison at a fixed max-norm error")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark instead: saturation, then Poisson arrivals")
    ap.add_argument("--precision", choices=("fp32", "split", "split-fp16"), default="fp32",
                    help="product of the timed steps (split: BF16 for LOW products, "
                         "split-fp16: FP16 at a per-leaf scale)")
    ap.add_argument("--sub-cull", action="store_true",
                    help="sub-leaf culling (32 x 32 sub-products inside 64 x 64 leaves); "
                         "value and roofline then count the performed sub-products")
    ap.add_argument("--low-tol", type=float, default=0.8192,
                    help="split precision: absolute LOW threshold on the norm product")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense FP32 GEMM context of the same matrix")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the epsilon-sparsified tree comparison")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving run that follows the main workload")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-budget-gib", type=float, default=96.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the SpAMM path here is single-device "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    if args.serve:
        return serve_main(args)

    import numpy as np
    import torch

    import paper_1203_1692_amd as sp
    import workloads

    wl = workloads.WORKLOADS[args.workload]
    tau = wl.tau if args.tau is None else args.tau
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sp.load()

    t_gen = time.perf_counter()
    A = wl.matrix()
    t_gen = time.perf_counter() - t_gen
    n, leaf = wl.n, wl.leaf
    dA = torch.from_numpy(A).to(dev)
    C = torch.empty_like(dA)
    torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    split = args.precision != "fp32"
    f16 = args.precision == "split-fp16"
    prec = sp.PREC_SPLIT_FP16 if f16 else sp.PREC_SPLIT_BF16 if split else sp.PREC_FP32
    sub = args.sub_cull
    if sub and (split or leaf != 64):
        print("--sub-cull needs FP32 precision and a 64 x 64 leaf workload", file=sys.stderr)
        return 2
    if sub:
        # the other legs compare against the whole-leaf product: not run here
        args.no_sparse = args.no_matched_error = args.no_cpu_baseline = True

    def step():
        tree = sp.build_tree(dA, leaf, bf16=split and not f16, fp16=f16,
                             subnorms=sub)                            # syncs once (root norm)
        st = sp.multiply_ex(tree, tree, tau, C, precision=prec,
                            low_tol=args.low_tol if split else 0.0,
                            sub_cull=sub)                             # events around cull and GEMM
        tree.free()
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    ms_step = (t1 - t0) * 1e3 / args.steps
    st = stats[-1]
    flops = st["flops"]    # with sub-leaf culling: 2 * 32^3 per performed sub-product
    K = st["tasks"]
    gemm_ms = sum(s["numeric_ms"] for s in stats) / len(stats)
    cull_ms = sum(s["symbolic_ms"] for s in stats) / len(stats)
    value = flops / (ms_step * 1e-3) / 1e12
    gemm_tflops = flops / (gemm_ms * 1e-3) / 1e12

    # ---- error on sampled output leaves -------------------------------------
    d = st["depth"]
    N = 1 << d
    tiles = sample_tiles(N, args.sample_tiles)
    Ch = C.cpu().numpy()
    err_exact = 0.0
    for (I, J) in tiles:
        r0, r1 = I * leaf, min((I + 1) * leaf, n)
        c0, c1 = J * leaf, min((J + 1) * leaf, n)
        if r0 >= n or c0 >= n:
            continue
        exact = A[r0:r1].astype(np.float64) @ A[:, c0:c1].astype(np.float64)
        err_exact = max(err_exact, float(np.abs(Ch[r0:r1, c0:c1] - exact).max()))

    out = {
        "metric": "kept-tile TFLOP/s (2 n_b^3 K per step / step time)",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": wl.name, "n": n, "n_padded": leaf << d, "leaf": leaf, "tau": tau,
            "depth": d, "kept_tasks": K, "kept_per_tier": st["kept"],
            "kept_fraction": K / float(N) ** 3, "block_entries": st["block_entries"],
            "ms_multiply": round(cull_ms + gemm_ms, 3), "ms_cull": round(cull_ms, 3),
            "ms_leaf_gemm": round(gemm_ms, 3),
            "ms_build": round(ms_step - cull_ms - gemm_ms, 3),
            "max_norm_err_vs_fp64_dense_sampled": err_exact,
            "error_sample_tiles": len(tiles),
            "effective_tflops_2n3": round(2.0 * n ** 3 / (ms_step * 1e-3) / 1e12, 3),
        },
        "roofline": {
            "bound": "mfma",
            "achieved": round(gemm_tflops, 3),
            "peak": MFMA_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(gemm_tflops / MFMA_FP32_PEAK_TFLOPS, 4),
            "traffic": measured_traffic(wl.name),
        },
    }
    if sub:
        out["config"]["sub_cull"] = True
        out["config"]["sub_products"] = st["subtasks"]
        out["config"]["flops_counted"] = "2 * 32^3 per performed 32 x 32 sub-product"
        out["roofline"]["traffic"] = measured_sub_traffic(wl.name, tau)
    if split:
        # the split kernel moves whole 16-bit leaves: rate it against HBM
        tb = measured_split_traffic(wl.name, tau, args.low_tol, "fp16" if f16 else "bf16")
        gbs = tb / (gemm_ms * 1e-3) / 1e9 if tb is not None else None
        out["dtype"] = "f32+f16" if f16 else "f32+bf16"
        out["config"]["precision"] = "split-fp16" if f16 else "split-bf16"
        out["config"]["low_tol"] = args.low_tol
        out["config"]["tasks_low"] = st["tasks_low"]
        out["roofline"] = {
            "bound": "hbm", "achieved": round(gbs, 1) if gbs else None, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None, "traffic": tb,
        }

    # ---- context: the dense FP32 product of the same matrix (torch.matmul) ------
    # the paper's cross-over against SGEMM; not part of the timed step
    if not args.no_dense and not split and not sub:
        D = torch.empty_like(C)
        torch.matmul(dA, dA, out=D)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(2):
            torch.matmul(dA, dA, out=D)
        ev[1].record()
        torch.cuda.synchronize()
        dense_ms = ev[0].elapsed_time(ev[1]) / 2
        del D
        spamm_ms = cull_ms + gemm_ms
        out["dense_fp32_context"] = {
            "op": "torch.matmul (FP32, rocBLAS/hipBLASLt) of the same n x n matrix",
            "ms": round(dense_ms, 3), "tflops": round(2.0 * n ** 3 / (dense_ms * 1e-3) / 1e12, 3),
            "spamm_ms_multiply": round(spamm_ms, 3),
            "spamm_speedup": round(dense_ms / spamm_ms, 3),
        }

    # ---- epsilon-sparsified tree of the same matrix ----------------------------
    # leaves below tau / ||A||_F dropped at build; the product keeps the same
    # leaf products, so C must equal the dense step's bit for bit
    if not args.no_sparse:
        C2 = torch.empty_like(C)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sparse = sp.build_tree_sparse(dA, leaf, tau)
        torch.cuda.synchronize()
        t_build = (time.perf_counter() - t) * 1e3
        sst = sp.multiply_ex(sparse, sparse, tau, C2)
        sto = sparse.storage()
        dense_bytes = sp.build_tree(dA, leaf).storage()["bytes"]
        out["sparse_tree"] = {
            "tau": tau, "leaves_stored": sto["stored"], "leaves_total": sto["total"],
            "stored_fraction": round(sto["stored"] / sto["total"], 4),
            "device_bytes": sto["bytes"], "dense_device_bytes": dense_bytes,
            "ms_build": round(t_build, 3),
            "ms_multiply": round(sst["symbolic_ms"] + sst["numeric_ms"], 3),
            "tasks": sst["tasks"], "C_bitwise_equal_dense": bool(torch.equal(C, C2)),
        }
        sparse.free()
        del C2

    # ---- FP32 vs split precision at the same max-norm error -------------------
    # The paper compares variants with tau adjusted so that their max-norm
    # errors against the double-precision product match (Sec. IV.B).  Target
    # E* = the error of the FP32 product at the configured tau; for each
    # variant, the fastest grid point whose error is <= E* (errors measured on
    # the same seeded output leaves, dense FP64 reference).
    if not args.no_matched_error:
        out["matched_error"] = matched_error(sp, wl, A, dA, C, tau, leaf, n, N)

    # ---- CPU baseline: the FP64 oracle on the sampled output leaves ----------
    if not args.no_cpu_baseline:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        otiles = sample_tiles(N, args.oracle_tiles, seed=1)
        t = time.perf_counter()
        Ct, counts, _ = oracle.spamm_tiles(A, A, leaf, tau, otiles, threads=threads)
        t = time.perf_counter() - t
        cflops = 2.0 * leaf ** 3 * float(counts.sum())
        err_oracle = 0.0
        for s, (I, J) in enumerate(otiles):
            r0, r1 = I * leaf, min((I + 1) * leaf, n)
            c0, c1 = J * leaf, min((J + 1) * leaf, n)
            if r0 >= n or c0 >= n:
                continue
            err_oracle = max(err_oracle, float(np.abs(
                Ch[r0:r1, c0:c1] - Ct[s, :r1 - r0, :c1 - c0]).max()))
        out["config"]["max_norm_err_vs_oracle_sampled"] = err_oracle
        out["config"]["oracle_sample_tiles"] = len(otiles)
        out["cpu_baseline"] = {
            "value": cflops / t / 1e12,
            "unit": "TFLOP/s",
            "cores": threads,
            "kind": "oracle",
            "sample": (f"{len(otiles)} seeded output leaves of {wl.name} (tau={tau:g}), "
                       f"{int(counts.sum())} kept leaf products, recursive FP64 oracle incl. its "
                       f"full-matrix norm pass, {t:.1f} s wall"),
        }
    # ---- the paper's own figures (single CPU core, FP32 SSE kernels), for
    # context only: another machine and other matrices, never a target -------
    out["paper_context"] = PAPER_CONTEXT
    # ---- serving: a stream of products and squaring chains --------------------
    if not args.no_serve:
        del dA, C
        torch.cuda.empty_cache()
        sv = serve_bench(sp, torch, dev, args.serve_requests, args.serve_slots,
                         args.serve_budget_gib)
        for part in [sv["saturation"], *sv["loads"].values()]:
            part.pop("by_n", None)
        out["serving"] = sv
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
