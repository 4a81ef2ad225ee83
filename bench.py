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
oracle on a seeded sample of output leaves of the same matrix.
`matched_error` compares FP32 with the split precisions (BF16, BF16 with
compensated HIGH products, FP16) and sub-leaf culling at the FP32 product's
own whole-matrix error.  `serving`
then drives a stream of 2000 products and squaring chains of uneven size
through the continuous-batching server: saturation throughput, and p50/p99
latency under Poisson arrivals at 0.5x and 0.8x of it (`--serve` runs only
that, `--no-serve` skips it).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_FP32_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
MFMA_16BIT_PEAK_TFLOPS = 2516.6 # MI355X dense BF16 / FP16 matrix peak
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


def code_only(text: str) -> str:
    """C++ source without its comments, trailing blanks and empty lines
    (string and character literals kept whole): what the compiler sees."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    lines = (line.rstrip() for line in "".join(out).split("\n"))
    return "\n".join(line for line in lines if line)


def kernel_source_digest() -> str:
    """SHA-256 over the leaf GEMM's source and its layout header (code only:
    a comment edit does not change the kernel the counters were taken on) and
    the build flags file (every byte)."""
    h = hashlib.sha256()
    for rel in GEMM_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            data = f.read()
        if not rel.endswith(".py"):
            data = code_only(data.decode("utf-8")).encode("utf-8")
        h.update(data)
    return h.hexdigest()


def gemm_kernel_name(precision: str, leaf: int, depth: int, sub: bool = False) -> str:
    """The leaf-GEMM kernel the library picks for a product (its plan's kind)."""
    if sub:
        return "leaf_gemm_sub_wide" if depth >= 2 else "leaf_gemm_sub<64>"
    if precision == "split-bf16":
        return ("leaf_gemm_split_wide<false>" if leaf == 64 and depth >= 2
                else f"leaf_gemm_split<{leaf}, false, false>")
    if precision == "split-bf16x3":
        return ("leaf_gemm_split_wide<true>" if leaf == 64 and depth >= 2
                else f"leaf_gemm_split<{leaf}, false, true>")
    if precision == "split-fp16":
        return f"leaf_gemm_split<{leaf}, true, false>"
    return "leaf_gemm_wide32" if leaf == 64 and depth >= 2 else f"leaf_gemm<{leaf}>"


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


def measured_split_traffic(workload: str, tau: float, theta: float, fmt: str = "bf16"):
    """HBM bytes per launch of the split kernel (LOW operands in `fmt`) at
    (tau, theta) from the committed counter runs, or None when absent or the
    kernel sources changed since."""
    import glob
    kind = {"bf16": "leaf_gemm_split", "fp16": "leaf_gemm_split_fp16",
            "bf16x3": "leaf_gemm_split_x3"}[fmt]
    # one record per measured (tau, theta): <kind>_<workload>[_<point>]_traffic.json
    digest = kernel_source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles",
                                              f"{kind}_{workload}*_traffic.json"))):
        t = json.load(open(path))
        if (t.get("gemm_sources_sha256") == digest and
                abs(t.get("tau", -1.0) - tau) <= 1e-12 * tau and
                abs(t.get("theta", -1.0) - theta) <= 1e-12 * theta):
            return t["bytes_per_launch"]
    return None


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


def dense_fp64(torch, dA, dB=None):
    """The exact reference of Eq. matrix error: the dense product in FP64 on
    the device (each FP32 entry widened exactly; rounding error ~n 2^-53)."""
    A64 = dA.double()
    B64 = A64 if dB is None else dB.double()
    out = A64 @ B64
    del A64, B64
    return out


def max_err_full(C, exact, chunk: int = 4096) -> float:
    """max |C - exact| over every element of the n x n product."""
    e = 0.0
    for r in range(0, C.shape[0], chunk):
        e = max(e, float((C[r:r + chunk].double() - exact[r:r + chunk]).abs().max()))
    return e


def timed_product(sp, tree, tau, C, reps, precision=0, low_rel=0.0, sub_cull=False):
    """Best-of-reps cull + leaf GEMM time (HIP events) and the last stats."""
    best = None
    for _ in range(reps):
        st = sp.multiply_ex(tree, tree, tau, C, precision=precision, low_rel=low_rel,
                            sub_cull=sub_cull)
        ms = st["symbolic_ms"] + st["numeric_ms"]
        if best is None or ms < best[0]:
            best = (ms, st["numeric_ms"], st["symbolic_ms"])
    return best, st


THETAS = (1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7)     # relative split thresholds
TARGETS = (1e-5, 1e-6)                                   # fixed max-norm errors


def fastest_within(points, kind, target):
    ok = [p for p in points if p["precision"] == kind and p["err"] <= target]
    return min(ok, key=lambda p: p["ms"]) if ok else None


def refine_candidates(points, kinds, target):
    """(kind, tau, theta) of the quarter-decade neighbours (tau x 10^{-1/4,
    0, 1/4}, and theta alike when the kind has one) of each kind's fastest
    point within `target`, without the centre and without points already
    measured."""
    seen = {(p["precision"], p["tau"], p["theta"]) for p in points}
    todo = []
    for k in kinds:
        b = fastest_within(points, k, target)
        if b is None:
            continue
        for dt in (-1, 0, 1):
            for dh in ((-1, 0, 1) if b["theta"] else (0,)):
                key = (k, b["tau"] * 10.0 ** (dt / 4),
                       b["theta"] * 10.0 ** (dh / 4) if b["theta"] else 0.0)
                if (dt or dh) and key not in seen:
                    todo.append(key)
                    seen.add(key)
    return todo


def matched_error(sp, torch, wl, dA, C, exact, tau, leaf, reps=2):
    """FP32 against split precision (and sub-leaf culling) at the same
    max-norm error (Sec. IV.B, Sec. V.C: tolerances adjusted per variant until
    the errors of Eq. matrix error match).  Every grid point's error is taken
    over the whole matrix against the dense FP64 product.  Targets: the FP32
    product's own error at the configured tau, and 1e-5 and 1e-6."""
    taus = [tau * 10.0 ** (h / 2) for h in range(11)]       # tau x 10^{0, 0.5, ..., 5}
    points = []
    tree = sp.build_tree(dA, leaf, bf16=True)
    for t_ in taus:
        (ms, g_ms, _), st = timed_product(sp, tree, t_, C, reps)
        points.append({"precision": "fp32", "tau": t_, "theta": 0.0, "ms": round(ms, 3),
                       "ms_leaf_gemm": round(g_ms, 3), "err": max_err_full(C, exact),
                       "tasks": st["tasks"], "low_frac": 0.0})
        for th in THETAS:
            for kind, prec in (("split-bf16", sp.PREC_SPLIT_BF16),
                               ("split-bf16x3", sp.PREC_SPLIT_BF16X3)):
                (ms, g_ms, _), st = timed_product(sp, tree, t_, C, reps, prec, th)
                points.append({"precision": kind, "tau": t_, "theta": th, "ms": round(ms, 3),
                               "ms_leaf_gemm": round(g_ms, 3), "err": max_err_full(C, exact),
                               "tasks": st["tasks"],
                               "low_frac": round(st["tasks_low"] / max(1, st["tasks"]), 4)})
    tree.free()
    tree = sp.build_tree(dA, leaf, fp16=True)
    for t_ in taus:
        for th in THETAS:
            (ms, g_ms, _), st = timed_product(sp, tree, t_, C, reps, sp.PREC_SPLIT_FP16, th)
            points.append({"precision": "split-fp16", "tau": t_, "theta": th, "ms": round(ms, 3),
                           "ms_leaf_gemm": round(g_ms, 3), "err": max_err_full(C, exact),
                           "tasks": st["tasks"],
                           "low_frac": round(st["tasks_low"] / max(1, st["tasks"]), 4)})
    tree.free()
    if leaf == 64:
        # sub-leaf culling: 32 x 32 sub-products tested inside each 64 x 64 one
        sub_tree = sp.build_tree(dA, leaf, subnorms=True)
        for h in range(-2, 10):                                # tau x 10^{-1, ..., 4.5}
            t_ = tau * 10.0 ** (h / 2)
            (ms, g_ms, _), st = timed_product(sp, sub_tree, t_, C, reps, sub_cull=True)
            points.append({"precision": "fp32-subleaf", "tau": t_, "theta": 0.0,
                           "ms": round(ms, 3), "ms_leaf_gemm": round(g_ms, 3),
                           "err": max_err_full(C, exact), "tasks": st["tasks"],
                           "sub_products": st["subtasks"],
                           "sub_fraction": round(st["subtasks"] / max(1, 8 * st["tasks"]), 4)})
        sub_tree.free()
    floor = next(p["err"] for p in points if p["precision"] == "fp32" and p["tau"] == tau)
    kinds = ("fp32", "split-bf16", "split-bf16x3", "split-fp16", "fp32-subleaf")
    # refinement: the paper adjusts each variant's tolerances until the errors
    # match; around each variant's fastest grid point within the FP32
    # product's error, its quarter-decade neighbours in tau (and theta)
    todo = refine_candidates(points, kinds, floor)
    trees = {}
    for k, t_, th in todo:
        kw = ({"fp16": True} if k == "split-fp16" else
              {"subnorms": True} if k == "fp32-subleaf" else {"bf16": True})
        name = next(iter(kw))
        if name not in trees:
            trees[name] = sp.build_tree(dA, leaf, **kw)
        prec = {"fp32": 0, "split-bf16": sp.PREC_SPLIT_BF16, "split-bf16x3": sp.PREC_SPLIT_BF16X3,
                "split-fp16": sp.PREC_SPLIT_FP16, "fp32-subleaf": 0}[k]
        (ms, g_ms, _), st = timed_product(sp, trees[name], t_, C, reps, prec, th,
                                          sub_cull=k == "fp32-subleaf")
        pt = {"precision": k, "tau": t_, "theta": th, "ms": round(ms, 3),
              "ms_leaf_gemm": round(g_ms, 3), "err": max_err_full(C, exact),
              "tasks": st["tasks"], "refined": True}
        if k == "fp32-subleaf":
            pt.update(sub_products=st["subtasks"],
                      sub_fraction=round(st["subtasks"] / max(1, 8 * st["tasks"]), 4))
        else:
            pt["low_frac"] = round(st["tasks_low"] / max(1, st["tasks"]), 4)
        points.append(pt)
    for t in trees.values():
        t.free()

    def at(target):
        best = {k: fastest_within(points, k, target) for k in kinds}
        f32 = best["fp32"]
        out = {"target_err": target, "fastest": best,
               "speedup_vs_fp32": {k: (round(f32["ms"] / best[k]["ms"], 3)
                                       if f32 and best[k] else None) for k in kinds[1:]}}
        if f32 is None:
            out["note"] = ("no FP32 point reaches this error: at tau = %g the FP32 product's own "
                           "rounding leaves %.3g" % (tau, floor))
        return out

    res = {"err_reference": "whole matrix, max-norm, against the dense FP64 product (Eq. matrix "
                            "error)",
           "fp32_error_at_tau": floor,
           "at_fp32_error": at(floor),
           "at_targets": {f"{t:g}": at(t) for t in TARGETS},
           "grid": "tau x 10^{0, 0.5, ..., 5}; theta in %s for the three split formats "
                   "(BF16, BF16 with compensated HIGH products, FP16); sub-leaf culling "
                   "tau x 10^{-1, -0.5, ..., 4.5}; then, around each variant's fastest point "
                   "within the FP32 product's error, its neighbours at tau x 10^{+-1/4} "
                   "(and theta x 10^{+-1/4}): %d more points" % (list(THETAS), len(todo))}
    plain = next(p for p in points if p["precision"] == "fp32" and p["tau"] == tau)
    sub = [p for p in points if p["precision"] == "fp32-subleaf" and p["tau"] == tau]
    if sub:
        res["subleaf_same_tau"] = {"tau": tau, "leaf_products": plain["tasks"],
                                   "sub_products": sub[0]["sub_products"],
                                   "sub_fraction": sub[0]["sub_fraction"],
                                   "ms_plain": plain["ms"], "ms_subleaf": sub[0]["ms"],
                                   "err_plain": plain["err"], "err_subleaf": sub[0]["err"]}
    m = res["at_fp32_error"]["fastest"]
    depth = max(0, math.ceil(math.log2(wl.n / leaf))) if wl.n > leaf else 0
    for kind, fmt in (("split-bf16", "bf16"), ("split-bf16x3", "bf16x3"),
                      ("split-fp16", "fp16")):
        pt = m.get(kind)
        if pt is None:
            continue
        tb = measured_split_traffic(wl.name, pt["tau"], pt["theta"], fmt)
        if tb is not None:
            gbs = tb / (pt["ms_leaf_gemm"] * 1e-3) / 1e9
            # and against the matrix units: LOW products at the dense 16-bit
            # peak, HIGH ones at the FP32 one (compensated: three products at
            # the 16-bit peak)
            low = pt["tasks"] * pt["low_frac"]
            high_s = ((pt["tasks"] - low) * 3 / (MFMA_16BIT_PEAK_TFLOPS * 1e12)
                      if fmt == "bf16x3" else (pt["tasks"] - low) / (MFMA_FP32_PEAK_TFLOPS * 1e12))
            mfma_ms = 2.0 * leaf ** 3 * (low / (MFMA_16BIT_PEAK_TFLOPS * 1e12) + high_s) * 1e3
            res[f"{kind}_roofline"] = {
                "kernel": gemm_kernel_name(kind, leaf, depth), "bound": "hbm",
                "achieved": round(gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": tb,
                "mfma_ideal_ms": round(mfma_ms, 3),
                "mfma_frac": round(mfma_ms / pt["ms_leaf_gemm"], 4)}
    return res


def run_config(sp, torch, dev, name, reps, tau=None, precisions=((0, 0.0),), with_exact=True):
    """One of the other configurations of the benchmark: build + product timed
    with HIP events per stage (best of `reps`), kept-leaf TFLOP/s on the
    multiply and the whole step, the cull's share, and the whole-matrix
    max-norm error against the dense FP64 product."""
    import workloads
    wl = workloads.WORKLOADS[name]
    A = wl.matrix()
    dA = torch.from_numpy(A).to(dev)
    C = torch.empty_like(dA)
    exact = dense_fp64(torch, dA) if with_exact else None
    out = {"workload": wl.name, "n": wl.n, "leaf": wl.leaf, "points": []}
    for t_ in ([tau] if tau is not None else list(wl.taus)):
        for prec, th in precisions:
            kw = dict(bf16=prec == sp.PREC_SPLIT_BF16, fp16=prec == sp.PREC_SPLIT_FP16)
            tb = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                tree = sp.build_tree(dA, wl.leaf, **kw)
                tb.append((time.perf_counter() - t0) * 1e3)
                if _ < reps - 1:
                    tree.free()
            (ms, g_ms, c_ms), st = timed_product(sp, tree, t_, C, reps, prec, th)
            tree.free()
            flops = st["flops"]
            pt = {"precision": {0: "fp32", 1: "split-bf16", 2: "split-fp16",
                                3: "split-bf16x3"}[prec], "tau": t_,
                  "theta": th, "tasks": st["tasks"], "tasks_low": st["tasks_low"],
                  "ms_build": round(min(tb), 4), "ms_cull": round(c_ms, 4),
                  "ms_leaf_gemm": round(g_ms, 4), "ms_multiply": round(ms, 4),
                  "cull_share": round(c_ms / ms, 4) if ms > 0 else None,
                  "kept_tile_tflops_multiply": round(flops / (ms * 1e-3) / 1e12, 3),
                  "kept_tile_tflops_step": round(flops / ((ms + min(tb)) * 1e-3) / 1e12, 3)}
            if exact is not None:
                pt["max_norm_err_vs_fp64_dense"] = max_err_full(C, exact)
            out["points"].append(pt)
    del dA, C, exact
    torch.cuda.empty_cache()
    return out


def algdecay_sweep(sp, torch, dev, reps):
    """The tau sweep of algdecay-n16384: plain FP32 against split BF16 (with
    FP32 or compensated HIGH products) at theta = 1e-4 at each configured
    tau, and FP32 against the three split formats
    at the fixed errors 1e-5 and 1e-6 (tau on a 10^{1/2} grid from 1e-10 to
    1e-4, theta from 1e-4 to 1e-9)."""
    import workloads
    wl = workloads.WORKLOADS["algdecay-n16384"]
    dA = torch.from_numpy(wl.matrix()).to(dev)
    C = torch.empty_like(dA)
    exact = dense_fp64(torch, dA)
    tree = sp.build_tree(dA, wl.leaf, bf16=True)
    sweep = []
    for t_ in wl.taus:
        row = {"tau": t_}
        for kind, prec, th in (("fp32", 0, 0.0), ("split-bf16", sp.PREC_SPLIT_BF16, 1e-4),
                               ("split-bf16x3", sp.PREC_SPLIT_BF16X3, 1e-4)):
            (ms, g_ms, c_ms), st = timed_product(sp, tree, t_, C, reps, prec, th)
            row[kind] = {"ms": round(ms, 4), "ms_cull": round(c_ms, 4),
                         "ms_leaf_gemm": round(g_ms, 4), "tasks": st["tasks"],
                         "tasks_low": st["tasks_low"], "err": max_err_full(C, exact)}
        row["speedup_split"] = round(row["fp32"]["ms"] / row["split-bf16"]["ms"], 3)
        row["speedup_split_x3"] = round(row["fp32"]["ms"] / row["split-bf16x3"]["ms"], 3)
        sweep.append(row)
    points = []
    thetas = [10.0 ** -e for e in range(4, 10)]                # 1e-4 ... 1e-9
    t16 = sp.build_tree(dA, wl.leaf, fp16=True)
    for h in range(13):                                       # tau = 1e-10 ... 1e-4
        t_ = 1e-10 * 10.0 ** (h / 2)
        runs = [("fp32", tree, 0, 0.0)]
        runs += [("split-bf16", tree, sp.PREC_SPLIT_BF16, th) for th in thetas]
        runs += [("split-bf16x3", tree, sp.PREC_SPLIT_BF16X3, th) for th in thetas]
        runs += [("split-fp16", t16, sp.PREC_SPLIT_FP16, th) for th in thetas]
        for kind, tr, prec, th in runs:
            (ms, g_ms, _), st = timed_product(sp, tr, t_, C, reps, prec, th)
            points.append({"precision": kind, "tau": t_, "theta": th, "ms": round(ms, 4),
                           "err": max_err_full(C, exact), "tasks": st["tasks"],
                           "tasks_low": st["tasks_low"]})
    tree.free()
    t16.free()
    # epsilon-sparsified trees (leaves below tau / ||A||_F not stored) at each
    # configured tau: storage and product time against the dense tree, C
    # bitwise equal
    sparse = []
    dense_tree = sp.build_tree(dA, wl.leaf)
    dense_bytes = dense_tree.storage()["bytes"]
    C2 = torch.empty_like(C)
    for t_ in wl.taus:
        sp.multiply_ex(dense_tree, dense_tree, t_, C)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_tree = sp.build_tree_sparse(dA, wl.leaf, t_)
        torch.cuda.synchronize()
        t_build = (time.perf_counter() - t0) * 1e3
        (ms, g_ms, _), st = timed_product(sp, st_tree, t_, C2, reps)
        (ms_d, _, _), _ = timed_product(sp, dense_tree, t_, C, reps)
        sto = st_tree.storage()
        sparse.append({"tau": t_, "leaves_stored": sto["stored"], "leaves_total": sto["total"],
                       "stored_fraction": round(sto["stored"] / sto["total"], 4),
                       "device_bytes": sto["bytes"], "dense_device_bytes": dense_bytes,
                       "ms_build_host_timed": round(t_build, 3), "ms_multiply": round(ms, 4),
                       "ms_multiply_dense_tree": round(ms_d, 4),
                       "C_bitwise_equal_dense": bool(torch.equal(C, C2))})
        st_tree.free()
    dense_tree.free()
    del C2
    matched = {}
    for target in TARGETS:
        kinds = ("fp32", "split-bf16", "split-bf16x3", "split-fp16")
        best = {k: fastest_within(points, k, target) for k in kinds}
        f32 = best["fp32"]
        best["speedup_vs_fp32"] = {k: (round(f32["ms"] / best[k]["ms"], 3)
                                       if f32 and best[k] else None)
                                   for k in kinds[1:]}
        matched[f"{target:g}"] = best
    del dA, C, exact
    torch.cuda.empty_cache()
    return {"workload": wl.name, "n": wl.n, "leaf": wl.leaf, "tau_sweep": sweep,
            "matched_error": matched, "sparse_tree": sparse,
            "error": "whole matrix, max-norm, against the dense FP64 product"}


def write_traffic_record(args) -> int:
    """HBM bytes per launch of one kernel from two rocprofv3 --pmc runs of the
    same bench command with --copy-calibration: the FETCH_SIZE and
    WRITE_SIZE counters (KiB per dispatch) of the kernel, each scaled by
    true / counted bytes of the three 1 GiB device copies of that run."""
    import csv
    kernel, fcsv, wcsv = args.traffic_record

    def rows(path, counter):
        out = []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") == counter:
                    out.append((r["Kernel_Name"], float(r["Counter_Value"]),
                                int(r.get("Grid_Size", 0) or 0)))
        return out

    rec = {"kernel": kernel, "gemm_sources_sha256": kernel_source_digest(),
           "copy_calibration_KiB": {"true": 1 << 20}, "scale": {},
           "kernel_KiB_per_dispatch": {}}
    for counter, path in (("FETCH_SIZE", fcsv), ("WRITE_SIZE", wcsv)):
        rs = rows(path, counter)
        # the three 1 GiB device copies: a grid of 131072 work items each
        copies = [v for k, v, g in rs if "copyBuffer" in k and g == 131072]
        if len(copies) != 3:
            copies = [v for k, v, g in rs
                      if "copyBuffer" in k and 0.4 * (1 << 20) <= v <= 2.5 * (1 << 20)]
        ker = [v for k, v, g in rs if k.startswith(kernel) or ("::" + kernel) in k]
        if not copies or not ker:
            print(f"{counter}: copies {len(copies)}, {kernel} dispatches {len(ker)}",
                  file=sys.stderr)
            return 1
        cal = sum(copies) / len(copies)
        rec["copy_calibration_KiB"][counter] = cal
        rec["scale"][counter] = (1 << 20) / cal
        rec["kernel_KiB_per_dispatch"][counter] = sum(ker) / len(ker)
    rd = rec["kernel_KiB_per_dispatch"]["FETCH_SIZE"] * rec["scale"]["FETCH_SIZE"] * 1024
    wr = rec["kernel_KiB_per_dispatch"]["WRITE_SIZE"] * rec["scale"]["WRITE_SIZE"] * 1024
    rec.update(read_bytes_per_launch=rd, write_bytes_per_launch=wr, bytes_per_launch=rd + wr)
    for k in ("workload", "tau") + (("theta",) if "split" in kernel else ()):
        if getattr(args, k, None) is not None:
            rec[k] = getattr(args, k)
    out = args.record_out or os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))
    return 0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_single_core_c1() -> dict:
    """The full FP64 oracle at expdecay-n1024 on one core (the paper times one
    pinned core): a child process with one OpenMP thread and one CPU."""
    import subprocess
    code = ("import os, sys, time, json; sys.path.insert(0, %r); os.sched_setaffinity(0, "
            "{sorted(os.sched_getaffinity(0))[0]}); import workloads, oracle; "
            "wl = workloads.WORKLOADS['expdecay-n1024']; A = wl.matrix(); ts = []\n"
            "for _ in range(3):\n t = time.perf_counter(); r = oracle.spamm(A, A, wl.leaf, wl.tau, "
            "want_keys=False); ts.append(time.perf_counter() - t)\n"
            "print(json.dumps({'K': r.K, 's': sorted(ts)[1]}))" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    flops = 2.0 * 32 ** 3 * d["K"]
    return {"workload": "expdecay-n1024", "tau": 1e-6, "threads": 1, "kind": "oracle",
            "ms": round(d["s"] * 1e3, 2), "gflops": round(flops / d["s"] / 1e9, 4),
            "note": "full recursive FP64 oracle (norms + product), median of 3, one pinned core"}


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
    grew = {k: info1[k] - info0[k] for k in ("launches", "launched_products", "rounds",
                                              "round_steps")}
    return out, kept, dict(t0=t0, t_first=t_first, t_last=t_last, t_end=t_end, sched_busy=busy,
                           **grew)


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
        # shared launches: GEMM launch groups, and rounds of tree builds + culls
        "gemm_launch_groups": tm.get("launches"),
        "products_per_gemm_group": (round(tm["launched_products"] / tm["launches"], 3)
                                    if tm.get("launches") else None),
        "rounds": tm.get("rounds"),
        "steps_per_round": (round(tm["round_steps"] / tm["rounds"], 3)
                            if tm.get("rounds") else None),
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


def serve_one_call_concurrent(sp, torch, reqs, inputs, threads=16):
    """The same requests through the one-call API from `threads` host
    threads, each on a stream of its own (tree build, which reads back the
    root norm, then an asynchronous product per step; one synchronization
    per request): the plain GPU form used concurrently."""
    import threading
    from workloads import SERVE_LEAF, SERVE_THETA
    dev = torch.cuda.current_device()
    errors = []

    def worker(k):
        try:
            torch.cuda.set_device(dev)
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for req in reqs[k::threads]:
                    X = inputs[req.index]
                    prec = sp.PREC_SPLIT_BF16 if req.split else sp.PREC_FP32
                    for _ in range(max(1, req.chain_len)):
                        t = sp.build_tree(X, SERVE_LEAF, stream=st, bf16=req.split)
                        C = torch.empty_like(X)
                        sp.multiply_ex(t, t, req.tau, C, stream=st, precision=prec,
                                       low_rel=SERVE_THETA if req.split else 0.0, stats=False)
                        t.free()
                        X = C
                    st.synchronize()
        except Exception as e:        # reported below
            errors.append(repr(e))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ths = [threading.Thread(target=worker, args=(k,)) for k in range(threads)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"requests_per_s": round(len(reqs) / wall, 2), "wall_s": round(wall, 3),
            "threads": threads, "errors": errors[:3],
            "note": f"{threads} host threads on {threads} streams, each request through "
                    "spamm_build_tree + asynchronous spamm_multiply_opts per step"}


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
    conc = serve_one_call_concurrent(sp, torch, reqs, inputs)
    print(f"one-call API, 16 threads: {conc['requests_per_s']} req/s",
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
        "one_call_concurrent": conc,
        "served_speedup_vs_one_call_concurrent":
            round(sat["throughput_rps"] / conc["requests_per_s"], 3),
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
    ap.add_argument("--oracle-tiles", type=int, default=3072,
                    help="output leaves computed by the FP64 oracle (CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--no-matched-error", action="store_true",
                    help="skip the FP32-vs-split comparison at a fixed max-norm error")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark instead: saturation, then Poisson arrivals")
    ap.add_argument("--precision", choices=("fp32", "split", "split-x3", "split-fp16"),
                    default="fp32",
                    help="product of the timed steps (split: BF16 for LOW products, "
                         "split-x3: also compensated BF16 HIGH products, "
                         "split-fp16: FP16 at a per-leaf scale)")
    ap.add_argument("--sub-cull", action="store_true",
                    help="sub-leaf culling (32 x 32 sub-products inside 64 x 64 leaves); "
                         "value and roofline then count the performed sub-products")
    ap.add_argument("--theta", type=float, default=1e-4,
                    help="split precision: LOW iff the norm product < theta ||A||_F ||B||_F")
    ap.add_argument("--no-error", action="store_true",
                    help="skip the whole-matrix error against the dense FP64 product (and the "
                         "matched-error comparison that needs it): short profiler runs")
    ap.add_argument("--traffic-record", nargs=3, metavar=("KERNEL", "FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic record of KERNEL from two rocprofv3 --pmc "
                         "counter CSVs (FETCH_SIZE, WRITE_SIZE) of one bench run with "
                         "--copy-calibration, then exit (no GPU)")
    ap.add_argument("--record-out", default=None, help="path of the traffic record")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (expdecay-n1024, cluster300-n7500, "
                         "the algdecay-n16384 tau sweep)")
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

    if args.traffic_record:
        return write_traffic_record(args)

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
    x3 = args.precision == "split-x3"
    prec = (sp.PREC_SPLIT_FP16 if f16 else sp.PREC_SPLIT_BF16X3 if x3
            else sp.PREC_SPLIT_BF16 if split else sp.PREC_FP32)
    split_kind = "split-fp16" if f16 else "split-bf16x3" if x3 else "split-bf16"
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
                            low_rel=args.theta if split else 0.0,
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

    # ---- error over the whole matrix against the dense FP64 product ----------
    d = st["depth"]
    N = 1 << d
    Ch = C.cpu().numpy()
    exact = None if args.no_error else dense_fp64(torch, dA)
    err_exact = None if exact is None else max_err_full(C, exact)

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
            "max_norm_err_vs_fp64_dense": err_exact,
            "error_reference": "every element of C against the dense FP64 product on the GPU",
            "effective_tflops_2n3": round(2.0 * n ** 3 / (ms_step * 1e-3) / 1e12, 3),
        },
        "roofline": {
            "kernel": gemm_kernel_name("fp32", leaf, d, sub),
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
        tb = measured_split_traffic(wl.name, tau, args.theta,
                                    "fp16" if f16 else "bf16x3" if x3 else "bf16")
        gbs = tb / (gemm_ms * 1e-3) / 1e9 if tb is not None else None
        out["dtype"] = "f32+f16" if f16 else "bf16" if x3 else "f32+bf16"
        out["config"]["precision"] = split_kind
        out["config"]["theta"] = args.theta
        out["config"]["tasks_low"] = st["tasks_low"]
        out["roofline"] = {
            "kernel": gemm_kernel_name(split_kind, leaf, d),
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
    if not args.no_matched_error and exact is not None:
        out["matched_error"] = matched_error(sp, torch, wl, dA, C, exact, tau, leaf)
    del exact
    torch.cuda.empty_cache()

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
            "threads": threads,
            "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": (f"{len(otiles)} seeded output leaves of {wl.name} (tau={tau:g}), "
                       f"{int(counts.sum())} kept leaf products, recursive FP64 oracle incl. its "
                       f"full-matrix norm pass, {t:.1f} s wall on {threads} OpenMP threads"),
            "single_core_full_c1": oracle_single_core_c1(),
        }
    # ---- the other configurations: the small case, the n = 7500 cluster and
    # the algebraic-decay tau sweep (plain FP32 against split BF16) -----------
    if not args.no_configs and not sub:
        del dA, C
        torch.cuda.empty_cache()
        out["configs"] = {
            "expdecay-n1024": run_config(sp, torch, dev, "expdecay-n1024", reps=20),
            "cluster300-n7500": run_config(sp, torch, dev, "cluster300-n7500", reps=10),
            "algdecay-n16384": algdecay_sweep(sp, torch, dev, reps=5),
        }
        print("configs done", file=sys.stderr, flush=True)
    # ---- the paper's own figures (single CPU core, FP32 SSE kernels), for
    # context only: another machine and other matrices, never a target -------
    out["paper_context"] = PAPER_CONTEXT
    # ---- serving: a stream of products and squaring chains --------------------
    if not args.no_serve:
        dA = C = None
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
