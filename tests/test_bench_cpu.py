"""bench.py's host-side contract, without a GPU: one GPU only (more exits
with a message), the traffic figures are used only for the kernel sources
they were measured on, and the sampling / summary helpers."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_exits_with_a_message(argv, env):
    e = dict(os.environ, **env)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], env=e,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    rec = {"workload": "w", "gemm_sources_sha256": bench.kernel_source_digest(),
           "bytes_per_launch": 1234.0}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(path))
    assert bench.measured_traffic("w") == 1234.0
    assert bench.measured_traffic("other") is None
    path.write_text(json.dumps(dict(rec, gemm_sources_sha256="0" * 64)))
    assert bench.measured_traffic("w") is None
    path.write_text("not json")
    assert bench.measured_traffic("w") is None
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("w") is None


def test_source_digest_covers_the_kernel_and_its_build_flags():
    assert len(bench.kernel_source_digest()) == 64
    assert any(s.endswith("gemm.hip") for s in bench.GEMM_SOURCES)
    assert any(s.endswith("_build.py") for s in bench.GEMM_SOURCES)
    for rel in bench.GEMM_SOURCES:
        assert os.path.exists(os.path.join(ROOT, rel)), rel


def test_committed_split_traffic_records_name_their_point():
    import glob
    for kind, fmt in (("leaf_gemm_split", "bf16"), ("leaf_gemm_split_fp16", "fp16"),
                      ("leaf_gemm_split_x3", "bf16x3")):
        paths = sorted(glob.glob(os.path.join(
            ROOT, "profiles", f"{kind}_cluster1310-n32750*_traffic.json")))
        assert paths
        points = set()
        for path in paths:
            rec = json.load(open(path))
            assert rec["tau"] > 0 and rec["theta"] > 0 and rec["bytes_per_launch"] > 0
            assert rec["workload"] == "cluster1310-n32750"
            assert (rec["tau"], rec["theta"]) not in points
            points.add((rec["tau"], rec["theta"]))
        for tau, theta in points:
            # another point, or other kernel sources, never reuse a record
            if (tau * 10, theta) not in points:
                assert bench.measured_split_traffic("cluster1310-n32750", tau * 10,
                                                    theta, fmt) is None
            assert bench.measured_split_traffic("cluster1310-n32750", tau,
                                                theta * 2, fmt) is None


def test_sample_tiles_distinct_sorted_in_range():
    t = bench.sample_tiles(64, 100, seed=3)
    assert len(t) == 100 and len(set(t)) == 100
    assert t == sorted(t)
    assert all(0 <= i < 64 and 0 <= j < 64 for i, j in t)
    assert bench.sample_tiles(4, 100) == [(i, j) for i in range(4) for j in range(4)]


def test_percentile_and_empty():
    assert bench.percentile([], 50) is None
    assert bench.percentile([1.0, 2.0, 3.0], 50) == 2.0
    assert bench.percentile(list(range(101)), 99) == 99.0


def test_paper_context_is_context_only():
    c = bench.PAPER_CONTEXT
    assert "context only" in c["note"]
    assert c["spamm_numeric_gflops_dense_16x16_blocks"]["AMD Opteron 6168 (1.8 GHz)"] == 8.1
    assert all(v > 0 for v in c["sgemm_gflops_large_n"].values())


def test_committed_sub_traffic_record_names_its_point():
    path = os.path.join(ROOT, "profiles", "leaf_gemm_sub_cluster1310-n32750_traffic.json")
    rec = json.load(open(path))
    assert rec["tau"] > 0 and rec["bytes_per_launch"] > 0
    assert bench.measured_sub_traffic("cluster1310-n32750", rec["tau"] * 10) is None
    assert bench.measured_sub_traffic("other-workload", rec["tau"]) is None


def test_refine_candidates_are_the_quarter_decade_neighbours():
    pts = [
        {"precision": "fp32", "tau": 1e-5, "theta": 0.0, "ms": 9.0, "err": 1.0},
        {"precision": "fp32", "tau": 1e-4, "theta": 0.0, "ms": 5.0, "err": 1.0},     # fastest
        {"precision": "fp32", "tau": 1e-3, "theta": 0.0, "ms": 2.0, "err": 3.0},     # too coarse
        {"precision": "split-bf16", "tau": 1e-4, "theta": 1e-6, "ms": 1.0, "err": 0.5},
        {"precision": "split-bf16", "tau": 1e-4, "theta": 1e-5, "ms": 0.5, "err": 9.0},
        {"precision": "split-fp16", "tau": 1e-4, "theta": 1e-6, "ms": 1.0, "err": 9.0},  # none within
    ]
    got = bench.refine_candidates(pts, ("fp32", "split-bf16", "split-fp16"), 1.0)
    q = 10.0 ** 0.25
    fp32 = sorted(t for k, t, h in got if k == "fp32")
    assert len(fp32) == 2 and abs(fp32[0] * q / 1e-4 - 1) < 1e-12 and abs(fp32[1] / q / 1e-4 - 1) < 1e-12
    assert all(h == 0.0 for k, t, h in got if k == "fp32")
    split = [(t, h) for k, t, h in got if k == "split-bf16"]
    assert len(split) == 8 and (1e-4, 1e-6) not in split
    assert {round(t / 1e-4, 6) for t, h in split} == {round(1 / q, 6), 1.0, round(q, 6)}
    assert not any(k == "split-fp16" for k, t, h in got)
    # a neighbour already measured is not repeated
    pts.append({"precision": "fp32", "tau": 1e-4 * q, "theta": 0.0, "ms": 6.0, "err": 2.0})
    again = bench.refine_candidates(pts, ("fp32",), 1.0)
    assert len(again) == 1


@pytest.mark.parametrize("precision,sub,page", [
    ("fp32", False, "kernels_cluster1310-n32750_trace.md"),
    ("split-bf16", False, "kernels_split_cluster1310-n32750_trace.md"),
    ("split-bf16x3", False, "kernels_split_x3_cluster1310-n32750_trace.md"),
    ("split-fp16", False, "kernels_split_fp16_cluster1310-n32750_trace.md"),
    ("fp32", True, "kernels_subleaf_cluster1310-n32750_trace.md"),
])
def test_reported_kernel_names_are_the_traced_ones(precision, sub, page):
    # the bench reports each variant's roofline under the name rocprofv3
    # printed for the kernel the library launched (leaf 64, depth 9)
    name = bench.gemm_kernel_name(precision, 64, 9, sub)
    text = open(os.path.join(ROOT, "profiles", page)).read()
    assert f"spamm::{name}" in text


def test_code_only_digest_ignores_comments_and_sees_code():
    src = ('// header\n#include "a.h"  // trailing\nint f(int x) {   /* block\n spans */ return x;'
           '\n\n  const char *s = "// kept /* kept */"; char q = \'"\';  \n}\n')
    got = bench.code_only(src)
    assert got == ('#include "a.h"\nint f(int x) {     return x;\n'
                   '  const char *s = "// kept /* kept */"; char q = \'"\';\n}')
    assert bench.code_only(src.replace("header", "other words")) == got
    assert bench.code_only(src.replace("return x", "return -x")) != got
    # a block comment between two tokens keeps them apart
    assert bench.code_only("a/**/b") == "a b"
    # the kernel sources' comments and code are told apart as the compiler
    # would: nothing after stripping looks like a comment opener outside a string
    for rel in bench.GEMM_SOURCES:
        if rel.endswith(".py"):
            continue
        code = bench.code_only(open(os.path.join(ROOT, rel)).read())
        assert "//" not in code and "/*" not in code


def test_code_only_agrees_with_the_preprocessors_comment_removal():
    import re
    import shutil
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    for rel in bench.GEMM_SOURCES:
        if rel.endswith(".py"):
            continue
        path = os.path.join(ROOT, rel)
        # -fpreprocessed: remove comments, expand nothing (it drops a main
        # file's #pragma once, the one other difference)
        cpp = subprocess.run([gxx, "-x", "c++", "-fpreprocessed", "-dD", "-E", "-P", path],
                             capture_output=True, text=True, check=True).stdout
        mine = bench.code_only(open(path).read()).replace("#pragma once", "")
        assert re.sub(r"\s+", "", mine) == re.sub(r"\s+", "", cpp), rel
