"""The serving loop on the GPU.

* every request's C is bit-identical whether it runs alone or in a mix of
  uneven n, tau, leaf, precision (FP32, BF16, compensated BF16 and FP16 split) and chain
  length (fixed owner and k order per output leaf), and equal to the
  one-call API's result;
* teacher-forced parity with the oracle at every step: step s of a request
  (its input X_s as the GPU holds it) has the oracle's task keys bit for bit,
  class bits included (a split request's relative threshold theta is taken
  by the library against each step's own roots), the served task counts are
  the sums over the steps, and every step's C, the served C included, is
  within Higham's elementwise bound around the oracle's product;
* admission under a budget that holds one request at a time, rejection of a
  request larger than the budget, destroy with requests pending, NaN input
  and an overflowing chain reported as non-finite, poll semantics, several
  submitting threads, and C aliasing A in a chain.
"""
import math
import threading

import numpy as np
import pytest

import oracle
import workloads
from bounds import class_bound

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def decay(n, rate, seed, scale=1.0, sym=True):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return (scale * A).astype(np.float32)


def gershgorin_scaled(A):
    """X_0 = A / max_i sum_j |a_ij|: every power of X_0 stays bounded."""
    return (A / np.abs(A.astype(np.float64)).sum(axis=1).max()).astype(np.float32)


# (n, leaf, tau, precision, theta (relative LOW threshold), chain_len, distinct B, rate, seed)
MIX = [
    (100, 16, 1e-6, 0, 0.0, 0, False, 0.1, 1),
    (257, 32, 1e-6, 1, 1e-3, 0, False, 0.1, 2),
    (512, 32, 1e-8, 0, 0.0, 0, True, 0.05, 3),
    (700, 64, 1e-6, 1, 1e-4, 0, False, 0.02, 4),
    (1024, 32, 1e-6, 0, 0.0, 3, False, 0.1, 5),
    (1024, 32, 1e-8, 1, 1e-4, 3, False, 0.2, 6),
    (333, 32, 0.0, 0, 0.0, 0, True, 0.3, 7),
    (1500, 64, 1e-4, 0, 0.0, 0, False, 0.05, 8),
    (64, 64, 1e-6, 1, 1e-2, 2, False, 0.1, 9),
    (2048, 32, 1e-6, 1, 1e-4, 0, False, 0.1, 10),
    (900, 16, 1e-8, 0, 0.0, 2, False, 0.15, 11),
    (512, 32, 1e-6, 0, 0.0, 0, False, 0.5, 12),
    (1, 32, 0.0, 0, 0.0, 0, False, 0.1, 13),
    (1200, 32, 1e-6, 1, 1e-3, 0, True, 0.08, 14),
    (600, 32, 1e-6, 2, 1e-3, 0, False, 0.1, 15),
    (1024, 64, 1e-8, 2, 1e-4, 2, False, 0.15, 16),
    (300, 32, 1e-6, 2, 1e-2, 0, True, 0.1, 17),
    (800, 64, 1e-6, 3, 1e-4, 0, False, 0.02, 18),
    (1024, 32, 1e-8, 3, 1e-4, 3, False, 0.2, 19),
]


def make_inputs(spec):
    import torch
    n, leaf, tau, prec, theta, chain, distinct, rate, seed = spec
    A = decay(n, rate, seed)
    if chain:
        A = gershgorin_scaled(A)
    B = decay(n, rate * 1.3, seed + 100, sym=False) if distinct else None
    dA = torch.from_numpy(A).cuda()
    dB = None if B is None else torch.from_numpy(B).cuda()
    return A, B, dA, dB


def reference(gpu, spec, dA, dB, low_tol=0.0, keep_steps=False):
    """The same request through the one-call API, step by step: symbolic +
    numeric per step, with the spec's relative split threshold theta (or an
    absolute low_tol).  Returns (C, steps): with keep_steps, per step its input
    X_s as the GPU holds it, the plan's task keys and counts and its C."""
    import torch
    n, leaf, tau, prec, theta, chain, *_ = spec
    bf = prec in (gpu.PREC_SPLIT_BF16, gpu.PREC_SPLIT_BF16X3)
    f16 = prec == gpu.PREC_SPLIT_FP16
    rel = theta if (prec and not low_tol) else 0.0
    X = dA
    steps = []
    for _ in range(max(1, chain)):
        tA = gpu.build_tree(X, leaf, bf16=bf, fp16=f16)
        tB = tA if (dB is None or chain) else gpu.build_tree(dB, leaf, bf16=bf, fp16=f16)
        C = torch.empty_like(dA)
        plan = gpu.symbolic(tA, tB, tau, precision=prec, low_tol=low_tol, low_rel=rel)
        plan.numeric(C)
        st = plan.stats()
        if keep_steps:
            steps.append(dict(X=X.cpu().numpy(), keys=plan.tasks(), K=st["tasks"],
                              Klow=st["tasks_low"], C=C.cpu().numpy()))
        else:
            steps.append(dict(K=st["tasks"], Klow=st["tasks_low"]))
        plan.free()
        X = C
    return X, steps


@pytest.fixture(scope="module")
def mix(gpu):
    import torch
    inputs = [make_inputs(s) for s in MIX]
    refs = [reference(gpu, s, a[2], a[3], keep_steps=s[0] <= 1200) for s, a in zip(MIX, inputs)]
    torch.cuda.synchronize()

    def submit(srv, i, C):
        n, leaf, tau, prec, theta, chain, *_ = MIX[i]
        return srv.submit(inputs[i][2], C, tau, leaf, B=inputs[i][3], precision=prec,
                          low_rel=theta if prec else 0.0, chain_len=chain)

    alone = []
    srv = gpu.Server(8 * GiB, max_slots=8)
    for i in range(len(MIX)):
        C = torch.full_like(inputs[i][2], float("nan"))
        res = srv.wait(submit(srv, i, C))
        alone.append((C, res))
    srv.destroy()

    srv = gpu.Server(8 * GiB, max_slots=16)
    outs = [torch.full_like(a[2], float("nan")) for a in inputs]
    tickets = [submit(srv, i, outs[i]) for i in range(len(MIX))]
    results = [srv.wait(t) for t in tickets]
    info = srv.info()
    srv.destroy()
    return dict(inputs=inputs, refs=refs, alone=alone, outs=outs, results=results, info=info)


@pytest.mark.parametrize("i", range(len(MIX)))
def test_same_alone_and_in_mix(mix, i):
    import torch
    C_alone, r_alone = mix["alone"][i]
    C_mix, r_mix = mix["outs"][i], mix["results"][i]
    assert r_alone["status"] == 0 and r_mix["status"] == 0
    assert torch.equal(C_alone, C_mix)
    assert r_alone["tasks"] == r_mix["tasks"] and r_alone["tasks_low"] == r_mix["tasks_low"]
    assert r_mix["steps"] == max(1, MIX[i][5])
    # and the one-call API gives the same bits and counts, step by step
    X, steps = mix["refs"][i]
    assert torch.equal(C_mix, X)
    assert r_mix["tasks"] == sum(st["K"] for st in steps)
    assert r_mix["tasks_low"] == sum(st["Klow"] for st in steps)
    assert r_mix["flops"] == 2.0 * MIX[i][1] ** 3 * r_mix["tasks"]
    assert 0.0 <= r_mix["queue_ms"] <= r_mix["latency_ms"]


def test_mix_was_batched(mix):
    info = mix["info"]
    assert info["admitted"] == info["completed"] == len(MIX)
    assert info["max_batch"] > 1, info
    assert info["launched_products"] == sum(max(1, s[5]) for s in MIX)
    assert info["launches"] < info["launched_products"]
    assert info["peak_active"] > 1
    assert info["queued"] == 0
    assert 0 < info["used"] <= info["peak_used"] <= info["budget"]


# requests deeper than the rounds take (depth 9 and 10: the per-slot path),
# beside one that the rounds batch; same fields as MIX
DEEP = [
    (16384, 32, 1e-6, 0, 0.0, 2, False, 0.5, 21),     # depth 9, a chain of two squarings
    (32768, 32, 1e-6, 3, 1e-4, 0, False, 0.5, 22),    # depth 10, compensated split
    (512, 32, 1e-6, 1, 1e-4, 0, False, 0.1, 23),      # depth 4, batched beside them
]


def test_deep_requests_on_the_per_slot_path(gpu):
    """Requests of depth 9 and 10 run on the per-slot path while a shallow one
    goes through a round: C bit-identical to the one-call API step by step,
    task counts summed over the steps, the first step's counts against the
    oracle's."""
    import torch
    fmt = {1: "bf16", 2: "fp16", 3: "bf16x3"}
    ins = []
    for n, leaf, tau, prec, theta, chain, distinct, rate, seed in DEEP:
        A = workloads.exp_decay(n, rate, seed)
        if chain:
            A = gershgorin_scaled(A)
        ins.append(torch.from_numpy(A).cuda())
    refs = [reference(gpu, s, dA, None) for s, dA in zip(DEEP, ins)]
    torch.cuda.synchronize()
    srv = gpu.Server(64 * GiB, max_slots=4)
    outs = [torch.full_like(dA, float("nan")) for dA in ins]
    tickets = [srv.submit(ins[i], outs[i], s[2], s[1], precision=s[3],
                          low_rel=s[4] if s[3] else 0.0, chain_len=s[5])
               for i, s in enumerate(DEEP)]
    results = [srv.wait(t) for t in tickets]
    srv.destroy()
    for i, s in enumerate(DEEP):
        X, steps = refs[i]
        r = results[i]
        assert r["status"] == 0, r
        assert r["steps"] == max(1, s[5])
        assert torch.equal(outs[i], X)
        assert r["tasks"] == sum(st["K"] for st in steps)
        assert r["tasks_low"] == sum(st["Klow"] for st in steps)
        A = ins[i].cpu().numpy()
        kw = dict(low_rel=s[4], low_fmt=fmt[s[3]]) if s[3] else {}
        ref = oracle.spamm(A, A, s[1], s[2], want_C=False, **kw)
        assert steps[0]["K"] == ref.K and steps[0]["Klow"] == ref.Klow
    assert 0 < results[1]["tasks_low"] < results[1]["tasks"]


ORACLE_CASES = [i for i, s in enumerate(MIX) if s[0] <= 1200]


@pytest.mark.parametrize("i", ORACLE_CASES)
def test_matches_oracle_every_step(mix, i):
    """Teacher-forced: the oracle takes each step's input as the GPU holds it
    (a chain's X_s is the GPU's FP32 result of step s-1) and must give the
    same task keys (class bits included) and a product within Higham's bound
    of that step's C; the served counts are the sums over the steps."""
    n, leaf, tau, prec, theta, chain, *_ = MIX[i]
    A, B = mix["inputs"][i][0], mix["inputs"][i][1]
    fmt = {2: "fp16", 3: "bf16x3"}.get(prec, "bf16")
    _, steps = mix["refs"][i]
    assert len(steps) == max(1, chain)
    K = Klow = 0
    for s, st in enumerate(steps):
        X = st["X"]
        if s == 0:
            assert np.array_equal(X.view(np.uint32), A.view(np.uint32))
        Y = X if (chain or B is None) else B
        ref = oracle.spamm(X, Y, leaf, tau, low_rel=theta if prec else 0.0, low_fmt=fmt)
        assert np.array_equal(st["keys"], ref.keys), f"step {s}: task keys differ"
        assert st["K"] == ref.K and st["Klow"] == ref.Klow, f"step {s}"
        C = mix["outs"][i].cpu().numpy() if s == len(steps) - 1 else st["C"]
        assert np.array_equal(C.view(np.uint32), st["C"].view(np.uint32))
        err = np.abs(C.astype(np.float64) - ref.C)
        worst = float(np.max(err - class_bound(X, Y, leaf, ref.keys, fmt)))
        assert worst <= 0.0, f"step {s}: rounding bound exceeded by {worst}"
        K += ref.K
        Klow += ref.Klow
    assert mix["results"][i]["tasks"] == K
    assert mix["results"][i]["tasks_low"] == Klow
    if prec and theta and n > leaf:
        assert Klow > 0     # (a one-leaf product is its own norm product: never LOW)


def test_tiny_budget_one_at_a_time(gpu):
    import torch
    specs = [MIX[2], MIX[3], MIX[9], MIX[7]]
    need = [gpu.request_footprint(s[0], s[1], s[2], s[3], 1e-3, s[5], s[6]) for s in specs]
    srv = gpu.Server(max(need), max_slots=4)
    try:
        ins = [make_inputs(s) for s in specs]
        refs = [reference(gpu, s, a[2], a[3], low_tol=1e-3 if s[3] else 0.0)
                for s, a in zip(specs, ins)]
        outs = [torch.empty_like(a[2]) for a in ins]
        tickets = [srv.submit(a[2], C, s[2], s[1], B=a[3], precision=s[3],
                              low_tol=1e-3 if s[3] else 0.0, chain_len=s[5])
                   for s, a, C in zip(specs, ins, outs)]
        res = [srv.wait(t) for t in tickets]
        info = srv.info()
        assert all(r["status"] == 0 for r in res)
        for C, ref in zip(outs, refs):
            assert torch.equal(C, ref[0])
        assert info["peak_used"] <= max(need)
        assert info["peak_active"] < len(specs)
        # a request larger than the whole budget is refused at submit
        big = torch.zeros(4096, 4096, device="cuda")
        with pytest.raises(gpu.SpammError) as ei:
            srv.submit(big, torch.empty_like(big), 1e-6, 32)
        assert ei.value.code == gpu.SPAMM_E_NOMEM
    finally:
        srv.destroy()


def test_destroy_with_requests_pending(gpu):
    import torch
    A = torch.from_numpy(decay(1024, 0.1, 0)).cuda()
    outs = [torch.empty_like(A) for _ in range(24)]
    srv = gpu.Server(4 * GiB, max_slots=2)
    for C in outs:
        srv.submit(A, C, 1e-6, 32, chain_len=2)
    srv.destroy()        # drops the queued ones, drains the admitted ones
    srv = gpu.Server(4 * GiB, max_slots=2)
    C = torch.empty_like(A)
    r = srv.wait(srv.submit(A, C, 1e-6, 32))
    srv.destroy()
    t = gpu.build_tree(A, 32)
    ref = torch.empty_like(A)
    gpu.multiply_ex(t, t, 1e-6, ref)
    assert r["status"] == 0 and torch.equal(C, ref)


def test_nonfinite_input_and_overflowing_chain(gpu):
    import torch
    A = decay(300, 0.1, 3)
    bad = A.copy()
    bad[17, 200] = np.nan
    big = decay(300, 0.1, 4, scale=1e20)
    good = gershgorin_scaled(decay(300, 0.1, 5))
    srv = gpu.Server(2 * GiB, max_slots=4)
    try:
        dbad, dbig, dgood = (torch.from_numpy(x).cuda() for x in (bad, big, good))
        outs = [torch.empty_like(dbad) for _ in range(3)]
        t1 = srv.submit(dbad, outs[0], 1e-6, 32)
        t2 = srv.submit(dbig, outs[1], 1e-6, 32, chain_len=3)
        t3 = srv.submit(dgood, outs[2], 1e-6, 32, chain_len=3)
        r1, r2, r3 = srv.wait(t1), srv.wait(t2), srv.wait(t3)
        assert r1["status"] == gpu.SPAMM_E_NONFINITE
        assert r2["status"] == gpu.SPAMM_E_NONFINITE     # X_1 = A^2 overflows FP32
        assert r3["status"] == 0
        ref = reference(gpu, (300, 32, 1e-6, 0, 0.0, 3, False, 0, 0), dgood, None)[0]
        assert torch.equal(outs[2], ref)
    finally:
        srv.destroy()


def test_poll_semantics(gpu):
    import torch
    A = torch.from_numpy(decay(256, 0.1, 1)).cuda()
    srv = gpu.Server(GiB, max_slots=1)
    try:
        with pytest.raises(gpu.SpammError) as ei:
            srv.poll(12345)
        assert ei.value.code == gpu.SPAMM_E_INVAL
        C = torch.empty_like(A)
        t = srv.submit(A, C, 1e-6, 32)
        assert t > 0
        r = srv.wait(t)
        assert r["status"] == 0
        with pytest.raises(gpu.SpammError):
            srv.poll(t)                   # already collected
        t2 = srv.submit(A, C, 1e-6, 32)
        assert t2 > t
        srv.wait(t2)
    finally:
        srv.destroy()


def test_submitters_on_several_threads(gpu):
    import torch
    specs = [(n, 32, 1e-6, 0, 0.0, c, False, 0.1, 50 + k)
             for k, (n, c) in enumerate([(256, 0), (512, 2), (384, 0), (640, 1)] * 2)]
    ins = [make_inputs(s) for s in specs]
    refs = [reference(gpu, s, a[2], None)[0] for s, a in zip(specs, ins)]
    torch.cuda.synchronize()
    outs = [torch.empty_like(a[2]) for a in ins]
    srv = gpu.Server(4 * GiB, max_slots=8)
    errors = []

    def worker(idx):
        try:
            for i in idx:
                s = specs[i]
                t = srv.submit(ins[i][2], outs[i], s[2], s[1], chain_len=s[5], sync=False)
                assert srv.wait(t)["status"] == 0
        except Exception as e:      # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(range(k, len(specs), 4),)) for k in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    srv.destroy()
    assert not errors, errors
    for C, ref in zip(outs, refs):
        assert torch.equal(C, ref)


def test_chain_in_place(gpu):
    import torch
    A = gershgorin_scaled(decay(700, 0.1, 21))
    X = torch.from_numpy(A).cuda()
    ref = reference(gpu, (700, 32, 1e-7, 1, 0.0, 4, False, 0, 0), X.clone(), None,
                    low_tol=1e-4)[0]
    srv = gpu.Server(2 * GiB, max_slots=2)
    try:
        r = srv.wait(srv.submit(X, X, 1e-7, 32, precision=gpu.PREC_SPLIT_BF16, low_tol=1e-4,
                                chain_len=4))
    finally:
        srv.destroy()
    assert r["status"] == 0 and r["steps"] == 4
    assert torch.equal(X, ref)
