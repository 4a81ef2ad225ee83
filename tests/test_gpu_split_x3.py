"""Compensated split precision (PREC_SPLIT_BF16X3) on the GPU against the
oracle's bf16x3 mode.

* task keys bit-exact with the class bit, kept and LOW counts equal the
  oracle's (the classes are those of the plain BF16 split);
* C within Higham's bound around the oracle's product, where only FP32
  accumulation differs (every product of two bfloat16 values is exact in
  FP32): |C_gpu - C_oracle| <= gamma_m sum |terms| + m 2^-126, a HIGH
  product contributing the three terms hi_a hi_b, hi_a lo_b, lo_a hi_b
  (bounded by (|hi_a| + |lo_a|)(|hi_b| + |lo_b|)), m = 3 n_b K_ij + 1;
* the cases run every kernel that takes the mode: 32 x 32 leaves, 64 x 64
  leaves below depth 2 (2 x 2 blocks) and from depth 2 (4 x 4 blocks);
* low_tol = 0 (every product HIGH) is within 2^-14 sum |a||b| of the exact
  product, and closer to it than BF16 operands alone;
* the HIGH products differ from the FP32 kernel's only by that error;
* with every product LOW the mode is the BF16 split bit for bit; nothing
  kept writes zeros; entries that would overflow their bfloat16 part are
  refused (SPAMM_E_RANGE), on the one-call path and in the server.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def decay(n, rate, seed, sym=True):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return A.astype(np.float32)


def bf16_round(P):
    import torch
    return torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32)).to(torch.bfloat16).to(
        torch.float64).numpy()


CASES = {
    # name: (A, B or None, leaf, tau, low_tol); kernel in the comment
    "mixed-b32": lambda: (workloads.exp_decay(1024, 0.1, 0), None, 32, 1e-6, 1e-2),      # 2x2
    "mixed-wide-b64": lambda: (decay(700, 0.02, 1), None, 64, 1e-6, 2e-2),              # 4x4
    "all-high-wide-b64": lambda: (decay(520, 0.03, 2), None, 64, 1e-5, 0.0),            # 4x4
    "all-high-d1-b64": lambda: (decay(100, 0.05, 3), None, 64, 0.0, 0.0),               # 2x2
    "nonsym-b32": lambda: (decay(256, 0.05, 4, sym=False), decay(256, 0.08, 5, sym=False), 32,
                           1e-5, 5e-2),
    "nonsym-wide-b64": lambda: (decay(300, 0.04, 6, sym=False), decay(300, 0.06, 7, sym=False),
                                64, 1e-6, 3e-2),
    "single-leaf-b64": lambda: (decay(50, 0.1, 8), None, 64, 0.0, 0.0),                # d = 0
    "ragged-b32": lambda: (decay(333, 0.04, 9), None, 32, 1e-5, 1e-2),
    "algdecay-b64": lambda: (workloads.alg_decay(1000, 3.0, 0), None, 64, 1e-8, 1e-4),
}


def padded(A, leaf):
    d, np_ = oracle.depth(A.shape[0], leaf)
    P = np.zeros((np_, np_), dtype=np.float32)
    P[:A.shape[0], :A.shape[0]] = A
    return P, d


def abs_parts(P):
    """|hi| + |lo| elementwise, by torch's rounding and float32 subtraction."""
    H = bf16_round(P)
    L = bf16_round(P - H.astype(np.float32))
    return np.abs(H) + np.abs(L)


def x3_bound(A, B, leaf, keys):
    PA, d = padded(A, leaf)
    PB, _ = padded(B, leaf)
    N = 1 << d
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    ops = {0: (abs_parts(PA), abs_parts(PB)), 1: (np.abs(bf16_round(PA)), np.abs(bf16_round(PB)))}
    M = np.zeros(PA.shape)
    cnt = np.zeros((N, N), dtype=np.int64)
    for key in keys:
        key = int(key)
        I, J = inv[(key >> 32) & 0x7FFFFFFF]
        k = key & 0xFFFFFFFF
        X, Y = ops[key >> 63]
        M[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] += (
            X[I * leaf:(I + 1) * leaf, k * leaf:(k + 1) * leaf] @ Y[k * leaf:(k + 1) * leaf,
                                                                  J * leaf:(J + 1) * leaf])
        cnt[I, J] += 1
    m = 3 * leaf * np.kron(cnt, np.ones((leaf, leaf))) + 1
    gamma = m * U32 / (1 - m * U32)
    n = A.shape[0]
    return (gamma * M + m * 2.0 ** -126)[:n, :n]


@pytest.fixture(scope="module")
def runs(gpu):
    import torch
    cache = {}

    def get(name):
        if name not in cache:
            A, B, leaf, tau, low = CASES[name]()
            Bm = A if B is None else B
            print(f"[x3] {name} n={A.shape[0]} leaf={leaf} tau={tau} low_tol={low}", flush=True)
            ref = oracle.spamm(A, Bm, leaf, tau, low_tol=low, low_fmt="bf16x3")
            dA = torch.from_numpy(A).cuda()
            tA = gpu.build_tree(dA, leaf, bf16=True)
            tB = tA if B is None else gpu.build_tree(torch.from_numpy(B).cuda(), leaf, bf16=True)
            plan = gpu.symbolic(tA, tB, tau, precision=gpu.PREC_SPLIT_BF16X3, low_tol=low)
            C = torch.full_like(dA, float("nan"))
            plan.numeric(C)
            torch.cuda.synchronize()
            cache[name] = dict(A=A, B=Bm, leaf=leaf, tau=tau, low=low, ref=ref, tA=tA, tB=tB,
                               plan=plan, C=C.cpu().numpy(), dA=dA)
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_x3_task_list_with_classes(runs, name):
    r = runs(name)
    keys = r["plan"].tasks()
    assert np.array_equal(keys, r["ref"].keys)
    st = r["plan"].stats()
    assert st["tasks"] == r["ref"].K and st["tasks_low"] == r["ref"].Klow
    assert st["kept"] == [int(v) for v in r["ref"].Kt]
    if "high" in name or name.startswith("single"):
        assert st["tasks_low"] == 0 < st["tasks"]
    if name.startswith("mixed") or name.startswith("nonsym"):
        assert 0 < st["tasks_low"] < st["tasks"]


@pytest.mark.parametrize("name", list(CASES))
def test_x3_product_within_bound(runs, name):
    r = runs(name)
    assert np.all(np.isfinite(r["C"]))
    err = np.abs(r["C"].astype(np.float64) - r["ref"].C)
    worst = float(np.max(err - x3_bound(r["A"], r["B"], r["leaf"], r["ref"].keys)))
    assert worst <= 0.0, f"bound exceeded by {worst}"


@pytest.mark.parametrize("name", ["all-high-wide-b64", "all-high-d1-b64", "single-leaf-b64"])
def test_x3_all_high_against_exact_and_fp32(gpu, runs, name):
    import torch
    r = runs(name)
    A = r["A"].astype(np.float64)
    # the exact product of the kept leaves: tau keeps every product here
    # except the all-high-wide case, where the oracle's FP32-operand product
    # over the same keys is the reference
    exact = oracle.spamm(r["A"], r["B"], r["leaf"], r["tau"]).C
    absprod = np.abs(A) @ np.abs(r["B"].astype(np.float64))
    C = r["C"].astype(np.float64)
    n = A.shape[0]
    gam = (3 * n + 1) * U32
    assert np.all(np.abs(C - exact) <= (2.0 ** -14 + gam) * absprod + 1e-30)
    # closer to the exact product than BF16 operands alone
    t = gpu.build_tree(r["dA"], r["leaf"], bf16=True)
    Cb = torch.empty_like(r["dA"])
    gpu.multiply_ex(t, t, r["tau"], Cb, precision=gpu.PREC_SPLIT_BF16, low_tol=1e30)
    eb = np.abs(Cb.cpu().numpy().astype(np.float64) - exact).max()
    assert np.abs(C - exact).max() < 0.05 * eb
    # and from the FP32 kernel by no more than that error
    Cf = torch.empty_like(r["dA"])
    gpu.multiply_ex(t, t, r["tau"], Cf)
    assert np.all(np.abs(C - Cf.cpu().numpy()) <= (2.0 ** -13 + 2 * gam) * absprod + 1e-30)


def test_x3_repeat_is_bit_identical(gpu):
    import torch
    A = decay(700, 0.02, 1)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 64, bf16=True)
    C1, C2 = torch.empty_like(dA), torch.empty_like(dA)
    gpu.multiply_ex(t, t, 1e-6, C1, precision=gpu.PREC_SPLIT_BF16X3, low_rel=1e-3)
    gpu.multiply_ex(t, t, 1e-6, C2, precision=gpu.PREC_SPLIT_BF16X3, low_rel=1e-3)
    assert torch.equal(C1.view(torch.int32), C2.view(torch.int32))


def test_x3_argument_errors(gpu):
    import torch
    A = decay(256, 0.05, 10)
    dA = torch.from_numpy(A).cuda()
    plain = gpu.build_tree(dA, 32)
    with pytest.raises(gpu.SpammError):
        gpu.symbolic(plain, plain, 1e-6, precision=gpu.PREC_SPLIT_BF16X3, low_tol=1e-3)
    t16 = gpu.build_tree(dA, 32, fp16=True)
    with pytest.raises(gpu.SpammError):
        gpu.symbolic(t16, t16, 1e-6, precision=gpu.PREC_SPLIT_BF16X3, low_tol=1e-3)
    sub = gpu.build_tree(dA, 64, bf16=True, subnorms=True)
    with pytest.raises(gpu.SpammError):
        gpu.symbolic(sub, sub, 1e-6, precision=gpu.PREC_SPLIT_BF16X3, sub_cull=True)


def test_x3_refuses_entries_that_overflow_their_bf16_part(gpu):
    """An entry at or above 2^128 (1 - 2^-9) rounds to an infinite bfloat16
    part: the compensated mode refuses operands whose squared norm reaches
    the square of that bound, on the one-call path and in the server."""
    import torch
    A = decay(200, 0.1, 12)
    A[3, 3] = np.float32(2.0 ** 128 * (1 - 2.0 ** -9))   # rounds to an infinite bfloat16
    assert float(A[3, 3]) == 2.0 ** 128 * (1 - 2.0 ** -9)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 32, bf16=True)
    with pytest.raises(gpu.SpammError) as ei:
        gpu.symbolic(t, t, 1e-6, precision=gpu.PREC_SPLIT_BF16X3, low_rel=1e-3)
    assert ei.value.code == gpu.SPAMM_E_RANGE
    # the plain BF16 split takes it (its HIGH products stay FP32)
    gpu.symbolic(t, t, 1e-6, precision=gpu.PREC_SPLIT_BF16, low_rel=1e-3).free()
    # just below the bound of the norm: accepted
    B = decay(200, 0.1, 12)
    B[3, 3] = np.float32(1e38)
    tb = gpu.build_tree(torch.from_numpy(B).cuda(), 32, bf16=True)
    gpu.symbolic(tb, tb, 1e-6, precision=gpu.PREC_SPLIT_BF16X3, low_rel=1e-3).free()
    srv = gpu.Server(2 << 30, max_slots=2)
    try:
        C = torch.empty_like(dA)
        r = srv.wait(srv.submit(dA, C, 1e-6, 32, precision=gpu.PREC_SPLIT_BF16X3, low_rel=1e-3))
        assert r["status"] == gpu.SPAMM_E_RANGE
    finally:
        srv.destroy()


@pytest.mark.parametrize("n,leaf", [(300, 32), (700, 64)])
def test_x3_all_low_is_the_bf16_split_bit_for_bit(gpu, n, leaf):
    """With every product LOW the compensated mode runs only BF16 products,
    in the same order as the BF16 split (2 x 2 and 4 x 4 kernels)."""
    import torch
    A = decay(n, 0.05, 13)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, leaf, bf16=True)
    C3, Cb = torch.empty_like(dA), torch.empty_like(dA)
    s3 = gpu.multiply_ex(t, t, 1e-6, C3, precision=gpu.PREC_SPLIT_BF16X3, low_tol=1e30)
    sb = gpu.multiply_ex(t, t, 1e-6, Cb, precision=gpu.PREC_SPLIT_BF16, low_tol=1e30)
    assert s3["tasks_low"] == s3["tasks"] == sb["tasks"] > 0
    assert torch.equal(C3.view(torch.int32), Cb.view(torch.int32))


def test_x3_nothing_kept_writes_zeros(gpu):
    import torch
    A = decay(400, 0.1, 14)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 64, bf16=True)
    C = torch.full_like(dA, float("nan"))
    st = gpu.multiply_ex(t, t, 1e3, C, precision=gpu.PREC_SPLIT_BF16X3, low_rel=1e-3)
    assert st["tasks"] == 0
    assert torch.count_nonzero(C).item() == 0
