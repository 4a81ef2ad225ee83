"""Split precision on the GPU against the oracle's split mode.

* task keys bit-exact, including the class bit (63) of LOW products;
* kept and LOW counts equal the oracle's;
* C within Higham's bound around the oracle's split product (LOW operands
  rounded to bfloat16, products exact in FP64; only FP32 accumulation
  differs): |C_gpu - C_oracle| <= gamma_m sum_kept |X||Y| + m 2^-126, with
  X, Y the operands of each product's class, m = n_b K_ij + 1, u = 2^-24;
* low_tol = 0 gives the FP32 product's values.
"""
import math

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
    # name: (A, B or None, leaf, tau, low_tol)
    "mixed-b32": lambda: (workloads.exp_decay(1024, 0.1, 0), None, 32, 1e-6, 1e-2),
    "mixed-b64": lambda: (decay(700, 0.02, 1), None, 64, 1e-6, 2e-2),
    "all-low-b32": lambda: (decay(300, 0.05, 2), None, 32, 0.0, 1e30),
    "none-low-b64": lambda: (decay(300, 0.05, 3), None, 64, 1e-4, 0.0),
    "nonsym-b32": lambda: (decay(256, 0.05, 4, sym=False), decay(256, 0.08, 5, sym=False), 32,
                           1e-5, 5e-2),
    "single-leaf-b64": lambda: (decay(50, 0.1, 6), None, 64, 0.0, 1e30),
    "ragged-b32": lambda: (decay(333, 0.04, 7), None, 32, 1e-5, 1e-2),
    "algdecay-b64": lambda: (workloads.alg_decay(1000, 3.0, 0), None, 64, 1e-8, 1e-4),
}


def padded(A, leaf):
    d, np_ = oracle.depth(A.shape[0], leaf)
    P = np.zeros((np_, np_), dtype=np.float32)
    P[:A.shape[0], :A.shape[0]] = A
    return P, d


def split_bound(A, B, leaf, keys):
    PA, d = padded(A, leaf)
    PB, _ = padded(B, leaf)
    N = 1 << d
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    ops = {0: (np.abs(PA.astype(np.float64)), np.abs(PB.astype(np.float64))),
           1: (np.abs(bf16_round(PA)), np.abs(bf16_round(PB)))}
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
    m = leaf * np.kron(cnt, np.ones((leaf, leaf))) + 1
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
            ref = oracle.spamm(A, Bm, leaf, tau, low_tol=low)
            dA = torch.from_numpy(A).cuda()
            tA = gpu.build_tree(dA, leaf, bf16=True)
            tB = tA if B is None else gpu.build_tree(torch.from_numpy(B).cuda(), leaf, bf16=True)
            plan = gpu.symbolic(tA, tB, tau, precision=gpu.PREC_SPLIT_BF16, low_tol=low)
            C = torch.full_like(dA, float("nan"))
            plan.numeric(C)
            torch.cuda.synchronize()
            cache[name] = dict(A=A, B=Bm, leaf=leaf, tau=tau, low=low, ref=ref, tA=tA, tB=tB,
                               plan=plan, C=C.cpu().numpy(), dA=dA)
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_split_task_list_with_classes(runs, name):
    r = runs(name)
    keys = r["plan"].tasks()
    assert np.array_equal(keys, r["ref"].keys)
    st = r["plan"].stats()
    assert st["tasks"] == r["ref"].K and st["tasks_low"] == r["ref"].Klow
    assert st["kept"] == [int(v) for v in r["ref"].Kt]
    if name.startswith("all-low") or name.startswith("single-leaf"):
        assert st["tasks_low"] == st["tasks"] > 0
    if name.startswith("none-low"):
        assert st["tasks_low"] == 0
    if name.startswith("mixed"):
        assert 0 < st["tasks_low"] < st["tasks"]


@pytest.mark.parametrize("name", list(CASES))
def test_split_product_within_bound(runs, name):
    r = runs(name)
    assert np.all(np.isfinite(r["C"]))
    err = np.abs(r["C"].astype(np.float64) - r["ref"].C)
    worst = float(np.max(err - split_bound(r["A"], r["B"], r["leaf"], r["ref"].keys)))
    assert worst <= 0.0, f"bound exceeded by {worst}"


def test_split_with_zero_low_tol_equals_fp32(gpu):
    import torch
    A = decay(512, 0.05, 9)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 64, bf16=True)
    C1 = torch.empty_like(dA)
    C2 = torch.empty_like(dA)
    gpu.multiply_ex(t, t, 1e-6, C1)
    st = gpu.multiply_ex(t, t, 1e-6, C2, precision=gpu.PREC_SPLIT_BF16, low_tol=0.0)
    assert st["tasks_low"] == 0
    assert torch.equal(C1, C2)


def test_split_error_vs_dense_fp64_is_stated(gpu):
    """LOW products carry about 2^-8 relative error each: the split product's
    max-norm error against the dense FP64 product stays below the truncation
    bound plus sum_LOW 2 * 2^-8 ||A_ik|| ||B_kj|| (bf16 rounding of both
    operands) plus the FP32 rounding."""
    import torch
    A = workloads.exp_decay(1024, 0.1, 0)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 32, bf16=True)
    C = torch.empty_like(dA)
    st = gpu.multiply_ex(t, t, 1e-6, C, precision=gpu.PREC_SPLIT_BF16, low_rel=1e-4)
    exact = A.astype(np.float64) @ A.astype(np.float64)
    err = float(np.abs(C.cpu().numpy() - exact).max())
    nrm = np.sqrt(oracle.norms(A, 32)[-1])
    ref = oracle.spamm(A, A, 32, 1e-6, want_C=False, low_rel=1e-4)
    assert st["tasks_low"] == ref.Klow
    inv = {oracle.linear_index(i, j): (i, j) for i in range(32) for j in range(32)}
    lowsum = {}   # per output leaf: sum over its LOW products of ||A_ik|| ||A_kj||
    for key in ref.keys:
        key = int(key)
        if key >> 63:
            I, J = inv[(key >> 32) & 0x7FFFFFFF]
            k = key & 0xFFFFFFFF
            lowsum[(I, J)] = lowsum.get((I, J), 0.0) + nrm[I, k] * nrm[k, J]
    worst_low = max(lowsum.values())
    trunc = oracle.spamm(A, A, 32, 1e-6).C
    bound = float(np.abs(trunc - exact).max()) + (2 * 2.0 ** -9 + 2.0 ** -18) * worst_low \
        + 1e-5 * math.sqrt(t.norm2) ** 2
    assert st["tasks_low"] > 0
    assert err <= bound


def test_split_argument_errors(gpu):
    import torch
    A = torch.from_numpy(decay(200, 0.05, 1)).cuda()
    plain = gpu.build_tree(A, 32)
    with pytest.raises(gpu.SpammError) as ei:
        gpu.symbolic(plain, plain, 1e-6, precision=gpu.PREC_SPLIT_BF16, low_tol=1e-3)
    assert ei.value.code == gpu.SPAMM_E_INVAL
    with pytest.raises(gpu.SpammError):
        gpu.build_tree(A, 16, bf16=True)
    t = gpu.build_tree(A, 32, bf16=True)
    for bad in (-1.0, float("nan"), float("inf"), 1e-200):
        with pytest.raises(gpu.SpammError) as ei:
            gpu.symbolic(t, t, 1e-6, precision=gpu.PREC_SPLIT_BF16, low_tol=bad)
        assert ei.value.code == gpu.SPAMM_E_INVAL
    for bad in (-1.0, float("nan"), float("inf"), 1e-200):
        with pytest.raises(gpu.SpammError) as ei:
            gpu.symbolic(t, t, 1e-6, precision=gpu.PREC_SPLIT_BF16, low_rel=bad)
        assert ei.value.code == gpu.SPAMM_E_INVAL
    with pytest.raises(gpu.SpammError) as ei:     # one threshold, not both
        gpu.symbolic(t, t, 1e-6, precision=gpu.PREC_SPLIT_BF16, low_tol=1e-3, low_rel=1e-4)
    assert ei.value.code == gpu.SPAMM_E_INVAL
    with pytest.raises(gpu.SpammError):
        gpu.symbolic(t, t, 1e-6, precision=7)


# ---- relative threshold theta, evaluated by the library ------------------------

REL_CASES = {
    # name: (A, B or None, leaf, tau, theta, format)
    "rel-b32-1e-4": lambda: (workloads.exp_decay(1024, 0.1, 0), None, 32, 1e-6, 1e-4, "bf16"),
    "rel-b32-1e-2": lambda: (workloads.exp_decay(1024, 0.1, 0), None, 32, 1e-6, 1e-2, "bf16"),
    "rel-b64-fp16": lambda: (decay(700, 0.02, 1), None, 64, 1e-6, 1e-3, "fp16"),
    "rel-nonsym-b32": lambda: (decay(256, 0.05, 4, sym=False), decay(256, 0.08, 5, sym=False),
                               32, 1e-5, 3e-3, "bf16"),
    "rel-nonsym-fp16": lambda: (decay(256, 0.05, 4, sym=False),
                                50.0 * decay(256, 0.08, 5, sym=False), 32, 1e-5, 3e-3, "fp16"),
    "rel-single-leaf": lambda: (decay(50, 0.1, 6), None, 64, 0.0, 2.0, "bf16"),
    "rel-algdecay-b64": lambda: (workloads.alg_decay(1000, 3.0, 0), None, 64, 1e-8, 1e-4,
                                 "bf16"),
}


@pytest.mark.parametrize("name", list(REL_CASES))
def test_relative_threshold_task_list_and_product(gpu, name):
    """LOW iff norm product < theta ||A||_F ||B||_F, the bound formed by the
    library from the two trees' roots: task keys with class bits bit-exact
    against the oracle's relative mode, C within Higham's bound over each
    class's operands."""
    import torch
    from bounds import class_bound
    A, B, leaf, tau, theta, fmt = REL_CASES[name]()
    Bm = A if B is None else B
    prec = gpu.PREC_SPLIT_FP16 if fmt == "fp16" else gpu.PREC_SPLIT_BF16
    ref = oracle.spamm(A, Bm, leaf, tau, low_rel=theta, low_fmt=fmt)
    dA = torch.from_numpy(A).cuda()
    kw = {fmt: True}
    tA = gpu.build_tree(dA, leaf, **kw)
    tB = tA if B is None else gpu.build_tree(torch.from_numpy(B).cuda(), leaf, **kw)
    plan = gpu.symbolic(tA, tB, tau, precision=prec, low_rel=theta)
    C = torch.full_like(dA, float("nan"))
    plan.numeric(C)
    torch.cuda.synchronize()
    assert np.array_equal(plan.tasks(), ref.keys)
    st = plan.stats()
    assert st["tasks"] == ref.K and st["tasks_low"] == ref.Klow
    assert 0 < ref.Klow, name
    if name != "rel-single-leaf":
        assert ref.Klow < ref.K, name
    err = np.abs(C.cpu().numpy().astype(np.float64) - ref.C)
    worst = float(np.max(err - class_bound(A, Bm, leaf, ref.keys, fmt)))
    assert worst <= 0.0, f"bound exceeded by {worst}"


# ---- FP16 LOW operands (per-leaf power-of-two scale) ---------------------------

def fp16_leaves(P, leaf, S):
    """P (padded FP32) with every leaf rounded through numpy float16 at the
    scale exponent of its squared norm S[I, J] (oracle.fp16_exponent),
    binary16 subnormals flushed to zero."""
    N = P.shape[0] // leaf
    R = np.zeros(P.shape)
    for I in range(N):
        for J in range(N):
            e = oracle.fp16_exponent(S[I, J])
            blk = P[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf].astype(np.float64) * 2.0 ** e
            h = blk.astype(np.float16).astype(np.float64)
            R[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] = \
                np.where(np.abs(h) < 2.0 ** -14, 0.0, h) * 2.0 ** -e
    return R


def split16_bound(A, B, leaf, keys):
    """As split_bound with FP16 LOW operands; each LOW product is summed on its
    own and added (one more FP32 rounding per product): m = (n_b + 1) K + 1."""
    PA, d = padded(A, leaf)
    PB, _ = padded(B, leaf)
    N = 1 << d
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    ops = {0: (np.abs(PA.astype(np.float64)), np.abs(PB.astype(np.float64))),
           1: (np.abs(fp16_leaves(PA, leaf, oracle.norms(A, leaf)[-1])),
               np.abs(fp16_leaves(PB, leaf, oracle.norms(B, leaf)[-1])))}
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
    m = (leaf + 1) * np.kron(cnt, np.ones((leaf, leaf))) + 1
    gamma = m * U32 / (1 - m * U32)
    n = A.shape[0]
    return (gamma * M + m * 2.0 ** -126)[:n, :n]


@pytest.fixture(scope="module")
def runs16(gpu):
    import torch
    cache = {}

    def get(name):
        if name not in cache:
            A, B, leaf, tau, low = CASES[name]()
            Bm = A if B is None else B
            ref = oracle.spamm(A, Bm, leaf, tau, low_tol=low, low_fmt="fp16")
            dA = torch.from_numpy(A).cuda()
            tA = gpu.build_tree(dA, leaf, fp16=True)
            tB = tA if B is None else gpu.build_tree(torch.from_numpy(B).cuda(), leaf, fp16=True)
            plan = gpu.symbolic(tA, tB, tau, precision=gpu.PREC_SPLIT_FP16, low_tol=low)
            C = torch.full_like(dA, float("nan"))
            plan.numeric(C)
            torch.cuda.synchronize()
            cache[name] = dict(A=A, B=Bm, leaf=leaf, tau=tau, low=low, ref=ref, plan=plan,
                               C=C.cpu().numpy())
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_fp16_task_list_with_classes(runs16, name):
    r = runs16(name)
    assert np.array_equal(r["plan"].tasks(), r["ref"].keys)
    st = r["plan"].stats()
    assert st["tasks"] == r["ref"].K and st["tasks_low"] == r["ref"].Klow


@pytest.mark.parametrize("name", list(CASES))
def test_fp16_product_within_bound(runs16, name):
    r = runs16(name)
    assert np.all(np.isfinite(r["C"]))
    err = np.abs(r["C"].astype(np.float64) - r["ref"].C)
    worst = float(np.max(err - split16_bound(r["A"], r["B"], r["leaf"], r["ref"].keys)))
    assert worst <= 0.0, f"bound exceeded by {worst}"


def test_fp16_tiny_entries_keep_their_digits(gpu):
    """Entries far below binary16's range (1e-30 .. 1e-40) survive because each
    leaf is scaled by its own power of two: the all-LOW FP16 product of such a
    matrix matches the oracle's as closely as one of order-one entries."""
    import torch
    A = decay(200, 0.05, 31) * np.float32(1e-33)
    B = decay(200, 0.07, 32, sym=False)
    ref = oracle.spamm(A, B, 32, 0.0, low_tol=1e30, low_fmt="fp16")
    assert ref.Klow == ref.K
    tA = gpu.build_tree(torch.from_numpy(A).cuda(), 32, fp16=True)
    tB = gpu.build_tree(torch.from_numpy(B).cuda(), 32, fp16=True)
    C = torch.empty((200, 200), device="cuda")
    gpu.multiply_ex(tA, tB, 0.0, C, precision=gpu.PREC_SPLIT_FP16, low_tol=1e30)
    got = C.cpu().numpy().astype(np.float64)
    scale = np.abs(ref.C).max()
    assert scale > 0 and np.abs(got - ref.C).max() <= 1e-5 * scale
    exact = A.astype(np.float64) @ B.astype(np.float64)
    # unscaled binary16 would flush every entry to zero (a 100 % error)
    assert np.abs(got - exact).max() <= 1e-2 * np.abs(exact).max()


def test_fp16_zero_low_tol_equals_fp32(gpu):
    import torch
    A = decay(512, 0.05, 9)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 64, fp16=True)
    C1, C2 = torch.empty_like(dA), torch.empty_like(dA)
    gpu.multiply_ex(t, t, 1e-6, C1)
    st = gpu.multiply_ex(t, t, 1e-6, C2, precision=gpu.PREC_SPLIT_FP16, low_tol=0.0)
    assert st["tasks_low"] == 0
    assert torch.equal(C1, C2)


def test_fp16_error_below_bf16_at_same_classes(gpu):
    """Same tau and low_tol, so the same LOW set: the FP16 product's max-norm
    error against the dense FP64 product is well below the BF16 one's, and
    within the truncation error plus sum_LOW (2 2^-11 + 2^-22) ||A_ik|| ||B_kj||
    plus the FP32 rounding."""
    import torch
    A = workloads.exp_decay(1024, 0.1, 0)
    dA = torch.from_numpy(A).cuda()
    t16 = gpu.build_tree(dA, 32, fp16=True)
    tb = gpu.build_tree(dA, 32, bf16=True)
    C16, Cb = torch.empty_like(dA), torch.empty_like(dA)
    s16 = gpu.multiply_ex(t16, t16, 1e-6, C16, precision=gpu.PREC_SPLIT_FP16, low_rel=1e-2)
    sb = gpu.multiply_ex(tb, tb, 1e-6, Cb, precision=gpu.PREC_SPLIT_BF16, low_rel=1e-2)
    assert s16["tasks_low"] == sb["tasks_low"] > 0
    exact = A.astype(np.float64) @ A.astype(np.float64)
    e16 = float(np.abs(C16.cpu().numpy() - exact).max())
    eb = float(np.abs(Cb.cpu().numpy() - exact).max())
    assert e16 < eb / 4
    nrm = np.sqrt(oracle.norms(A, 32)[-1])
    ref = oracle.spamm(A, A, 32, 1e-6, want_C=False, low_rel=1e-2, low_fmt="fp16")
    assert s16["tasks_low"] == ref.Klow
    inv = {oracle.linear_index(i, j): (i, j) for i in range(32) for j in range(32)}
    lowsum = {}
    for key in ref.keys:
        key = int(key)
        if key >> 63:
            I, J = inv[(key >> 32) & 0x7FFFFFFF]
            k = key & 0xFFFFFFFF
            lowsum[(I, J)] = lowsum.get((I, J), 0.0) + nrm[I, k] * nrm[k, J]
    trunc = oracle.spamm(A, A, 32, 1e-6).C
    bound = float(np.abs(trunc - exact).max()) + (2 * 2.0 ** -11 + 2.0 ** -22) * \
        max(lowsum.values()) + 1e-5 * t16.norm2
    assert e16 <= bound


def test_fp16_argument_errors(gpu):
    import torch
    A = torch.from_numpy(decay(200, 0.05, 1)).cuda()
    tb = gpu.build_tree(A, 32, bf16=True)
    t16 = gpu.build_tree(A, 32, fp16=True)
    for t, prec in ((tb, gpu.PREC_SPLIT_FP16), (t16, gpu.PREC_SPLIT_BF16)):
        with pytest.raises(gpu.SpammError) as ei:
            gpu.symbolic(t, t, 1e-6, precision=prec, low_tol=1e-3)
        assert ei.value.code == gpu.SPAMM_E_INVAL
    with pytest.raises(gpu.SpammError):
        gpu.build_tree(A, 16, fp16=True)
    with pytest.raises(gpu.SpammError):
        gpu.build_tree(A, 32, fp16=True, bf16=True)
