"""A seeded random sweep of the GPU path against the oracle: odd n (1 .. 1500),
all leaf sizes, tau from 0 to 1e-2, decay rates from dense to nearly
diagonal, A = B or distinct B, FP32 and the three split precisions (BF16,
BF16 with compensated HIGH products, FP16).

For every case: the sorted task keys (class bit included) bit-exact, kept and
LOW counts equal, and C within Higham's elementwise bound around the oracle's
product, built from each class's operands (m = n_b K + 1, one more rounding
per LOW product with FP16 operands).  Also seeded cases of sub-leaf culling
(performed sub-products against the leaf-32 oracle) and of sparsified trees
(stored leaves, keys, C bit-identical to the dense product)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def make_cases(count=36, seed=2024, nmax=700, first=0):
    rng = np.random.default_rng(seed)
    cases = []
    for c in range(first, first + count):
        leaf = int(rng.choice([16, 32, 64], p=[0.2, 0.4, 0.4]))
        n = int(rng.integers(1, nmax + 1))
        prec = "fp32" if leaf == 16 else str(rng.choice(["fp32", "bf16", "fp16"]))
        cases.append(dict(id=c, n=n, leaf=leaf, prec=prec,
                          tau=float(rng.choice([0.0, 1e-8, 1e-6, 1e-4, 1e-2])),
                          rate=float(rng.uniform(0.0, 0.5)), distinct=bool(rng.random() < 0.4),
                          theta=float(rng.choice([1e-3, 1e-1])), seed=int(rng.integers(1 << 30))))
    return cases


CASES = make_cases() + make_cases(count=24, seed=2025, nmax=1500, first=36)


def make_x3_cases(count=24, seed=2028, nmax=1200, first=400):
    rng = np.random.default_rng(seed)
    return [dict(id=c, n=int(rng.integers(1, nmax + 1)), leaf=int(rng.choice([32, 64])),
                 prec="bf16x3", tau=float(rng.choice([0.0, 1e-8, 1e-6, 1e-4, 1e-2])),
                 rate=float(rng.uniform(0.0, 0.5)), distinct=bool(rng.random() < 0.4),
                 theta=float(rng.choice([1e-3, 1e-1, 1e-5])), seed=int(rng.integers(1 << 30)))
            for c in range(first, first + count)]


X3_CASES = make_x3_cases()


def matrix(n, rate, seed, transpose=False):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    env = np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    A = rng.uniform(-1, 1, (n, n)) * env
    return np.ascontiguousarray((A.T if transpose else A).astype(np.float32))


def low_operand(X, S, fmt):
    if fmt in ("bf16", "bf16x3"):
        import torch
        return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(torch.bfloat16).to(
            torch.float64).numpy()
    e = oracle.fp16_exponent(S)
    h = (X * 2.0 ** e).astype(np.float16).astype(np.float64)
    return np.where(np.abs(h) < 2.0 ** -14, 0.0, h) * 2.0 ** -e


def high_operand(X, fmt):
    """|hi| + |lo| of the two bfloat16 parts (compensated HIGH products), else X."""
    if fmt != "bf16x3":
        return X
    import torch
    X32 = np.ascontiguousarray(X, dtype=np.float32)
    H = torch.from_numpy(X32).to(torch.bfloat16).to(torch.float32).numpy()
    L = torch.from_numpy(X32 - H).to(torch.bfloat16).to(torch.float64).numpy()
    return np.abs(H.astype(np.float64)) + np.abs(L)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"c{c['id']}-n{c['n']}-b{c['leaf']}-{c['prec']}")
def test_random_case(gpu, case):
    check_case(gpu, case)


@pytest.mark.parametrize("case", X3_CASES,
                         ids=lambda c: f"x{c['id']}-n{c['n']}-b{c['leaf']}-{c['prec']}")
def test_random_case_x3(gpu, case):
    check_case(gpu, case)


def check_case(gpu, case):
    import torch
    print(f"[random] {case}", flush=True)
    n, leaf, prec, tau = case["n"], case["leaf"], case["prec"], case["tau"]
    A = matrix(n, case["rate"], case["seed"])
    B = matrix(n, case["rate"] * 1.5, case["seed"] + 1, transpose=True) if case["distinct"] else A
    split = prec != "fp32"
    sA, sB = oracle.norms(A, leaf), oracle.norms(B, leaf)
    low = case["theta"] * float(np.sqrt(sA[0][0, 0]) * np.sqrt(sB[0][0, 0])) if split else 0.0
    ref = oracle.spamm(A, B, leaf, tau, low_tol=low, low_fmt=prec if split else "bf16")
    dA = torch.from_numpy(A).cuda()
    kw = dict(bf16=(prec in ("bf16", "bf16x3")), fp16=(prec == "fp16"))
    tA = gpu.build_tree(dA, leaf, **kw)
    tB = tA if B is A else gpu.build_tree(torch.from_numpy(B).cuda(), leaf, **kw)
    p = {"fp32": gpu.PREC_FP32, "bf16": gpu.PREC_SPLIT_BF16, "fp16": gpu.PREC_SPLIT_FP16,
         "bf16x3": gpu.PREC_SPLIT_BF16X3}[prec]
    plan = gpu.symbolic(tA, tB, tau, precision=p, low_tol=low)
    C = torch.full_like(dA, float("nan"))
    plan.numeric(C)
    torch.cuda.synchronize()
    st = plan.stats()
    assert np.array_equal(plan.tasks(), ref.keys)
    assert st["tasks"] == ref.K and st["tasks_low"] == ref.Klow
    # Higham's bound around the oracle's product
    d, np_ = oracle.depth(n, leaf)
    N = 1 << d
    PA = np.zeros((np_, np_))
    PB = np.zeros((np_, np_))
    PA[:n, :n], PB[:n, :n] = A, B
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    M = np.zeros((np_, np_))
    cnt = np.zeros((N, N), dtype=np.int64)
    for key in ref.keys:
        key = int(key)
        I, J = inv[(key >> 32) & 0x7FFFFFFF]
        k = key & 0xFFFFFFFF
        X = PA[I * leaf:(I + 1) * leaf, k * leaf:(k + 1) * leaf]
        Y = PB[k * leaf:(k + 1) * leaf, J * leaf:(J + 1) * leaf]
        if key >> 63:
            X, Y = low_operand(X, sA[-1][I, k], prec), low_operand(Y, sB[-1][k, J], prec)
        else:
            X, Y = high_operand(X, prec), high_operand(Y, prec)
        M[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] += np.abs(X) @ np.abs(Y)
        cnt[I, J] += 1
    per = leaf + 1 if prec == "fp16" else 3 * leaf if prec == "bf16x3" else leaf
    m = per * np.kron(cnt, np.ones((leaf, leaf))) + 1
    bound = (m * U32 / (1 - m * U32) * M + m * 2.0 ** -126)[:n, :n]
    got = C.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - ref.C) <= bound)


# ---- sub-leaf culling and sparsified trees, seeded -------------------------------

def tree_cases(count, seed, first):
    rng = np.random.default_rng(seed)
    return [dict(id=c, n=int(rng.integers(1, 1201)), tau=float(rng.choice([0.0, 1e-8, 1e-6, 1e-4, 1e-2])),
                 rate=float(rng.uniform(0.0, 0.5)), distinct=bool(rng.random() < 0.4),
                 seed=int(rng.integers(1 << 30)), leaf=int(rng.choice([16, 32, 64])))
            for c in range(first, first + count)]


SUB_CASES = tree_cases(16, 2026, 100)
SPARSE_CASES = tree_cases(16, 2027, 200)


def higham(A, B, leaf, keys, n):
    d, np_ = oracle.depth(n, leaf)
    N = 1 << d
    PA = np.zeros((np_, np_))
    PB = np.zeros((np_, np_))
    PA[:n, :n], PB[:n, :n] = np.abs(A), np.abs(B)
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    M = np.zeros((np_, np_))
    cnt = np.zeros((N, N), dtype=np.int64)
    for key in keys:
        I, J = inv[int(key) >> 32]
        k = int(key) & 0xFFFFFFFF
        M[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] += \
            PA[I * leaf:(I + 1) * leaf, k * leaf:(k + 1) * leaf] @ PB[k * leaf:(k + 1) * leaf, J * leaf:(J + 1) * leaf]
        cnt[I, J] += 1
    m = leaf * np.kron(cnt, np.ones((leaf, leaf))) + 1
    return (m * U32 / (1 - m * U32) * M + m * 2.0 ** -126)[:n, :n]


@pytest.mark.parametrize("case", SUB_CASES, ids=lambda c: f"sub{c['id']}-n{c['n']}")
def test_random_subleaf_case(gpu, case):
    """Leaf 64 with sub-leaf culling: the performed 32 x 32 sub-products equal
    the leaf-32 oracle's task set, C within the leaf-32 rounding bound."""
    import torch
    n, tau = case["n"], case["tau"]
    A = matrix(n, case["rate"], case["seed"])
    B = matrix(n, case["rate"] * 1.5, case["seed"] + 1, transpose=True) if case["distinct"] else A
    ref = oracle.spamm(A, B, 32, tau)
    dA = torch.from_numpy(A).cuda()
    tA = gpu.build_tree(dA, 64, subnorms=True)
    tB = tA if B is A else gpu.build_tree(torch.from_numpy(B).cuda(), 64, subnorms=True)
    plan = gpu.symbolic(tA, tB, tau, sub_cull=True)
    C = torch.full_like(dA, float("nan"))
    plan.numeric(C)
    torch.cuda.synchronize()
    assert np.array_equal(plan.subtasks(), ref.keys)
    assert plan.stats()["subtasks"] == ref.K
    got = C.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref.C) <= higham(A, B, 32, ref.keys, n))


@pytest.mark.parametrize("case", SPARSE_CASES, ids=lambda c: f"sp{c['id']}-n{c['n']}-b{c['leaf']}")
def test_random_sparse_case(gpu, case):
    """Epsilon-sparsified operands: stored leaves as the oracle's, task keys
    equal to the dense oracle product's, C bit-identical to the dense trees'."""
    import torch
    n, tau, leaf = case["n"], case["tau"], case["leaf"]
    A = matrix(n, case["rate"], case["seed"])
    B = matrix(n, case["rate"] * 1.5, case["seed"] + 1, transpose=True) if case["distinct"] else A
    nA2 = float(oracle.norms(A, leaf)[0][0, 0])
    nB2 = float(oracle.norms(B, leaf)[0][0, 0])
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    sA = gpu.build_tree_sparse(dA, leaf, tau, norm2_other=nB2)
    sB = sA if B is A else gpu.build_tree_sparse(dB, leaf, tau, norm2_other=nA2)
    _, kA = oracle.sparsify(A, leaf, tau, norm2_other=nB2)
    assert sA.storage()["stored"] == int(kA.sum())
    ref = oracle.spamm(A, B, leaf, tau, want_C=False)
    p = gpu.symbolic(sA, sB, tau)
    assert np.array_equal(p.tasks(), ref.keys)
    C1, C2 = torch.empty_like(dA), torch.empty_like(dA)
    p.numeric(C1)
    tA = gpu.build_tree(dA, leaf)
    tB = tA if B is A else gpu.build_tree(dB, leaf)
    gpu.multiply(tA, tB, tau, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
