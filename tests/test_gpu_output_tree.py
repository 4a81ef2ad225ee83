"""The tree of a product's output (spamm_build_tree_output, Sec. II.C) on the
GPU: built from C = A B and the plan that computed it, reading only the
leaves of C that a kept leaf product reaches.

* every norm tier bit-exact against the dense tree of the same C (and the
  leaf tier against the oracle's norms of the oracle's C where the two C
  agree bit for bit: the FP32 products of a leaf are summed in the same
  order), and the leaves stored = the output leaves the oracle's task keys
  reach;
* both packed copies reproduce C on the reached leaves and zero elsewhere,
  also when C holds garbage on the leaves no product reaches;
* the next product (the square of the output, one step of a squaring chain)
  taken on the output tree gives the task keys and the C of the dense tree bit
  for bit, in FP32 and in both split precisions;
* depth 0 (a single leaf), an output with no reached leaf at all, and
  a product of epsilon-sparsified BF16 trees with 64 x 64 leaves (the wide
  split kernel addressing its leaves through the slot map).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def decay(n, rate, seed):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    return (np.triu(A) + np.triu(A, 1).T).astype(np.float32)


# name: (n, decay rate, leaf, tau, precision name, seed)
CASES = {
    "fp32-n1000-b32": (1000, 0.15, 32, 1e-6, "fp32", 1),
    "fp32-n700-b64": (700, 0.1, 64, 1e-5, "fp32", 2),
    "fp32-n450-b16": (450, 0.3, 16, 1e-6, "fp32", 3),
    "bf16-n1024-b32": (1024, 0.12, 32, 1e-7, "bf16", 4),
    "fp16-n900-b32": (900, 0.12, 32, 1e-7, "fp16", 5),
    "bf16-n1100-b64": (1100, 0.08, 64, 1e-6, "bf16", 6),
}
THETA = 1e-3


def prec_args(gpu, name):
    if name == "fp32":
        return dict(precision=gpu.PREC_FP32), {}
    if name == "bf16":
        return dict(precision=gpu.PREC_SPLIT_BF16, low_rel=THETA), dict(bf16=True)
    return dict(precision=gpu.PREC_SPLIT_FP16, low_rel=THETA), dict(fp16=True)


def reached_leaves(keys, N):
    """Output leaves (linear index) with at least one kept product."""
    lc = np.unique((np.asarray(keys, dtype=np.uint64) >> np.uint64(32)) & np.uint64(0x7FFFFFFF))
    out = np.zeros(N * N, dtype=bool)
    out[lc.astype(np.int64)] = True
    return out


def inv(l, N):
    for i in range(N):
        for j in range(N):
            if oracle.linear_index(i, j) == l:
                return i, j
    raise ValueError(l)


@pytest.fixture(scope="module")
def runs(gpu):
    import torch
    cache = {}

    def get(name):
        if name in cache:
            return cache[name]
        n, rate, leaf, tau, pname, seed = CASES[name]
        A = decay(n, rate, seed)
        dA = torch.from_numpy(A).cuda()
        sym, tf = prec_args(gpu, pname)
        T = gpu.build_tree(dA, leaf, **tf)
        P = gpu.symbolic(T, T, tau, **sym)
        C = torch.empty_like(dA)
        P.numeric(C)
        torch.cuda.synchronize()
        out = gpu.build_tree_output(C, P, **tf)
        dense = gpu.build_tree(C, leaf, **tf)
        cache[name] = dict(A=A, dA=dA, leaf=leaf, tau=tau, sym=sym, tf=tf, T=T, P=P, C=C,
                           out=out, dense=dense, keys=P.tasks())
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_output_tree_norms_equal_dense_tree(runs, name):
    r = runs(name)
    d = r["dense"].depth
    for t in range(d + 1):
        a, b = r["out"].norms(t), r["dense"].norms(t)
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), f"tier {t}"
    N = 1 << d
    reached = reached_leaves(r["keys"], N)
    st = r["out"].storage()
    assert st["stored"] == int(reached.sum()) and st["total"] == N * N
    # an unreached leaf has norm +0; a reached one is what C holds
    leafn = r["out"].norms(d).reshape(-1)
    lin = np.array([[oracle.linear_index(i, j) for j in range(N)] for i in range(N)]).reshape(-1)
    by_lin = np.empty(N * N)
    by_lin[lin] = leafn
    assert np.all(by_lin[~reached] == 0.0)
    assert not np.signbit(by_lin[~reached]).any()


@pytest.mark.parametrize("name", list(CASES))
def test_output_tree_copies_reproduce_c(runs, name):
    r = runs(name)
    d = r["dense"].depth
    N = 1 << d
    n = r["A"].shape[0]
    reached = reached_leaves(r["keys"], N)
    M = np.zeros((N * r["leaf"],) * 2, dtype=bool)
    for i in range(N):
        for j in range(N):
            if reached[oracle.linear_index(i, j)]:
                M[i * r["leaf"]:(i + 1) * r["leaf"], j * r["leaf"]:(j + 1) * r["leaf"]] = True
    Cp = np.zeros((N * r["leaf"],) * 2, dtype=np.float32)
    Cp[:n, :n] = r["C"].cpu().numpy()
    want = np.where(M, Cp, np.float32(0.0))
    for copy in (0, 1):
        got = r["out"].matrix(copy)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), f"copy {copy}"
    # the leaves no product reaches are exactly zero in C itself
    assert np.all(Cp[~M] == 0.0)


@pytest.mark.parametrize("name", list(CASES))
def test_square_of_output_tree_equals_dense(runs, name, gpu):
    """One squaring-chain step X_2 = X_1 X_1 on the output tree of X_1 = A A."""
    import torch
    r = runs(name)
    po = gpu.symbolic(r["out"], r["out"], r["tau"], **r["sym"])
    pd = gpu.symbolic(r["dense"], r["dense"], r["tau"], **r["sym"])
    ko, kd = po.tasks(), pd.tasks()
    assert len(kd) > 0
    assert np.array_equal(ko, kd)
    C1, C2 = torch.empty_like(r["C"]), torch.empty_like(r["C"])
    po.numeric(C1)
    pd.numeric(C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


def test_unreached_leaves_are_not_read(gpu):
    """C with NaN on every leaf the product does not reach: the output tree
    equals the dense tree of the true product."""
    import torch
    A = decay(768, 0.25, 7)
    dA = torch.from_numpy(A).cuda()
    T = gpu.build_tree(dA, 32)
    P = gpu.symbolic(T, T, 1e-5)
    C = torch.empty_like(dA)
    P.numeric(C)
    torch.cuda.synchronize()
    N = 1 << T.depth                    # 768 = 24 leaves, padded to 32
    reached = reached_leaves(P.tasks(), N)
    assert not reached.all()
    bad = C.clone()
    for i in range(N):
        for j in range(N):
            if not reached[oracle.linear_index(i, j)]:
                bad[i * 32:(i + 1) * 32, j * 32:(j + 1) * 32] = float("nan")
    out = gpu.build_tree_output(bad, P)
    dense = gpu.build_tree(C, 32)
    for t in range(T.depth + 1):
        assert np.array_equal(out.norms(t).view(np.uint64), dense.norms(t).view(np.uint64))
    # NaN on a reached leaf is reported
    bad2 = C.clone()
    l0 = int(np.flatnonzero(reached)[0])
    i0, j0 = inv(l0, N)
    bad2[i0 * 32, j0 * 32] = float("nan")
    with pytest.raises(gpu.SpammError) as ei:
        gpu.build_tree_output(bad2, P)
    assert ei.value.code == gpu.SPAMM_E_NONFINITE


def test_single_leaf_and_nothing_reached(gpu):
    import torch
    A = decay(20, 0.1, 8)
    dA = torch.from_numpy(A).cuda()
    T = gpu.build_tree(dA, 32)
    assert T.depth == 0
    P = gpu.symbolic(T, T, 0.0)
    C = torch.empty_like(dA)
    P.numeric(C)
    torch.cuda.synchronize()
    out = gpu.build_tree_output(C, P)
    assert out.storage()["stored"] == 1
    assert np.array_equal(out.norms(0).view(np.uint64),
                          gpu.build_tree(C, 32).norms(0).view(np.uint64))
    # tau above every norm product: no product kept, C = 0, nothing stored
    B = decay(300, 0.2, 9)
    dB = torch.from_numpy(B).cuda()
    TB = gpu.build_tree(dB, 32)
    PB = gpu.symbolic(TB, TB, 1e6)
    CB = torch.full_like(dB, 7.0)
    PB.numeric(CB)
    torch.cuda.synchronize()
    assert len(PB.tasks()) == 0
    out = gpu.build_tree_output(CB, PB)
    assert out.storage()["stored"] == 0 and out.norm2 == 0.0


def test_sparse_bf16_leaf64_product_equals_dense(gpu):
    """Epsilon-sparsified BF16 trees with 64 x 64 leaves at depth >= 2: the
    wide split kernel reads their leaves through the slot map; same keys and
    C as the dense trees."""
    import torch
    A = decay(1000, 0.08, 10)
    dA = torch.from_numpy(A).cuda()
    tau = 1e-5
    s = gpu.build_tree_sparse(dA, 64, tau, bf16=True)
    d = gpu.build_tree(dA, 64, bf16=True)
    assert d.depth >= 2 and s.storage()["stored"] < s.storage()["total"]
    ps = gpu.symbolic(s, s, tau, precision=gpu.PREC_SPLIT_BF16, low_rel=THETA)
    pd = gpu.symbolic(d, d, tau, precision=gpu.PREC_SPLIT_BF16, low_rel=THETA)
    assert np.array_equal(ps.tasks(), pd.tasks())
    assert ps.stats()["tasks_low"] > 0
    C1, C2 = torch.empty_like(dA), torch.empty_like(dA)
    ps.numeric(C1)
    pd.numeric(C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
