"""Epsilon-sparsified trees on the GPU against the oracle.

* every norm tier bit-exact against the oracle's norms of the sparsified
  matrix (dropped leaves zeroed), root before dropping equal to the dense
  root;
* stored leaves = the oracle's kept leaves, and fewer device bytes than the
  dense tree;
* both packed copies reproduce the sparsified matrix;
* a product of sparsified trees: task keys bit-exact against the oracle's
  dense product, C bit-identical to the GPU product of the dense trees
  (same products, same owner and k order), also in split precision and with
  two operands sparsified against the larger norm;
* NaN in A is reported even where it would sit in a dropped leaf; every leaf
  dropped gives C = 0; tau = 0 keeps every nonzero leaf.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def decay(n, rate, seed, sym=True):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return A.astype(np.float32)


CASES = {
    # name: (A, leaf, tau)
    "expdecay-n1024-b32": lambda: (workloads.exp_decay(1024, 0.1, 0), 32, 1e-6),
    "decay-n700-b64": lambda: (decay(700, 0.1, 1), 64, 1e-5),
    "decay-n500-b16": lambda: (decay(500, 0.3, 2), 16, 1e-6),
    "decay-n333-b32": lambda: (decay(333, 0.2, 3), 32, 1e-3),
    "tau0-n300-b32": lambda: (decay(300, 0.5, 4), 32, 0.0),
}


def padded(A, leaf):
    d, np_ = oracle.depth(A.shape[0], leaf)
    P = np.zeros((np_, np_), dtype=np.float32)
    P[:A.shape[0], :A.shape[0]] = A
    return P


@pytest.fixture(scope="module")
def runs(gpu):
    import torch
    cache = {}

    def get(name):
        if name not in cache:
            A, leaf, tau = CASES[name]()
            S, keep = oracle.sparsify(A, leaf, tau)
            dA = torch.from_numpy(A).cuda()
            sparse = gpu.build_tree_sparse(dA, leaf, tau)
            dense = gpu.build_tree(dA, leaf)
            cache[name] = dict(A=A, S=S, keep=keep, leaf=leaf, tau=tau, dA=dA, sparse=sparse,
                               dense=dense)
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_sparse_norms_and_storage(runs, name):
    r = runs(name)
    t = r["sparse"]
    want = oracle.norms(r["S"], r["leaf"])
    for tier in range(t.depth + 1):
        assert np.array_equal(t.norms(tier), want[tier]), tier
    assert t.norm2 == want[0][0, 0]
    st = t.storage()
    assert st["stored"] == int(r["keep"].sum())
    assert st["total"] == r["keep"].size
    if name.startswith("tau0"):
        assert st["stored"] == int(np.count_nonzero(oracle.norms(r["A"], r["leaf"])[-1]))
    else:
        assert st["stored"] < st["total"]
        assert st["bytes"] < r["dense"].storage()["bytes"]


@pytest.mark.parametrize("name", list(CASES))
def test_sparse_packed_copies(runs, name):
    r = runs(name)
    want = padded(r["S"], r["leaf"])
    for copy in (0, 1):
        assert np.array_equal(r["sparse"].matrix(copy), want)


@pytest.mark.parametrize("name", list(CASES))
def test_sparse_product_equals_dense(gpu, runs, name):
    import torch
    r = runs(name)
    ref = oracle.spamm(r["A"], r["A"], r["leaf"], r["tau"], want_C=False)
    p = gpu.symbolic(r["sparse"], r["sparse"], r["tau"])
    assert np.array_equal(p.tasks(), ref.keys)
    C1, C2 = torch.empty_like(r["dA"]), torch.empty_like(r["dA"])
    p.numeric(C1)
    gpu.multiply(r["dense"], r["dense"], r["tau"], C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


def test_sparse_split_precision_equals_dense(gpu):
    import torch
    A = decay(800, 0.1, 5)
    dA = torch.from_numpy(A).cuda()
    tau, low = 1e-6, 1e-2
    s = gpu.build_tree_sparse(dA, 32, tau, bf16=True)
    d = gpu.build_tree(dA, 32, bf16=True)
    assert s.storage()["stored"] < s.storage()["total"]
    ps = gpu.symbolic(s, s, tau, precision=gpu.PREC_SPLIT_BF16, low_tol=low)
    pd = gpu.symbolic(d, d, tau, precision=gpu.PREC_SPLIT_BF16, low_tol=low)
    assert np.array_equal(ps.tasks(), pd.tasks())
    C1, C2 = torch.empty_like(dA), torch.empty_like(dA)
    ps.numeric(C1)
    pd.numeric(C2)
    torch.cuda.synchronize()
    assert ps.stats()["tasks_low"] > 0
    assert torch.equal(C1, C2)


def test_two_sparse_operands(gpu):
    import torch
    A = decay(512, 0.2, 6, sym=False)
    B = 30.0 * decay(512, 0.25, 7, sym=False)
    tau = 1e-4
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    nA2 = gpu.build_tree(dA, 32).norm2
    nB2 = gpu.build_tree(dB, 32).norm2
    sA = gpu.build_tree_sparse(dA, 32, tau, norm2_other=nB2)
    sB = gpu.build_tree_sparse(dB, 32, tau, norm2_other=nA2)
    _, kA = oracle.sparsify(A, 32, tau, norm2_other=nB2)
    _, kB = oracle.sparsify(B, 32, tau, norm2_other=nA2)
    assert sA.storage()["stored"] == kA.sum() and sB.storage()["stored"] == kB.sum()
    ref = oracle.spamm(A, B, 32, tau, want_C=False)
    p = gpu.symbolic(sA, sB, tau)
    assert np.array_equal(p.tasks(), ref.keys)
    C1, C2 = torch.empty_like(dA), torch.empty_like(dA)
    p.numeric(C1)
    gpu.multiply(gpu.build_tree(dA, 32), gpu.build_tree(dB, 32), tau, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


def test_sparse_nan_and_all_dropped(gpu):
    import torch
    A = decay(300, 0.3, 8)
    bad = A.copy()
    bad[290, 5] = np.nan               # far off the diagonal: its leaf would be dropped
    with pytest.raises(gpu.SpammError) as ei:
        gpu.build_tree_sparse(torch.from_numpy(bad).cuda(), 32, 1e-4)
    assert ei.value.code == gpu.SPAMM_E_NONFINITE
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree_sparse(dA, 32, 1e30)
    assert t.storage()["stored"] == 0 and t.norm2 == 0.0
    C = torch.full_like(dA, float("nan"))
    st = gpu.multiply_ex(t, t, 1e30, C)
    assert st["tasks"] == 0
    assert torch.count_nonzero(C).item() == 0


def test_sparse_full_size_cluster(gpu):
    """cluster300-n7500 at tau = 1e-8, leaf 32: stored leaves against the
    oracle's, task keys against the oracle's dense product, C bit-identical to
    the dense-tree product."""
    import torch
    wl = workloads.WORKLOADS["cluster300-n7500"]
    A = wl.matrix()
    print(f"\n[sparse] {wl.name} tau={wl.tau:g}", flush=True)
    dA = torch.from_numpy(A).cuda()
    s = gpu.build_tree_sparse(dA, wl.leaf, wl.tau)
    d = gpu.build_tree(dA, wl.leaf)
    _, keep = oracle.sparsify(A, wl.leaf, wl.tau)
    st = s.storage()
    assert st["stored"] == int(keep.sum()) < st["total"]
    p = gpu.symbolic(s, s, wl.tau)
    ref = oracle.spamm(A, A, wl.leaf, wl.tau, want_C=False)
    assert np.array_equal(p.tasks(), ref.keys)
    C1, C2 = torch.empty_like(dA), torch.empty_like(dA)
    p.numeric(C1)
    gpu.multiply(d, d, wl.tau, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


def test_sparse_largest_order_n65536(gpu):
    """The largest order of leaf-64 trees (n = 65536, N = 1024) sparsified at
    tau = 1e-6: stored leaves against the oracle's, task keys against the
    oracle's dense product, C bit-identical to the dense-tree product."""
    import torch
    A = workloads.exp_decay(65536, 0.5, 8)
    tau = 1e-6
    print(f"\n[sparse] expdecay0.5-n65536 tau={tau:g}", flush=True)
    dA = torch.from_numpy(A).cuda()
    s = gpu.build_tree_sparse(dA, 64, tau)
    _, keep = oracle.sparsify(A, 64, tau)
    st = s.storage()
    print(f"[sparse] stored {st['stored']} of {st['total']} leaves", flush=True)
    assert st["stored"] == int(keep.sum()) < st["total"]
    p = gpu.symbolic(s, s, tau)
    ref = oracle.spamm(A, A, 64, tau, want_C=False)
    assert np.array_equal(p.tasks(), ref.keys)
    C1 = torch.empty_like(dA)
    p.numeric(C1)
    del p, s
    d = gpu.build_tree(dA, 64)
    C2 = torch.empty_like(dA)
    gpu.multiply(d, d, tau, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    del d, C1, C2, dA
    torch.cuda.empty_cache()
