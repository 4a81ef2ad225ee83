"""GPU path against the FP64 oracle on the same seeded inputs.

* norms of every tier: bit-exact (FP64, canonical order);
* packed leaves: bit-exact copy of the zero-padded matrix;
* kept task list (sorted u64 keys) and kept counts per tier: bit-exact;
* C: within Higham's dot-product bound per element,
  |C_gpu - C_oracle| <= gamma_m * sum_kept |A||B| + m * 2^-126 * scale,
  gamma_m = m u / (1 - m u), u = 2^-24, m = n_b * K_ij + 1, and within the
  product's contract 1e-5 ||A||_F ||B||_F;
* repeat runs are bit-identical.
"""
import math

import numpy as np
import pytest

import inputs
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


def make(name):
    """(A, B or None for B = A, leaf, tau)"""
    if name == "expdecay-n1024":
        wl = workloads.WORKLOADS[name]
        return wl.matrix(), None, wl.leaf, wl.tau
    if name == "expdecay-n1024-tau0":
        return workloads.exp_decay(1024, 0.1, 0), None, 32, 0.0
    if name == "ragged-b16":
        return decay(300, 0.05, 1), None, 16, 1e-5
    if name == "odd-n-b32":
        return decay(333, 0.04, 2), None, 32, 1e-4
    if name == "n2mod4-b64":
        return decay(450, 0.03, 3), None, 64, 1e-6
    if name == "single-tile":
        return decay(20, 0.1, 4), None, 32, 0.0
    if name == "exact-tile-b64":
        return decay(64, 0.1, 5), None, 64, 0.0
    if name == "depth1-b64":
        return decay(100, 0.05, 6), None, 64, 1e-3
    if name == "nonsym-b32":
        return decay(256, 0.05, 7, sym=False), decay(256, 0.09, 8, sym=False), 32, 1e-3
    if name == "zero-tiles-b16":
        A = decay(256, 0.02, 9)
        A[16:48, :] = 0.0
        A[:, 16:48] = 0.0
        A[100:130, 150:190] = 0.0
        return A, None, 16, 1e-5
    if name == "denormals-b16":
        return workloads.exp_decay(512, 0.6, 0), None, 16, 0.0
    if name == "denormals-tau-b16":
        return workloads.exp_decay(512, 0.6, 0), None, 16, 1e-40
    if name == "algdecay-b64":
        return workloads.alg_decay(1000, 3.0, 0), None, 64, 1e-6
    if name.startswith("sumorder-b"):
        # leaf norms whose bits depend on the summation order (inputs.sum_order)
        b = int(name[len("sumorder-b"):])
        return inputs.sum_order(b), None, b, 0.0
    raise KeyError(name)


CASES = ["expdecay-n1024", "expdecay-n1024-tau0", "ragged-b16", "odd-n-b32", "n2mod4-b64",
         "single-tile", "exact-tile-b64", "depth1-b64", "nonsym-b32", "zero-tiles-b16",
         "denormals-b16", "denormals-tau-b16", "algdecay-b64", "sumorder-b16", "sumorder-b32",
         "sumorder-b64"]


class GpuRun:
    def __init__(self, sp, A, B, leaf, tau):
        import torch
        self.dA = torch.from_numpy(A).cuda()
        self.tA = sp.build_tree(self.dA, leaf)
        if B is None:
            self.tB = self.tA
        else:
            self.dB = torch.from_numpy(B).cuda()
            self.tB = sp.build_tree(self.dB, leaf)
        self.plan = sp.symbolic(self.tA, self.tB, tau)
        C = torch.full_like(self.dA, float("nan"))    # every element must be written
        self.plan.numeric(C)
        torch.cuda.synchronize()
        self.C = C.cpu().numpy()


def padded(A, leaf):
    d, np_ = oracle.depth(A.shape[0], leaf)
    P = np.zeros((np_, np_), dtype=np.float32)
    P[:A.shape[0], :A.shape[0]] = A
    return P, d


def rounding_bound(A, B, leaf, keys):
    """gamma_m * sum_kept |A_ik||B_kj| elementwise, m = leaf * K_ij + 1."""
    PA, d = padded(A, leaf)
    PB, _ = padded(B, leaf)
    N = 1 << d
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    M = np.zeros(PA.shape, dtype=np.float64)
    cnt = np.zeros((N, N), dtype=np.int64)
    aA, aB = np.abs(PA.astype(np.float64)), np.abs(PB.astype(np.float64))
    for key in keys:
        I, J = inv[int(key) >> 32]
        k = int(key) & 0xFFFFFFFF
        M[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] += (
            aA[I * leaf:(I + 1) * leaf, k * leaf:(k + 1) * leaf]
            @ aB[k * leaf:(k + 1) * leaf, J * leaf:(J + 1) * leaf])
        cnt[I, J] += 1
    m = leaf * np.kron(cnt, np.ones((leaf, leaf))) + 1
    gamma = m * U32 / (1 - m * U32)
    scale = max(1.0, float(aA.max()), float(aB.max())) ** 2
    n = A.shape[0]
    return (gamma * M + m * 2.0 ** -126 * scale)[:n, :n]


@pytest.fixture(scope="module")
def runs(gpu):
    cache = {}

    def get(name):
        if name not in cache:
            A, B, leaf, tau = make(name)
            Bm = A if B is None else B
            ref = oracle.spamm(A, Bm, leaf, tau)
            cache[name] = (A, Bm, leaf, tau, ref, GpuRun(gpu, A, B, leaf, tau))
        return cache[name]
    return get


@pytest.mark.parametrize("name", CASES)
def test_norms_bit_exact(runs, name):
    A, B, leaf, tau, ref, g = runs(name)
    for tree, M in ((g.tA, A), (g.tB, B)):
        tiers = oracle.norms(M, leaf)
        assert tree.depth == len(tiers) - 1
        for t, want in enumerate(tiers):
            got = tree.norms(t)
            assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), f"tier {t}"
        assert tree.norm2 == tiers[0][0, 0]


@pytest.mark.parametrize("name", CASES)
def test_packed_leaves_are_padded_copy(runs, name):
    A, B, leaf, tau, ref, g = runs(name)
    P, _ = padded(A, leaf)
    assert np.array_equal(g.tA.matrix(0).view(np.uint32), P.view(np.uint32))
    assert np.array_equal(g.tA.matrix(1).view(np.uint32), P.view(np.uint32))


@pytest.mark.parametrize("name", CASES)
def test_task_list_bit_exact(runs, name):
    A, B, leaf, tau, ref, g = runs(name)
    keys = g.plan.tasks()
    assert keys.dtype == np.uint64
    assert len(keys) == ref.K
    assert np.array_equal(keys, ref.keys)
    st = g.plan.stats()
    assert st["kept"] == [int(v) for v in ref.Kt]
    assert st["tasks"] == ref.K
    assert st["flops"] == 2.0 * leaf ** 3 * ref.K


@pytest.mark.parametrize("name", CASES)
def test_product_within_bounds(runs, name):
    A, B, leaf, tau, ref, g = runs(name)
    assert np.all(np.isfinite(g.C)), "some element of C was not written"
    err = np.abs(g.C.astype(np.float64) - ref.C)
    bound = rounding_bound(A, B, leaf, ref.keys)
    worst = float(np.max(err - bound))
    assert worst <= 0.0, f"rounding bound exceeded by {worst}"
    nA = math.sqrt(g.tA.norm2)
    nB = math.sqrt(g.tB.norm2)
    assert err.max() <= 1e-5 * nA * nB


def test_repeat_runs_bit_identical(gpu):
    import torch
    A, _, leaf, tau = make("expdecay-n1024")
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, leaf)
    C1 = torch.empty_like(dA)
    C2 = torch.empty_like(dA)
    gpu.multiply(t, t, tau, C1)
    gpu.multiply(t, t, tau, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1.view(torch.int32), C2.view(torch.int32))
    t2 = gpu.build_tree(dA, leaf)
    assert np.array_equal(t2.norms(t2.depth), t.norms(t.depth))


def test_one_call_multiply_matches_plan(runs, gpu):
    import torch
    A, B, leaf, tau, ref, g = runs("nonsym-b32")
    C = torch.empty_like(g.dA)
    st = gpu.multiply_ex(g.tA, g.tB, tau, C)
    assert np.array_equal(C.cpu().numpy().view(np.uint32), g.C.view(np.uint32))
    assert st["tasks"] == ref.K and st["numeric_ms"] >= 0.0 and st["symbolic_ms"] >= 0.0


def test_output_may_alias_tree_source(gpu):
    import torch
    A, _, leaf, tau = make("ragged-b16")
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, leaf)
    C = torch.empty_like(dA)
    gpu.multiply(t, t, tau, C)
    gpu.multiply(t, t, tau, dA)          # X <- X X in place
    torch.cuda.synchronize()
    assert torch.equal(C, dA)


def test_zero_matrix_gives_zero_product(gpu):
    import torch
    Z = torch.zeros(300, 300, device="cuda")
    t = gpu.build_tree(Z, 32)
    assert t.norm2 == 0.0
    C = torch.full_like(Z, 7.0)
    p = gpu.symbolic(t, t, 0.0)
    p.numeric(C)
    torch.cuda.synchronize()
    assert p.stats()["tasks"] == 0 and len(p.tasks()) == 0
    assert torch.count_nonzero(C).item() == 0


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_nonfinite_input_rejected(gpu, bad):
    import torch
    A = torch.from_numpy(decay(200, 0.05, 1)).cuda()
    A[123, 45] = bad
    with pytest.raises(gpu.SpammError) as ei:
        gpu.build_tree(A, 32)
    assert ei.value.code == gpu.SPAMM_E_NONFINITE


def test_bad_arguments_rejected(gpu):
    import torch
    A = torch.from_numpy(decay(200, 0.05, 1)).cuda()
    t32 = gpu.build_tree(A, 32)
    t16 = gpu.build_tree(A, 16)
    tb = gpu.build_tree(A[:100, :100].contiguous(), 32)
    for tau in (-1.0, float("nan"), float("inf"), 1e-200):
        with pytest.raises(gpu.SpammError) as ei:
            gpu.symbolic(t32, t32, tau)
        assert ei.value.code == gpu.SPAMM_E_INVAL
    for other in (t16, tb):
        with pytest.raises(gpu.SpammError) as ei:
            gpu.symbolic(t32, other, 1e-6)
        assert ei.value.code == gpu.SPAMM_E_MISMATCH
    with pytest.raises(gpu.SpammError) as ei:
        t32.norms(t32.depth + 1)
    assert ei.value.code == gpu.SPAMM_E_INVAL


def test_binding_keeps_trees_alive_for_their_plans(gpu):
    """A tree that a live plan reads cannot be freed through the binding; once
    the plan is freed it can, and a freed handle is refused."""
    import torch
    A = torch.from_numpy(np.eye(100, dtype=np.float32)).cuda()
    t = gpu.build_tree(A, 32)
    p = gpu.symbolic(t, t, 0.0)
    with pytest.raises(ValueError):
        t.free()
    C = torch.empty_like(A)
    p.numeric(C)
    torch.cuda.synchronize()
    assert torch.equal(C, A)
    p.free()
    t.free()
    with pytest.raises(ValueError):
        gpu.symbolic(t, t, 0.0)
