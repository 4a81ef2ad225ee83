"""GPU path against the oracle at the full sizes of the named workloads, in the
launch configuration bench.py times (one build + one multiply per matrix).

Where the oracle can afford the whole computation (every norm tier, the kept
task set and its count per tier) the comparison is complete and bit-exact; the
product C is compared on seeded samples of output leaves that the oracle
computes one by one (per-leaf recursion), including diagonal leaves where the
entries are largest, the last (partly padded) row and column of leaves, and
leaves with no kept product.  Bound per element: Higham's
|C_gpu - C_oracle| <= gamma_m sum_kept |A_ik||B_kj| + m 2^-126,
gamma_m = m u/(1 - m u), u = 2^-24, m = n_b K_ij + 1.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def leaf_block(M, I, J, leaf, n):
    out = np.zeros((leaf, leaf), dtype=np.float64)
    r0, c0 = I * leaf, J * leaf
    r1, c1 = min(r0 + leaf, n), min(c0 + leaf, n)
    if r0 < n and c0 < n:
        out[:r1 - r0, :c1 - c0] = M[r0:r1, c0:c1]
    return out


def tile_bound(A, leaf, I, J, klist):
    n = A.shape[0]
    M = np.zeros((leaf, leaf))
    for k in klist:
        M += np.abs(leaf_block(A, I, k, leaf, n)) @ np.abs(leaf_block(A, k, J, leaf, n))
    m = leaf * len(klist) + 1
    gamma = m * U32 / (1 - m * U32)
    return gamma * M + m * 2.0 ** -126


def choose_tiles(N, seed, count=48):
    rng = np.random.default_rng(seed)
    tiles = {(int(i), int(j)) for i, j in rng.integers(0, N, size=(count, 2))}
    tiles |= {(int(i), int(i)) for i in rng.integers(0, N, size=count // 4)}
    tiles |= {(N - 1, N - 1), (N - 1, 0), (0, N - 1), (0, 0), (N // 2, N // 2 + 1)}
    return sorted(tiles)


class FullRun:
    def __init__(self, sp, name, tau):
        import torch
        wl = workloads.WORKLOADS[name]
        self.wl, self.tau, self.leaf, self.n = wl, tau, wl.leaf, wl.n
        print(f"\n[fullsize] {name} tau={tau:g}: generating", flush=True)
        self.A = wl.matrix()
        dA = torch.from_numpy(self.A).cuda()
        self.tree = sp.build_tree(dA, wl.leaf)
        self.plan = sp.symbolic(self.tree, self.tree, tau)
        C = torch.full_like(dA, float("nan"))
        self.plan.numeric(C)
        torch.cuda.synchronize()
        del dA
        self.C = C.cpu().numpy()
        del C
        self.keys = self.plan.tasks()
        self.stats = self.plan.stats()
        print(f"[fullsize] {name}: K={self.stats['tasks']}", flush=True)


def check_norms(run):
    tiers = oracle.norms(run.A, run.leaf)
    for t, want in enumerate(tiers):
        got = run.tree.norms(t)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), f"tier {t}"


def check_sampled_product(run, seed):
    d = run.tree.depth
    N = 1 << d
    tiles = choose_tiles(N, seed)
    Ct, counts, kl = oracle.spamm_tiles(run.A, run.A, run.leaf, run.tau, tiles, threads=16,
                                        want_klists=True)
    hi = run.keys >> np.uint64(32)
    worst = -np.inf
    for s, (I, J) in enumerate(tiles):
        ks = kl[s, :counts[s]]
        lc = np.uint64(oracle.linear_index(I, J))
        lo, up = np.searchsorted(hi, lc, "left"), np.searchsorted(hi, lc, "right")
        gpu_k = (run.keys[lo:up] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        assert np.array_equal(gpu_k, ks.astype(np.int64)), (I, J)
        got = leaf_block(run.C, I, J, run.leaf, run.n)
        want = Ct[s]
        assert np.all(np.isfinite(got))
        err = np.abs(got - want)
        worst = max(worst, float(np.max(err - tile_bound(run.A, run.leaf, I, J, ks))))
        if counts[s] == 0:
            assert not np.any(got)
    assert worst <= 0.0, f"rounding bound exceeded by {worst}"
    nrm2 = run.tree.norm2
    err = max(float(np.abs(leaf_block(run.C, I, J, run.leaf, run.n) - Ct[s]).max())
              for s, (I, J) in enumerate(tiles))
    assert err <= 1e-5 * nrm2   # 1e-5 ||A||_F ||B||_F with B = A


# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cluster300(gpu):
    return FullRun(gpu, "cluster300-n7500", 1e-8)


def test_cluster300_norms(cluster300):
    check_norms(cluster300)


def test_cluster300_task_set(cluster300):
    r = cluster300
    ref = oracle.spamm(r.A, r.A, r.leaf, r.tau, want_C=False)
    assert r.stats["kept"] == [int(v) for v in ref.Kt]
    assert np.array_equal(r.keys, ref.keys)


def test_cluster300_sampled_product(cluster300):
    check_sampled_product(cluster300, seed=11)


@pytest.mark.parametrize("tau", [1e-4, 1e-6, 1e-8, 1e-10])
def test_algdecay_tau_sweep(gpu, tau):
    r = FullRun(gpu, "algdecay-n16384", tau)
    ref = oracle.spamm(r.A, r.A, r.leaf, tau, want_C=False)
    assert r.stats["kept"] == [int(v) for v in ref.Kt]
    assert np.array_equal(r.keys, ref.keys)
    check_sampled_product(r, seed=int(-math.log10(tau)))
    if tau == 1e-4:
        check_norms(r)


@pytest.fixture(scope="module")
def cluster1310(gpu):
    return FullRun(gpu, "cluster1310-n32750", 1e-8)


def test_cluster1310_norms(cluster1310):
    check_norms(cluster1310)


def test_cluster1310_task_set(cluster1310):
    r = cluster1310
    ref = oracle.spamm(r.A, r.A, r.leaf, r.tau, want_C=False)
    assert r.stats["kept"] == [int(v) for v in ref.Kt]
    assert len(r.keys) == ref.K
    assert np.array_equal(r.keys, ref.keys)


def test_cluster1310_sampled_product(cluster1310):
    check_sampled_product(cluster1310, seed=5)


class MatrixRun(FullRun):
    """FullRun on a given matrix (not a named workload)."""

    def __init__(self, sp, A, leaf, tau, label):
        import torch
        self.A, self.leaf, self.tau, self.n = A, leaf, tau, A.shape[0]
        print(f"\n[fullsize] {label} tau={tau:g}", flush=True)
        dA = torch.from_numpy(A).cuda()
        self.tree = sp.build_tree(dA, leaf)
        self.plan = sp.symbolic(self.tree, self.tree, tau)
        C = torch.full_like(dA, float("nan"))
        self.plan.numeric(C)
        torch.cuda.synchronize()
        del dA
        self.C = C.cpu().numpy()
        del C
        self.keys = self.plan.tasks()
        self.stats = self.plan.stats()
        print(f"[fullsize] {label}: K={self.stats['tasks']}", flush=True)


def test_largest_grid_n16384_leaf16(gpu):
    """The largest grid the library takes: N = 1024 leaves per dimension
    (n = 16384 at n_b = 16, 10 tiers below the root, worst-case task arena
    capacities); every norm tier and the whole task set bit-exact, C on
    sampled leaves; one more row or column is out of range."""
    import torch
    A = workloads.exp_decay(16384, 0.5, 3)
    r = MatrixRun(gpu, A, 16, 1e-6, "expdecay0.5-n16384-leaf16")
    assert r.tree.depth == 10
    check_norms(r)
    ref = oracle.spamm(r.A, r.A, 16, r.tau, want_C=False)
    assert r.stats["kept"] == [int(v) for v in ref.Kt]
    assert np.array_equal(r.keys, ref.keys)
    check_sampled_product(r, seed=3)
    big = torch.zeros(16385, 16385, device="cuda")
    with pytest.raises(gpu.SpammError) as ei:
        gpu.build_tree(big, 16)
    assert ei.value.code == gpu.SPAMM_E_RANGE


def test_largest_order_n65536_leaf64(gpu):
    """The largest order the library takes at n_b = 64: n = 65536 (N = 1024,
    n^2 = 2^32 elements, so every element offset needs 64-bit arithmetic);
    every norm tier and the whole task set bit-exact, C on sampled leaves
    (zero leaves where nothing is kept included)."""
    import torch
    A = workloads.exp_decay(65536, 0.5, 4)
    r = MatrixRun(gpu, A, 64, 1e-6, "expdecay0.5-n65536-leaf64")
    assert r.tree.depth == 10
    check_norms(r)
    ref = oracle.spamm(r.A, r.A, 64, r.tau, want_C=False)
    assert r.stats["kept"] == [int(v) for v in ref.Kt]
    assert np.array_equal(r.keys, ref.keys)
    check_sampled_product(r, seed=4)
    # the last element, written once, equals the oracle's
    Ct, _, _ = oracle.spamm_tiles(r.A, r.A, 64, r.tau, [(1023, 1023)], threads=16,
                                  want_klists=True)
    assert abs(float(r.C[-1, -1]) - Ct[0][-1, -1]) <= 1e-5 * r.tree.norm2
    del r
    torch.cuda.empty_cache()


# ---- split precision at full size -------------------------------------------

def round_leaf(X, S, fmt):
    """A leaf block rounded as a LOW operand: bfloat16, or binary16 at the
    scale exponent of its squared norm S (subnormals flushed)."""
    import torch
    if fmt in ("bf16", "bf16x3"):
        return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(torch.bfloat16).to(
            torch.float64).numpy()
    e = oracle.fp16_exponent(S)
    h = (X * 2.0 ** e).astype(np.float16).astype(np.float64)
    return np.where(np.abs(h) < 2.0 ** -14, 0.0, h) * 2.0 ** -e


def abs_parts(X):
    """|hi| + |lo| of a leaf block's two bfloat16 parts (torch's rounding,
    float32 subtraction)."""
    H = round_leaf(X, 0.0, "bf16")
    L = round_leaf(np.asarray(X, dtype=np.float32) - H.astype(np.float32), 0.0, "bf16")
    return np.abs(H) + np.abs(L)


class SplitRun:
    """A split product with an absolute threshold `low` or a relative one
    `rel` (theta, formed by the library from the tree's root)."""

    def __init__(self, sp, A, leaf, tau, low, fmt, label, rel=0.0):
        import torch
        self.A, self.leaf, self.tau, self.low, self.fmt, self.n = A, leaf, tau, low, fmt, A.shape[0]
        self.rel = rel
        print(f"\n[fullsize] {label} split-{fmt} tau={tau:g} low_tol={low:g} theta={rel:g}",
              flush=True)
        dA = torch.from_numpy(A).cuda()
        self.tree = sp.build_tree(dA, leaf, bf16=(fmt != "fp16"), fp16=(fmt == "fp16"))
        prec = {"fp16": sp.PREC_SPLIT_FP16, "bf16": sp.PREC_SPLIT_BF16,
                "bf16x3": sp.PREC_SPLIT_BF16X3}[fmt]
        self.plan = sp.symbolic(self.tree, self.tree, tau, precision=prec, low_tol=low,
                                low_rel=rel)
        C = torch.full_like(dA, float("nan"))
        self.plan.numeric(C)
        torch.cuda.synchronize()
        del dA
        self.C = C.cpu().numpy()
        del C
        self.keys = self.plan.tasks()
        self.stats = self.plan.stats()
        print(f"[fullsize] K={self.stats['tasks']} LOW={self.stats['tasks_low']}", flush=True)


def check_split(run, seed):
    """Every task key (class bit included) against the oracle's split mode;
    sampled output leaves against the oracle's per-leaf recursion within
    Higham's bound over each class's operands (m = n_b K + 1, one more
    rounding per LOW product with FP16; with compensated HIGH products three
    terms per product, bounded by (|hi_a| + |lo_a|)(|hi_b| + |lo_b|))."""
    ref = oracle.spamm(run.A, run.A, run.leaf, run.tau, want_C=False, low_tol=run.low,
                       low_fmt=run.fmt, low_rel=run.rel)
    assert run.stats["tasks"] == ref.K and run.stats["tasks_low"] == ref.Klow
    assert np.array_equal(run.keys, ref.keys)
    N = 1 << run.tree.depth
    S = oracle.norms(run.A, run.leaf)[-1]
    tiles = choose_tiles(N, seed, count=24)
    Ct, counts, kl = oracle.spamm_tiles(run.A, run.A, run.leaf, run.tau, tiles, threads=16,
                                        want_klists=True, low_tol=run.low, low_fmt=run.fmt,
                                        low_rel=run.rel)
    extra = 1 if run.fmt == "fp16" else 0
    worst = -np.inf
    for s, (I, J) in enumerate(tiles):
        M = np.zeros((run.leaf, run.leaf))
        for v in kl[s, :counts[s]]:
            k, low = int(v) & 0x3FFFFFFF, int(v) >> 30
            X = leaf_block(run.A, I, k, run.leaf, run.n)
            Y = leaf_block(run.A, k, J, run.leaf, run.n)
            if low:
                X, Y = round_leaf(X, S[I, k], run.fmt), round_leaf(Y, S[k, J], run.fmt)
            elif run.fmt == "bf16x3":
                X, Y = abs_parts(X), abs_parts(Y)
            M += np.abs(X) @ np.abs(Y)
        m = (3 * run.leaf if run.fmt == "bf16x3" else run.leaf + extra) * int(counts[s]) + 1
        bound = m * U32 / (1 - m * U32) * M + m * 2.0 ** -126
        got = leaf_block(run.C, I, J, run.leaf, run.n)
        assert np.all(np.isfinite(got))
        worst = max(worst, float(np.max(np.abs(got - Ct[s]) - bound)))
    assert worst <= 0.0, f"rounding bound exceeded by {worst}"


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_algdecay_split_theta_1e4(gpu, fmt):
    """algdecay-n16384 at tau = 1e-8 with LOW iff ||A_ik|| ||A_kj|| < 1e-4 ||A||_F^2
    (theta = 1e-4, the bound formed by the library)."""
    wl = workloads.WORKLOADS["algdecay-n16384"]
    A = wl.matrix()
    r = SplitRun(gpu, A, wl.leaf, 1e-8, 0.0, fmt, wl.name, rel=1e-4)
    assert 0 < r.stats["tasks_low"] < r.stats["tasks"]
    check_split(r, seed=21)


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "bf16x3"])
def test_largest_grid_split_n32768_leaf32(gpu, fmt):
    """Split precision (BF16 or FP16 LOW operands, FP32 or compensated HIGH
    products) at the largest grid of n_b = 32 (n = 32768, N = 1024 leaves
    per dimension, 10 tiers below the root; the 2 x 2 block kernels) with
    theta = 1e-4: every key with its class bit against the oracle's, sampled
    C within the bound."""
    import torch
    A = workloads.exp_decay(32768, 0.5, 5)
    r = SplitRun(gpu, A, 32, 1e-6, 0.0, fmt, "expdecay0.5-n32768-leaf32", rel=1e-4)
    assert r.tree.depth == 10
    assert 0 < r.stats["tasks_low"] < r.stats["tasks"]
    check_split(r, seed=23)
    del r
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "bf16x3"])
def test_largest_order_split_n65536_leaf64(gpu, fmt):
    """Split precision at the largest order of n_b = 64 (n = 65536, N =
    1024, 2^32 elements; the 4 x 4 block kernels with BF16 LOW operands, the
    2 x 2 one with FP16) with theta = 1e-4: every key with its class bit
    against the oracle's, sampled C within the bound."""
    import torch
    A = workloads.exp_decay(65536, 0.5, 6)
    r = SplitRun(gpu, A, 64, 1e-6, 0.0, fmt, "expdecay0.5-n65536-leaf64", rel=1e-4)
    assert r.tree.depth == 10
    assert 0 < r.stats["tasks_low"] < r.stats["tasks"]
    check_split(r, seed=24)
    del r
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tau", [1e-4, 1e-6, 1e-10])
def test_algdecay_split_tau_sweep_theta_1e4(gpu, tau):
    """The rest of the algdecay-n16384 tau sweep with BF16 LOW operands at
    theta = 1e-4: every key with its class bit, sampled C within the bound."""
    wl = workloads.WORKLOADS["algdecay-n16384"]
    r = SplitRun(gpu, wl.matrix(), wl.leaf, tau, 0.0, "bf16", wl.name, rel=1e-4)
    assert 0 < r.stats["tasks_low"] < r.stats["tasks"]
    check_split(r, seed=22)


def test_cluster1310_split_theta_1e4(cluster1310, gpu):
    """cluster1310-n32750 at tau = 1e-8 with LOW iff the norm product is below
    1e-4 ||A||_F^2 (nearly every product LOW): all keys with class bits."""
    r = SplitRun(gpu, cluster1310.A, cluster1310.leaf, 1e-8, 0.0, "bf16", "cluster1310-n32750",
                 rel=1e-4)
    assert r.stats["tasks_low"] > 0.9 * r.stats["tasks"]
    check_split(r, seed=33)


@pytest.mark.parametrize("fmt,tau,theta", [("bf16", 3.1622776601683795e-05, 1e-6),
                                           ("fp16", 1e-4, 1e-5), ("bf16x3", 1e-4, 3e-7)])
def test_cluster1310_split_matched_error_point(cluster1310, gpu, fmt, tau, theta):
    """cluster1310-n32750 at the split products' matched-error points of the
    benchmark (the fastest split product within the FP32 product's
    whole-matrix error)."""
    r = SplitRun(gpu, cluster1310.A, cluster1310.leaf, tau, 0.0, fmt, "cluster1310-n32750",
                 rel=theta)
    assert r.stats["tasks_low"] > 0.9 * r.stats["tasks"]
    check_split(r, seed=31)


# ---- the longest entry list a block can hold ------------------------------------

def test_longest_entry_list_leaf32_fp32(gpu):
    """n = 32768 at 32 x 32 leaves (N = 1024): with only the first 128 rows
    and columns non-zero, output leaf (0, 0) takes all 1024 values of k, as
    many entries as a block's list holds; the whole task set bit-exact, C on
    sampled leaves (the long one included) within the bound."""
    from inputs import arrow
    A = arrow(32768, 128, 21)
    r = MatrixRun(gpu, A, 32, 1e-7, "arrow-n32768-leaf32")
    ref = oracle.spamm(A, A, 32, 1e-7, want_C=False)
    assert r.stats["kept"] == [int(v) for v in ref.Kt]
    assert np.array_equal(r.keys, ref.keys)
    hi = r.keys >> np.uint64(32)
    assert int(np.count_nonzero(hi == np.uint64(oracle.linear_index(0, 0)))) == 1024
    check_sampled_product(r, seed=6)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_longest_entry_list_leaf32_split(gpu, fmt):
    """The same matrix with split precision (57 % of the products LOW): both
    schedules of the long block, every key with its class bit, sampled C
    within the class-aware bound."""
    from inputs import arrow
    A = arrow(32768, 128, 21)
    r = SplitRun(gpu, A, 32, 1e-7, 1e-2, fmt, "arrow-n32768-leaf32")
    assert 0.5 * r.stats["tasks"] < r.stats["tasks_low"] < 0.7 * r.stats["tasks"]
    check_split(r, seed=8)
