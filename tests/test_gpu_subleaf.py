"""Sub-leaf culling on the GPU against the oracle run with 32 x 32 leaves.

A leaf-64 tree built with sub-block norms carries the norm pyramid of a
leaf-32 tree; inside each kept 64 x 64 leaf product the GEMM tests the 8
products of 32 x 32 sub-blocks.  Checked:

* every norm tier (0..d+1) bit-exact against the oracle's leaf-32 norms;
* the packed leaves equal those of a plain leaf-64 tree;
* kept counts of tiers 0..d equal the leaf-32 oracle's;
* the performed sub-products, as keys on the 32 x 32 grid, bit-exact against
  the leaf-32 oracle's task keys, and their count;
* C within Higham's bound around the leaf-32 oracle's product
  (m = 32 K_ij + 1 per 32 x 32 output block);
* argument errors.
"""
import numpy as np
import pytest

import oracle
import workloads
from inputs import arrow

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def decay(n, rate, seed, sym=True):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return A.astype(np.float32)


CASES = {
    # name: (A, B or None, tau)
    "expdecay-n1024": lambda: (workloads.exp_decay(1024, 0.1, 0), None, 1e-6),
    "ragged-n700": lambda: (decay(700, 0.03, 1), None, 1e-5),
    "nonsym-n500": lambda: (decay(500, 0.05, 2, sym=False), decay(500, 0.04, 3, sym=False), 1e-4),
    "algdecay-n1500": lambda: (workloads.alg_decay(1500, 3.0, 0), None, 1e-8),
    "tau0-n300": lambda: (decay(300, 0.2, 4), None, 0.0),
    "single-n50": lambda: (decay(50, 0.1, 5), None, 1e-3),
    "n64": lambda: (decay(64, 0.3, 6), None, 1e-3),
    "coarse-n900": lambda: (decay(900, 0.02, 7), None, 1e-2),
}


def higham_bound(A, B, keys, n):
    """gamma_m sum_kept |A_ik||B_kj| + m 2^-126 over 32 x 32 blocks."""
    d, np_ = oracle.depth(n, 32)
    PA = np.zeros((np_, np_))
    PB = np.zeros((np_, np_))
    PA[:n, :n] = np.abs(A)
    PB[:n, :n] = np.abs(B)
    N = 1 << d
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    M = np.zeros((np_, np_))
    cnt = np.zeros((N, N), dtype=np.int64)
    for key in keys:
        key = int(key)
        I, J = inv[key >> 32]
        k = key & 0xFFFFFFFF
        M[I * 32:(I + 1) * 32, J * 32:(J + 1) * 32] += \
            PA[I * 32:(I + 1) * 32, k * 32:(k + 1) * 32] @ PB[k * 32:(k + 1) * 32, J * 32:(J + 1) * 32]
        cnt[I, J] += 1
    m = 32 * np.kron(cnt, np.ones((32, 32))) + 1
    gamma = m * U32 / (1 - m * U32)
    return (gamma * M + m * 2.0 ** -126)[:n, :n]


@pytest.fixture(scope="module")
def runs(gpu):
    import torch
    cache = {}

    def get(name):
        if name not in cache:
            A, B, tau = CASES[name]()
            Bm = A if B is None else B
            ref = oracle.spamm(A, Bm, 32, tau)
            dA = torch.from_numpy(A).cuda()
            tA = gpu.build_tree(dA, 64, subnorms=True)
            tB = tA if B is None else gpu.build_tree(torch.from_numpy(B).cuda(), 64, subnorms=True)
            plan = gpu.symbolic(tA, tB, tau, sub_cull=True)
            C = torch.full_like(dA, float("nan"))
            plan.numeric(C)
            torch.cuda.synchronize()
            cache[name] = dict(A=A, B=Bm, tau=tau, ref=ref, tA=tA, tB=tB, plan=plan,
                               C=C.cpu().numpy(), dA=dA)
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_subnorm_pyramid_is_leaf32_pyramid(runs, name):
    r = runs(name)
    want = oracle.norms(r["A"], 32)
    t = r["tA"]
    n = r["A"].shape[0]
    if n <= 32:
        # the leaf-32 tree is one leaf; the leaf-64 tree pads to 64, so its
        # sub-block tier is [[s, 0], [0, 0]]
        assert t.norms(0)[0, 0] == want[0][0, 0]
        assert np.array_equal(t.norms(1), np.array([[want[0][0, 0], 0.0], [0.0, 0.0]]))
        return
    assert len(want) == t.depth + 2
    for tier in range(t.depth + 2):
        assert np.array_equal(t.norms(tier), want[tier]), tier
    assert t.norm2 == want[0][0, 0]


@pytest.mark.parametrize("name", ["expdecay-n1024", "ragged-n700"])
def test_subnorm_tree_packs_like_plain_tree(gpu, runs, name):
    r = runs(name)
    plain = gpu.build_tree(r["dA"], 64)
    for copy in (0, 1):
        assert np.array_equal(r["tA"].matrix(copy), plain.matrix(copy))


@pytest.mark.parametrize("name", list(CASES))
def test_performed_subproducts_equal_leaf32_tasks(runs, name):
    r = runs(name)
    sub = r["plan"].subtasks()
    assert np.array_equal(sub, r["ref"].keys)
    st = r["plan"].stats()
    assert st["subtasks"] == r["ref"].K
    assert st["flops"] == 2.0 * 32 ** 3 * r["ref"].K
    d = st["depth"]
    if r["A"].shape[0] > 32:
        assert st["kept"][:d + 1] == [int(v) for v in r["ref"].Kt[:d + 1]]
        if name not in ("tau0-n300", "single-n50", "n64"):
            assert st["subtasks"] < 8 * st["tasks"]     # sub-blocks were culled


@pytest.mark.parametrize("name", list(CASES))
def test_subleaf_product_within_bound(runs, name):
    r = runs(name)
    assert np.all(np.isfinite(r["C"]))
    n = r["A"].shape[0]
    err = np.abs(r["C"].astype(np.float64) - r["ref"].C)
    worst = float(np.max(err - higham_bound(r["A"], r["B"], r["ref"].keys, n)))
    assert worst <= 0.0, f"bound exceeded by {worst}"


def test_subleaf_repeat_is_bit_identical(runs):
    import torch
    r = runs("algdecay-n1500")
    C2 = torch.empty_like(r["dA"])
    r["plan"].numeric(C2)
    assert np.array_equal(C2.cpu().numpy(), r["C"])
    assert r["plan"].stats()["subtasks"] == r["ref"].K   # counter restarts per pass


def test_subleaf_full_size_cluster(gpu):
    """cluster300-n7500 squared with leaf-64 storage and 32 x 32 sub-leaf
    culling: the performed sub-products against the oracle's leaf-32 task set."""
    import torch
    wl = workloads.WORKLOADS["cluster300-n7500"]
    A = wl.matrix()
    print(f"\n[subleaf] {wl.name} tau={wl.tau:g}", flush=True)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 64, subnorms=True)
    C = torch.empty_like(dA)
    plan = gpu.symbolic(t, t, wl.tau, sub_cull=True)
    plan.numeric(C)
    sub = plan.subtasks()
    ref = oracle.spamm(A, A, 32, wl.tau, want_C=False)
    assert sub.size == ref.K
    assert np.array_equal(sub, ref.keys)


def check_subleaf_large(gpu, A, tau, label, seed, count=24):
    """A leaf-64 sub-culled square of a large A: kept counts of tiers 0..d
    and the performed sub-products against the leaf-32 oracle's, sampled
    32 x 32 output blocks within Higham's bound around the oracle's."""
    import torch
    n = A.shape[0]
    print(f"\n[subleaf] {label} tau={tau:g}", flush=True)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 64, subnorms=True)
    plan = gpu.symbolic(t, t, tau, sub_cull=True)
    C = torch.full_like(dA, float("nan"))
    plan.numeric(C)
    torch.cuda.synchronize()
    del dA
    Ch = C.cpu().numpy()
    del C
    st = plan.stats()
    sub = plan.subtasks()
    print(f"[subleaf] {label}: leaf products {st['tasks']}, sub-products {st['subtasks']}",
          flush=True)
    ref = oracle.spamm(A, A, 32, tau, want_C=False)
    d = st["depth"]
    assert st["kept"][:d + 1] == [int(v) for v in ref.Kt[:d + 1]]
    assert sub.size == ref.K and st["subtasks"] == ref.K
    assert np.array_equal(sub, ref.keys)
    assert ref.K < 8 * st["tasks"]                      # sub-blocks were culled
    N = 1 << (d + 1)
    rng = np.random.default_rng(seed)
    tiles = [(int(f) // N, int(f) % N) for f in np.sort(rng.choice(N * N, count, replace=False))]
    # the band, where the products are, besides random blocks
    band = rng.choice(N - 1, 8, replace=False)
    tiles += [(0, 0), (N - 1, N - 1)] + [(int(i), int(i)) for i in band[:4]] + \
        [(int(i), int(i) + 1) for i in band[4:]]
    Ct, counts, kl = oracle.spamm_tiles(A, A, 32, tau, tiles, threads=16, want_klists=True)
    assert (counts > 0).sum() >= 10
    worst = -np.inf
    for s_, (I, J) in enumerate(tiles):
        M = np.zeros((32, 32))
        for v in kl[s_, :counts[s_]]:
            k = int(v) & 0x3FFFFFFF
            M += np.abs(A[I * 32:(I + 1) * 32, k * 32:(k + 1) * 32].astype(np.float64)) @ \
                np.abs(A[k * 32:(k + 1) * 32, J * 32:(J + 1) * 32].astype(np.float64))
        m = 32 * int(counts[s_]) + 1
        bound = m * U32 / (1 - m * U32) * M + m * 2.0 ** -126
        got = Ch[I * 32:(I + 1) * 32, J * 32:(J + 1) * 32]
        assert np.all(np.isfinite(got))
        worst = max(worst, float(np.max(np.abs(got - Ct[s_]) - bound)))
    assert worst <= 0.0, f"bound exceeded by {worst}"


def test_subleaf_largest_order_n65536(gpu):
    """The largest order of leaf-64 trees (n = 65536, N = 1024, tiers 0..10
    plus the sub-block tier: a 2048 x 2048 grid of 32 x 32 sub-blocks)."""
    import torch
    check_subleaf_large(gpu, workloads.exp_decay(65536, 0.5, 7), 1e-6,
                        "expdecay0.5-n65536", seed=31)
    torch.cuda.empty_cache()


def test_subleaf_argument_errors(gpu):
    import torch
    A = torch.from_numpy(decay(200, 0.05, 1)).cuda()
    with pytest.raises(gpu.SpammError) as ei:
        gpu.build_tree(A, 32, subnorms=True)
    assert ei.value.code == gpu.SPAMM_E_INVAL
    plain = gpu.build_tree(A, 64)
    with pytest.raises(gpu.SpammError) as ei:
        gpu.symbolic(plain, plain, 1e-6, sub_cull=True)
    assert ei.value.code == gpu.SPAMM_E_INVAL
    both = gpu.build_tree(A, 64, subnorms=True, bf16=True)
    with pytest.raises(gpu.SpammError) as ei:
        gpu.symbolic(both, both, 1e-6, precision=gpu.PREC_SPLIT_BF16, low_tol=1e-3, sub_cull=True)
    assert ei.value.code == gpu.SPAMM_E_INVAL
    p = gpu.symbolic(plain, plain, 1e-6)
    with pytest.raises(gpu.SpammError) as ei:
        p.subtasks()
    assert ei.value.code == gpu.SPAMM_E_INVAL
    # a sub-norm tree also serves whole-leaf products
    C1, C2 = torch.empty_like(A), torch.empty_like(A)
    s = gpu.build_tree(A, 64, subnorms=True)
    gpu.multiply_ex(s, s, 0.0, C1)
    gpu.multiply_ex(plain, plain, 0.0, C2)
    assert torch.equal(C1, C2)


def test_subleaf_block_with_the_longest_entry_list(gpu):
    """n = 32768: the output block of leaves (0, 0)-(1, 1) takes all 512
    values of k, the longest entry list a block holds at this order (every
    other block takes two), so the masks and stage list of every thread of
    the workgroup are used.  Performed sub-products bit-exact against the
    leaf-32 oracle; C on the long block and on sampled blocks against the
    oracle's per-leaf products within Higham's bound."""
    import torch
    n, tau = 32768, 1e-7
    A = arrow(n, 128, 21)
    print("\n[subleaf] arrow-n32768", flush=True)
    dA = torch.from_numpy(A).cuda()
    t = gpu.build_tree(dA, 64, subnorms=True)
    plan = gpu.symbolic(t, t, tau, sub_cull=True)
    C = torch.full_like(dA, float("nan"))
    plan.numeric(C)
    torch.cuda.synchronize()
    del dA
    sub = plan.subtasks()
    st = plan.stats()
    ref = oracle.spamm(A, A, 32, tau, want_C=False)
    assert sub.size == ref.K
    assert np.array_equal(sub, ref.keys)
    # the long block really is long, and sub-culling acts inside it
    hi = ref.keys >> np.uint64(32)
    lc = np.uint64(oracle.linear_index(0, 0))
    k00 = (ref.keys[hi == lc] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert len(np.unique(k00 // 2)) == 512           # every leaf-64 k for output leaf (0, 0)
    assert st["subtasks"] < 0.6 * 8 * st["tasks"]     # and about half the sub-products culled
    tiles = [(0, 0), (0, 1), (1, 0), (1, 1), (3, 3), (0, 1023), (1023, 0), (500, 700), (1023, 1023)]
    Ct, counts, kl = oracle.spamm_tiles(A, A, 32, tau, tiles, threads=16, want_klists=True)
    Cg = C.cpu().numpy()
    for s, (I, J) in enumerate(tiles):
        got = Cg[I * 32:(I + 1) * 32, J * 32:(J + 1) * 32].astype(np.float64)
        want = Ct[s]
        ks = kl[s, :counts[s]]
        M = np.zeros((32, 32))
        for k in ks:
            M += np.abs(A[I * 32:(I + 1) * 32, k * 32:(k + 1) * 32]).astype(np.float64) @ \
                np.abs(A[k * 32:(k + 1) * 32, J * 32:(J + 1) * 32]).astype(np.float64)
        m = 32 * len(ks) + 1
        bound = m * U32 / (1 - m * U32) * M + m * 2.0 ** -126
        assert np.all(np.abs(got - want) <= bound), (I, J)
