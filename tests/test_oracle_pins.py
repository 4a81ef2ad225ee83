"""Pins for the FP64 oracle against facts that do not come from the oracle.

Each test ties one part of the oracle to the paper or to mathematics that a
plausible mistake would violate:

* depth / padding (Sec. II.A) -- the real-valued ceil(log2(n/n_b)) formula;
* linear index (Eq. linear index) -- the convolution masks of Eq. convolution,
  the k-masks of the k-value sort and the "two digits per tier" structure;
* leaf and tier norms (Eq. norm) -- correctly rounded sums (math.fsum) within
  the pairwise-summation error bound, exact special cases;
* product (Eq. product) -- numpy's FP64 matrix product at tau = 0;
* task set (Eq. norm condition) -- brute-force enumeration of the flat leaf
  test (equal to the hierarchical one by monotonicity of the stored norms);
* truncation -- the per-tile bound sum_{skipped} ||A_ik||_F ||B_kj||_F.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

U = 2.0 ** -53  # unit roundoff, FP64


def lidx_table(m):
    return np.array([[oracle.linear_index(i, j) for j in range(m)] for i in range(m)],
                    dtype=np.uint64)


def rand_decay(n, rate, seed, sym=False):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    env = np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    A = rng.uniform(-1, 1, size=(n, n)) * env
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return A.astype(np.float32)


def padded(A, b):
    n = A.shape[0]
    d, np_ = oracle.depth(n, b)
    P = np.zeros((np_, np_), dtype=np.float64)
    P[:n, :n] = A
    return P, d


def flat_taskset(sA, sB, tau, L):
    """Brute force: all leaf triples passing the test on the stored norms."""
    T2 = tau * tau
    N = sA.shape[0]
    keys = []
    for I in range(N):
        for K in range(N):
            a = sA[I, K]
            if a == 0.0:
                continue
            for J in range(N):
                bb = sB[K, J]
                if bb != 0.0 and a * bb >= T2:
                    keys.append((int(L[I, J]) << 32) | K)
    return np.array(sorted(keys), dtype=np.uint64)


# --------------------------------------------------------------------------
# Sec. II.A: depth and padding
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,b,d,np_", [
    (1024, 32, 5, 1024),      # n=1024, leaf 32: depth 5
    (7500, 32, 8, 8192),      # 7500 padded to 8192
    (16384, 64, 8, 16384),
    (32750, 64, 9, 32768),    # 32750 padded to 32768
    (32, 32, 0, 32), (1, 16, 0, 16), (33, 32, 1, 64), (513, 16, 6, 1024),
])
def test_depth_closed_forms(n, b, d, np_):
    assert oracle.depth(n, b) == (d, np_)


def test_depth_matches_real_log_formula():
    for b in (16, 32, 64):
        for n in range(1, 6000, 7):
            d, np_ = oracle.depth(n, b)
            want = max(0, math.ceil(math.log2(n / b)))
            assert d == want, (n, b)
            assert np_ == b << d and np_ >= n and (d == 0 or np_ // 2 < n)


# --------------------------------------------------------------------------
# Eq. linear index vs Eq. convolution and the k-value masks
# --------------------------------------------------------------------------
def test_linear_index_convolution_and_masks():
    m = 64
    L = lidx_table(m)
    EVEN = np.uint64(0x5555555555555555)   # ...010101: column (k of A) bits
    ODD = np.uint64(0xAAAAAAAAAAAAAAAA)    # ...101010: row bits
    # bijection onto [0, m^2)
    assert np.array_equal(np.sort(L.ravel()), np.arange(m * m, dtype=np.uint64))
    # l_C = (l_A & ...101010) | (l_B & ...010101), exhaustively over i, k, j
    i = np.arange(m)[:, None, None]
    k = np.arange(m)[None, :, None]
    j = np.arange(m)[None, None, :]
    lA = L[i, k]
    lB = L[k, j]
    conv = (lA & ODD) | (lB & EVEN)
    assert np.array_equal(np.broadcast_to(L[i, j], conv.shape), conv)
    # k extracted from A's index with ...0101 and from B's with ...1010
    assert np.array_equal(L[:, :] & EVEN, np.broadcast_to(L[0:1, :], (m, m)))
    assert np.array_equal(L[:, :] & ODD, np.broadcast_to(L[:, 0:1], (m, m)))
    # each tier appends two digits on the right: row digit, then column digit
    h = m // 2
    for a in (0, 1):
        for c in (0, 1):
            child = L[a::2, c::2][:h, :h]
            assert np.array_equal(child, 4 * L[:h, :h] + np.uint64(2 * a + c))
    assert (L[0, 0], L[0, 1], L[1, 0], L[1, 1]) == (0, 1, 2, 3)


# --------------------------------------------------------------------------
# Eq. norm: leaf and tier squared norms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,b", [(96, 16), (100, 32), (256, 64)])
def test_leaf_norms_within_pairwise_bound(n, b):
    rng = np.random.default_rng(n + b)
    A = (rng.standard_normal((n, n)) * 10.0 ** rng.uniform(-20, 5, size=(n, n))).astype(np.float32)
    tiers = oracle.norms(A, b)
    P, d = padded(A, b)
    N = 1 << d
    leaf = tiers[d]
    bound = math.ceil(math.log2(b * b)) * U
    for I in range(N):
        for J in range(N):
            t = P[I * b:(I + 1) * b, J * b:(J + 1) * b]
            exact = math.fsum((t * t).ravel())
            assert abs(leaf[I, J] - exact) <= bound * exact * (1 + 1e-12)
    total = math.fsum((P * P).ravel())
    root_bound = (math.ceil(math.log2(b * b)) + 2 * d) * U
    assert abs(tiers[0][0, 0] - total) <= root_bound * total * (1 + 1e-12)


def test_tier_sums_are_child_quadrant_sums():
    A = rand_decay(200, 0.05, 3)
    tiers = oracle.norms(A, 16)
    for t in range(len(tiers) - 1):
        ch = tiers[t + 1]
        want = (ch[0::2, 0::2] + ch[0::2, 1::2]) + (ch[1::2, 0::2] + ch[1::2, 1::2])
        assert np.array_equal(tiers[t], want)
        # squared norms of parents dominate every child (monotone rounding)
        for a in (0, 1):
            for c in (0, 1):
                assert np.all(tiers[t] >= ch[a::2, c::2])


def test_norm_special_cases():
    n, b = 64, 16
    A = np.zeros((n, n), dtype=np.float32)
    A[3, 5] = 0.75                                  # single element: exactly x^2
    A[20:36, 40:56] = np.float32(2.0 ** -140)       # FP32 denormals only
    A[17, 17] = np.float32(1.0e-45)                 # smallest denormal
    leaf = oracle.norms(A, b)[2]
    assert leaf[0, 0] == 0.75 ** 2
    assert leaf[3, 3] == 0.0                        # an all-zero tile
    den = np.float64(np.float32(2.0 ** -140)) ** 2
    # tile (1,2) holds rows 16..31, cols 32..47 -> rows 20..31, cols 40..47: 12*8
    assert leaf[1, 2] == 96 * den
    assert leaf[1, 1] == np.float64(np.float32(1.0e-45)) ** 2 > 0.0


def test_norms_of_padded_matrix():
    A = rand_decay(37, 0.2, 5)       # 37 -> padded to 64 at b=16, d=2
    tiers = oracle.norms(A, 16)
    assert len(tiers) == 3
    leaf = tiers[2]
    assert leaf[3, 3] == 0.0 and leaf[3, 0] == 0.0 and leaf[0, 3] == 0.0
    assert leaf[2, 2] == pytest.approx(float(np.sum(A[32:, 32:].astype(np.float64) ** 2)),
                                       rel=1e-14)


# --------------------------------------------------------------------------
# Eq. product at tau = 0 is the dense product
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,b", [(200, 16), (96, 32), (130, 64), (20, 32)])
def test_tau0_is_dense_product(n, b):
    rng = np.random.default_rng(n)
    A = rng.uniform(-1, 1, (n, n)).astype(np.float32)   # not symmetric
    B = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    A[:, n // 3] = 0.0                                 # some zero tiles / columns
    r = oracle.spamm(A, B, b, 0.0)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    scale = np.linalg.norm(A.astype(np.float64)) * np.linalg.norm(B.astype(np.float64))
    assert np.abs(r.C - ref).max() <= 1e-12 * scale
    # at tau = 0 exactly the pairs with both tile norms non-zero are kept
    sA = oracle.norms(A, b)[-1]
    sB = oracle.norms(B, b)[-1]
    want = int(np.sum((sA > 0).astype(np.int64) @ (sB > 0).astype(np.int64)))
    assert r.K == want


def test_transposed_operand_is_detected():
    """A @ B and B @ A differ for these inputs, so the tau=0 pin above would
    catch an oracle that swapped or transposed an operand."""
    rng = np.random.default_rng(1)
    A = rng.uniform(-1, 1, (64, 64)).astype(np.float32)
    B = rng.uniform(-1, 1, (64, 64)).astype(np.float32)
    r = oracle.spamm(A, B, 16, 0.0)
    assert np.abs(r.C - B.astype(np.float64) @ A.astype(np.float64)).max() > 1.0
    assert np.abs(r.C - (A.astype(np.float64) @ B.astype(np.float64)).T).max() > 1.0


# --------------------------------------------------------------------------
# Eq. norm condition: task set == brute force, at every tier
# --------------------------------------------------------------------------
CASES = [
    ("decay", 256, 16, 1e-3), ("decay", 256, 16, 1e-6), ("decay", 300, 32, 1e-4),
    ("decay", 512, 32, 1e-8), ("zeros", 200, 16, 0.0), ("zeros", 200, 16, 1e-5),
    ("denorm", 128, 16, 1e-40), ("denorm", 128, 16, 0.0), ("nonsym", 192, 16, 1e-4),
]


def make_case(kind, n, seed=0):
    if kind == "decay":
        return rand_decay(n, 0.08, seed, sym=True), None
    if kind == "zeros":
        A = rand_decay(n, 0.05, seed, sym=True)
        A[16:48, :] = 0.0
        A[:, 16:48] = 0.0
        A[100:130, 150:190] = 0.0
        return A, None
    if kind == "denorm":
        A = rand_decay(n, 0.6, seed, sym=True)   # far tiles are FP32 denormals or 0
        return A, None
    if kind == "nonsym":
        return rand_decay(n, 0.05, seed), rand_decay(n, 0.1, seed + 1)
    raise ValueError(kind)


@pytest.mark.parametrize("kind,n,b,tau", CASES)
def test_taskset_equals_bruteforce(kind, n, b, tau):
    A, B = make_case(kind, n)
    B = A if B is None else B
    r = oracle.spamm(A, B, b, tau, want_C=False)
    tA, tB = oracle.norms(A, b), oracle.norms(B, b)
    d = len(tA) - 1
    L = lidx_table(1 << d)
    assert np.array_equal(r.keys, flat_taskset(tA[d], tB[d], tau, L))
    # tier counts equal the flat test at every tier (monotonicity)
    for t in range(d + 1):
        sa, sb = tA[t], tB[t]
        nz = ((sa[:, :, None] > 0) & (sb[None, :, :] > 0)
              & (sa[:, :, None] * sb[None, :, :] >= tau * tau))
        assert r.Kt[t] == int(nz.sum()), t


@pytest.mark.parametrize("tau", [1e-3, 1e-6])
def test_taskset_with_independent_norms(tau):
    """Norms recomputed by numpy (another summation order); triples within a
    relative 1e-9 of the threshold are excluded, the rest must agree."""
    A = rand_decay(384, 0.07, 11, sym=True)
    b = 32
    r = oracle.spamm(A, A, b, tau, want_C=False)
    P, d = padded(A, b)
    N = 1 << d
    s = (P * P).reshape(N, b, N, b).sum(axis=(1, 3))
    L = lidx_table(N)
    got = set(int(k) for k in r.keys)
    prod = s[:, :, None] * s[None, :, :]
    T2 = tau * tau
    for I in range(N):
        for K in range(N):
            for J in range(N):
                p = prod[I, K, J]
                if abs(p - T2) <= 1e-9 * T2:
                    continue
                key = (int(L[I, J]) << 32) | K
                assert (key in got) == (p >= T2 and s[I, K] > 0 and s[K, J] > 0)


def test_symmetric_square_gives_symmetric_taskset():
    A = workloads.exp_decay(512, 0.1, seed=0)
    b = 32
    r = oracle.spamm(A, A, b, 1e-6, want_C=False)
    d = oracle.depth(512, b)[0]
    L = lidx_table(1 << d)
    inv = {int(L[i, j]): (i, j) for i in range(1 << d) for j in range(1 << d)}
    triples = set()
    for key in r.keys:
        I, J = inv[int(key) >> 32]
        triples.add((I, int(key) & 0xFFFFFFFF, J))
    assert triples == {(J, K, I) for (I, K, J) in triples}


def test_ties_keep_and_drop():
    """Power-of-two tile norms make s_A * s_B == tau^2 exactly: kept (the
    paper drops only when the product is below tau)."""
    n, b = 64, 16
    A = np.zeros((n, n), dtype=np.float32)
    for I in range(4):
        A[I * 16, I * 16] = 1.0                 # diagonal tiles: norm 1
    A[0, 16] = 2.0 ** -10                        # tile (0,1): squared norm 2^-20
    A[16, 0] = 2.0 ** -10                        # tile (1,0)
    tau = 2.0 ** -10                             # tau^2 = 2^-20 = 1 * 2^-20
    r = oracle.spamm(A, A, b, tau, want_C=False)
    L = lidx_table(4)
    keys = set(int(k) for k in r.keys)
    assert ((int(L[0, 1]) << 32) | 0) in keys    # A00 * A01: 1 * 2^-20 == tau^2
    assert ((int(L[0, 0]) << 32) | 1) not in keys  # A01 * A10: 2^-40 < tau^2
    r2 = oracle.spamm(A, A, b, math.nextafter(tau, 1.0), want_C=False)
    keys2 = set(int(k) for k in r2.keys)
    assert ((int(L[0, 1]) << 32) | 0) not in keys2
    assert ((int(L[0, 0]) << 32) | 0) in keys2


# --------------------------------------------------------------------------
# Truncation bound and the per-tile recursion
# --------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [1e-2, 1e-4, 1e-6])
def test_truncation_bound_per_tile(tau):
    A = rand_decay(256, 0.06, 7, sym=True)
    b = 32
    r = oracle.spamm(A, A, b, tau)
    P, d = padded(A, b)
    N = 1 << d
    nrm = np.sqrt((P * P).reshape(N, b, N, b).sum(axis=(1, 3)))
    exact = P @ P
    L = lidx_table(N)
    inv = {int(L[i, j]): (i, j) for i in range(N) for j in range(N)}
    kept = {}
    for key in r.keys:
        kept.setdefault(inv[int(key) >> 32], set()).add(int(key) & 0xFFFFFFFF)
    Cp = np.zeros_like(P)
    Cp[:256, :256] = r.C
    for I in range(N):
        for J in range(N):
            ks = kept.get((I, J), set())
            bound = sum(nrm[I, k] * nrm[k, J] for k in range(N) if k not in ks)
            err = np.linalg.norm(exact[I * b:(I + 1) * b, J * b:(J + 1) * b]
                                 - Cp[I * b:(I + 1) * b, J * b:(J + 1) * b])
            assert err <= bound + 1e-12 * (1 + nrm[I].dot(nrm[:, J]))


def test_tile_recursion_matches_full():
    A = rand_decay(300, 0.05, 2, sym=True)
    B = rand_decay(300, 0.09, 4)
    b, tau = 32, 1e-4
    full = oracle.spamm(A, B, b, tau)
    d = oracle.depth(300, b)[0]
    N = 1 << d
    tiles = [(I, J) for I in range(N) for J in range(N)]
    Ct, counts, kl = oracle.spamm_tiles(A, B, b, tau, tiles, threads=4, want_klists=True)
    assert counts.sum() == full.K
    Cp = np.zeros((N * b, N * b))
    Cp[:300, :300] = full.C
    keys = []
    for s, (I, J) in enumerate(tiles):
        assert np.array_equal(Ct[s], Cp[I * b:(I + 1) * b, J * b:(J + 1) * b])
        ks = kl[s, :counts[s]]
        assert np.all(np.diff(ks) > 0)
        keys += [(oracle.linear_index(I, J) << 32) | int(k) for k in ks]
    assert np.array_equal(np.array(sorted(keys), dtype=np.uint64), full.keys)


def test_invalid_inputs_rejected():
    A = np.zeros((8, 8), dtype=np.float32)
    with pytest.raises(RuntimeError):
        oracle.spamm(A, A, 12, 0.0)           # leaf not a power of two
    with pytest.raises(RuntimeError):
        oracle.spamm(A, A, 16, -1.0)
    with pytest.raises(RuntimeError):
        oracle.spamm(A, A, 16, float("nan"))


# --------------------------------------------------------------------------
# Eq. norm: the summation ORDER of the FP64 squared norms (the reading that
# fixes it: leaf = pairwise sum over the leaf's row-major flattened index,
# parent = (s11 + s12) + (s21 + s22)).  The bound checks above hold for any
# order; these cases are built so that only that order gives the stated bits.
# --------------------------------------------------------------------------
E27 = np.float32(2.0 ** -27)   # its square 2^-54 is a quarter of ulp(1) = 2^-52


def order_leaf():
    """A 16 x 16 leaf: x = 1 at (0, 0) and x = 2^-27 at (1, 0..3).

    Squares: 1 and four times 2^-54.  Row-major flattened index e = 16 r + c:
    the 1 sits at e = 0, the small squares at e = 16..19.

    * pairwise over the row-major index: the block [0, 16) sums to 1, the
      block [16, 32) to exactly 4 * 2^-54 = 2^-52, and 1 + 2^-52 is exact,
      so s = 1 + 2^-52;
    * pairwise over the column-major index (e' = 16 c + r): the small
      squares sit at e' = 1, 17, 33, 49.  [0, 2) gives 1 + 2^-54 -> 1 (below
      half an ulp), [16, 32) gives 2^-54 and 1 + 2^-54 -> 1, [32, 64) gives
      2^-53 and 1 + 2^-53 is a tie that rounds to the even 1: s = 1;
    * sequential from e = 0: each 1 + 2^-54 rounds back to 1: s = 1;
    * numpy's sum of the same 256 values (eight strided partial sums per
      block of 128): the partial holding the 1 absorbs e = 16, the partials
      of e = 17, 18, 19 meet it as 2^-54 + 2^-53 pieces: s = 1.
    """
    A = np.zeros((16, 16), dtype=np.float32)
    A[0, 0] = 1.0
    A[1, 0:4] = E27
    return A


def test_leaf_norm_order_is_rowmajor_pairwise():
    A = order_leaf()
    want = 1.0 + 2.0 ** -52
    assert oracle.norms(A, 16)[0][0, 0] == want
    sq = (A.astype(np.float64) ** 2)

    def pairwise(v):
        if len(v) == 1:
            return v[0]
        h = len(v) // 2
        return pairwise(v[:h]) + pairwise(v[h:])

    def sequential(v):
        s = 0.0
        for x in v:
            s += x
        return s

    # the hand-derived value is the row-major pairwise sum, and every other
    # plausible order gives different bits on this leaf
    assert pairwise(list(sq.ravel())) == want
    assert pairwise(list(sq.T.ravel())) == 1.0             # column-major pairwise
    assert sequential(sq.ravel()) == 1.0                    # row-major sequential
    assert sequential(sq.T.ravel()) == 1.0
    assert float(np.sum(sq.ravel())) == 1.0                 # numpy's blocked pairwise
    assert math.fsum(sq.ravel()) == want                    # correctly rounded total


def order_parents():
    """A 32 x 32 matrix of four 16 x 16 leaves (tier 1):

        s(0,0) = 1              (one entry 1.0)
        s(0,1) = 0              (zero leaf)
        s(1,0) = 2^-53          (two entries 2^-27: 2^-54 + 2^-54, exact)
        s(1,1) = 2^-53          (two entries 2^-27)

    Root by (s11 + s12) + (s21 + s22) = (1 + 0) + (2^-53 + 2^-53)
    = 1 + 2^-52 (exact).  Column-first (s11 + s21) + (s12 + s22) =
    (1 + 2^-53) + 2^-53 = 1 + 2^-53, a tie, -> 1.  Sequential
    ((s11 + s12) + s21) + s22 = 1.  So the three orders give two values and
    only the row-pair order gives 1 + 2^-52."""
    A = np.zeros((32, 32), dtype=np.float32)
    A[0, 0] = 1.0
    A[16, 0:2] = E27
    A[17 + 4, 20:22] = E27
    return A


def test_parent_norm_order_is_row_pairs():
    tiers = oracle.norms(order_parents(), 16)
    leaf = tiers[1]
    assert leaf[0, 0] == 1.0 and leaf[0, 1] == 0.0
    assert leaf[1, 0] == 2.0 ** -53 and leaf[1, 1] == 2.0 ** -53
    assert tiers[0][0, 0] == 1.0 + 2.0 ** -52
    # the alternatives this pin rejects
    assert (leaf[0, 0] + leaf[1, 0]) + (leaf[0, 1] + leaf[1, 1]) == 1.0
    assert ((leaf[0, 0] + leaf[0, 1]) + leaf[1, 0]) + leaf[1, 1] == 1.0


def test_reordered_oracle_fails_the_order_pins(tmp_path):
    """Mutation check on the CPU: the oracle recompiled with its leaf sum made
    sequential, or its parent sum taken column-first, must fail the order
    pins above (so those pins see the order, not only the bound)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(oracle._SRC).read()
    seq = src.replace(
        "    int64_t h = len / 2;\n    return pairwise_sum(v, h) + pairwise_sum(v + h, len - h);",
        "    double s = 0.0;\n    for (int64_t i = 0; i < len; ++i)\n        s += v[i];\n"
        "    return s;")
    col = src.replace("pa[I * Nt + J] = (s11 + s12) + (s21 + s22);",
                      "pa[I * Nt + J] = (s11 + s21) + (s12 + s22);")
    assert seq != src and col != src
    for name, text, case, ok_value in (
            ("seq", seq, order_leaf(), 1.0 + 2.0 ** -52),
            ("col", col, order_parents(), 1.0 + 2.0 ** -52)):
        c = tmp_path / f"oracle_{name}.c"
        so = tmp_path / f"oracle_{name}.so"
        c.write_text(text)
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", str(so), str(c), "-lm"])
        lib = ctypes.CDLL(str(so))
        lib.oracle_norms.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.c_void_p]
        n = case.shape[0]
        d, _ = oracle.depth(n, 16)
        out = np.zeros(int(oracle._load().oracle_norms_len(d)), dtype=np.float64)
        a = np.ascontiguousarray(case)
        assert lib.oracle_norms(a.ctypes.data, n, 16, out.ctypes.data) == 0
        assert out[0] != ok_value, name          # the mutant's root differs
        assert oracle.norms(case, 16)[0][0, 0] == ok_value
