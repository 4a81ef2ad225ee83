"""Pins for the oracle's split-precision mode.

* bfloat16 rounding against torch's CPU float32 -> bfloat16 conversion
  (round to nearest even), on ties, denormals and extremes;
* low_tol = 0 reproduces the plain oracle exactly;
* every product LOW at tau = 0 gives numpy's FP64 product of the rounded
  matrices (an operand left unrounded, or rounded twice, fails it);
* the LOW class set equals brute-force enumeration of s_A s_B < low_tol^2
  among the kept products;
* a mixed product equals the per-leaf sum of numpy products, each with the
  operands its class prescribes.

binary16 LOW operands (per-leaf power-of-two scale):

* the scale exponent e of a leaf with squared norm S is the one integer with
  4^(13-e) <= S < 4^(14-e), so every entry is below 2^14 once scaled;
* the rounding equals numpy's float64 -> float16 conversion of x 2^e, on
  ties and scales from 2^-100 to 2^160, with a result below binary16's
  normal range (2^-14) flushed to zero;
* a mixed product equals the per-leaf sum of numpy products with each LOW
  leaf rounded through numpy's float16 at its own scale;
* its error against the unrounded product stays within the per-element
  rounding bound and is well below the bfloat16 one.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def decay(n, rate, seed, sym=True):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return A.astype(np.float32)


def bf16_np(A):
    return torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).to(torch.bfloat16).to(
        torch.float64).numpy()


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    vals = list(rng.standard_normal(2000).astype(np.float32))
    vals += list((rng.standard_normal(500) * 1e-40).astype(np.float32))       # denormals
    vals += [np.float32(3.0e38), np.float32(-3.3e38), np.float32(1.0e-45), np.float32(0.0),
             np.float32(-0.0)]
    # exact ties: low 16 bits 0x8000, with even and odd kept part
    for hi in (0x3F80, 0x3F81, 0x4000, 0x4001, 0x0001, 0x0002, 0xBF80, 0xBF81):
        vals.append(np.array([(hi << 16) | 0x8000], dtype=np.uint32).view(np.float32)[0])
        vals.append(np.array([(hi << 16) | 0x7FFF], dtype=np.uint32).view(np.float32)[0])
        vals.append(np.array([(hi << 16) | 0x8001], dtype=np.uint32).view(np.float32)[0])
    arr = np.array(vals, dtype=np.float32)
    want = bf16_np(arr)
    got = np.array([oracle.bf16(float(v)) for v in arr])
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("tau", [0.0, 1e-5])
def test_low_tol_zero_is_plain_oracle(tau):
    A, B = decay(200, 0.05, 1), decay(200, 0.07, 2, sym=False)
    a = oracle.spamm(A, B, 32, tau)
    b = oracle.spamm(A, B, 32, tau, low_tol=0.0)
    assert b.Klow == 0 and np.array_equal(a.keys, b.keys) and np.array_equal(a.C, b.C)


def test_all_low_is_product_of_rounded_matrices():
    rng = np.random.default_rng(3)
    A = rng.uniform(-1, 1, (150, 150)).astype(np.float32)
    B = rng.uniform(-1, 1, (150, 150)).astype(np.float32)
    r = oracle.spamm(A, B, 32, 0.0, low_tol=1e30)
    assert r.Klow == r.K > 0
    assert np.all(r.keys & oracle.LOW_BIT)
    ref = bf16_np(A) @ bf16_np(B)
    assert np.abs(r.C - ref).max() <= 1e-12 * np.abs(ref).max()
    # and it differs from the unrounded product, so the pin has teeth
    assert np.abs(r.C - A.astype(np.float64) @ B.astype(np.float64)).max() > 1e-4


@pytest.mark.parametrize("tau,low", [(1e-6, 1e-3), (1e-8, 1e-4), (0.0, 1e-2)])
def test_low_class_set_bruteforce(tau, low):
    A = decay(256, 0.06, 4)
    b = 32
    r = oracle.spamm(A, A, b, tau, want_C=False, low_tol=low)
    s = oracle.norms(A, b)[-1]
    N = s.shape[0]
    want = set()
    for I in range(N):
        for K in range(N):
            for J in range(N):
                sa, sb = s[I, K], s[K, J]
                if sa > 0 and sb > 0 and not (sa * sb < tau * tau) and sa * sb < low * low:
                    want.add((oracle.linear_index(I, J) << 32) | K)
    got = {int(k) & ~(1 << 63) for k in r.keys if int(k) >> 63}
    assert got == want and r.Klow == len(want)
    assert 0 < r.Klow < r.K


def test_mixed_product_per_leaf():
    A, B = decay(192, 0.04, 5), decay(192, 0.05, 6, sym=False)
    b, tau, low = 32, 1e-6, 3e-2
    r = oracle.spamm(A, B, b, tau, low_tol=low)
    assert 0 < r.Klow < r.K
    d, np_ = oracle.depth(192, b)
    N = 1 << d
    PA = np.zeros((np_, np_))
    PB = np.zeros((np_, np_))
    PA[:192, :192] = A
    PB[:192, :192] = B
    RA, RB = bf16_np(PA.astype(np.float32)), bf16_np(PB.astype(np.float32))
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    C = np.zeros((np_, np_))
    for key in r.keys:
        key = int(key)
        low_c = key >> 63
        I, J = inv[(key >> 32) & 0x7FFFFFFF]
        k = key & 0xFFFFFFFF
        X, Y = (RA, RB) if low_c else (PA, PB)
        C[I * b:(I + 1) * b, J * b:(J + 1) * b] += X[I * b:(I + 1) * b, k * b:(k + 1) * b] @ \
            Y[k * b:(k + 1) * b, J * b:(J + 1) * b]
    assert np.abs(C[:192, :192] - r.C).max() <= 1e-12 * (1 + np.abs(C).max())


def test_tile_recursion_matches_full_split():
    A = decay(256, 0.05, 7)
    b, tau, low = 32, 1e-7, 1e-2
    full = oracle.spamm(A, A, b, tau, low_tol=low)
    N = 8
    tiles = [(I, J) for I in range(N) for J in range(N)]
    Ct, counts, kl = oracle.spamm_tiles(A, A, b, tau, tiles, threads=4, want_klists=True,
                                        low_tol=low)
    keys = []
    for s_, (I, J) in enumerate(tiles):
        for v in kl[s_, :counts[s_]]:
            v = int(v)
            keys.append((oracle.linear_index(I, J) << 32) | (v & 0x3FFFFFFF) | ((v >> 30) << 63))
    order = np.argsort(np.array(keys, dtype=np.uint64) & ~oracle.LOW_BIT, kind="stable")
    assert np.array_equal(np.array(keys, dtype=np.uint64)[order], full.keys)
    Cp = np.zeros((N * b, N * b))
    Cp[:256, :256] = full.C
    for s_, (I, J) in enumerate(tiles):
        assert np.array_equal(Ct[s_], Cp[I * b:(I + 1) * b, J * b:(J + 1) * b])


# ---- binary16 LOW operands ---------------------------------------------------

@pytest.mark.parametrize("S", [1.0, 2.0, 4.0, 0.25, 3.999999, 4.000001, 1e-90, 7.3e-60,
                               1.5e30, 2.0 ** -298, 123456.0, 0.0])
def test_fp16_exponent_closed_form(S):
    import math
    e = oracle.fp16_exponent(S)
    if S == 0.0:
        assert e == 0
        return
    # the unique e with 4^(13-e) <= S < 4^(14-e), i.e. sqrt(S) 2^e in [2^13, 2^14)
    assert math.ldexp(1.0, 2 * (13 - e)) <= S < math.ldexp(1.0, 2 * (14 - e))


def test_fp16_rounding_matches_numpy():
    rng = np.random.default_rng(11)
    cases = []
    for e in (-100, -7, 0, 3, 13, 40, 100, 160):
        # magnitudes spanning binary16's normal and subnormal ranges after scaling
        mags = 2.0 ** rng.uniform(-30, 14, 400) * 2.0 ** -e
        xs = (rng.choice([-1.0, 1.0], 400) * mags).astype(np.float32)
        cases += [(float(x), e) for x in xs if x != 0 and abs(float(x) * 2.0 ** e) < 2.0 ** 14]
    # exact ties at several binades, normal and subnormal, even and odd kept part
    for base in (1.0, 1.0 + 2.0 ** -10, 2.0 ** -14, 2.0 ** -20, 2.0 ** -24, 3 * 2.0 ** -24):
        q = 2.0 ** (max(int(np.floor(np.log2(base))), -14) - 10)    # binary16 spacing at base
        cases += [(float(np.float32(base + q / 2)), 0), (float(np.float32(-(base + q / 2))), 0)]
    cases += [(0.0, 5), (float(np.float32(1e-45)), 149), (float(np.float32(1e-45)), 120)]
    # the boundary: within half a subnormal spacing below 2^-14 rounds up and
    # stays; one spacing below is a subnormal and becomes zero
    assert oracle.fp16_scaled(np.float32(2.0 ** -14 - 2.0 ** -26), 0) == 2.0 ** -14
    assert oracle.fp16_scaled(np.float32(2.0 ** -14 - 2.0 ** -24), 0) == 0.0
    assert oracle.fp16_scaled(np.float32(-(2.0 ** -14)), 0) == -(2.0 ** -14)
    for x, e in cases:
        h = float(np.float16(np.float64(np.float32(x)) * 2.0 ** e))
        want = (h if abs(h) >= 2.0 ** -14 else 0.0) * 2.0 ** -e
        got = oracle.fp16_scaled(np.float32(x), e)
        assert got == want, (x, e, got, want)


def fp16_leaves(P, b, S):
    """P (padded FP32) with every leaf rounded through numpy float16 at the
    scale exponent of its squared norm, binary16 subnormals flushed."""
    N = P.shape[0] // b
    R = np.zeros(P.shape)
    for I in range(N):
        for J in range(N):
            e = oracle.fp16_exponent(S[I, J])
            blk = P[I * b:(I + 1) * b, J * b:(J + 1) * b].astype(np.float64) * 2.0 ** e
            h = blk.astype(np.float16).astype(np.float64)
            R[I * b:(I + 1) * b, J * b:(J + 1) * b] = np.where(np.abs(h) < 2.0 ** -14, 0.0, h) * \
                2.0 ** -e
    return R


@pytest.mark.parametrize("n,b,tau,low", [(192, 32, 1e-6, 3e-2), (150, 16, 1e-7, 1e-1),
                                         (130, 64, 0.0, 1e30)])
def test_fp16_mixed_product_per_leaf(n, b, tau, low):
    A, B = decay(n, 0.04, 21), 1e-3 * decay(n, 0.3, 22, sym=False)
    r = oracle.spamm(A, B, b, tau, low_tol=low, low_fmt="fp16")
    assert r.Klow > 0
    rb = oracle.spamm(A, B, b, tau, low_tol=low)
    assert np.array_equal(r.keys, rb.keys) and r.Klow == rb.Klow     # same classes as bf16
    d, np_ = oracle.depth(n, b)
    N = 1 << d
    PA = np.zeros((np_, np_), dtype=np.float32)
    PB = np.zeros((np_, np_), dtype=np.float32)
    PA[:n, :n] = A
    PB[:n, :n] = B
    RA = fp16_leaves(PA, b, oracle.norms(A, b)[-1])
    RB = fp16_leaves(PB, b, oracle.norms(B, b)[-1])
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    C = np.zeros((np_, np_))
    for key in r.keys:
        key = int(key)
        I, J = inv[(key >> 32) & 0x7FFFFFFF]
        k = key & 0xFFFFFFFF
        X, Y = (RA, RB) if key >> 63 else (PA.astype(np.float64), PB.astype(np.float64))
        C[I * b:(I + 1) * b, J * b:(J + 1) * b] += X[I * b:(I + 1) * b, k * b:(k + 1) * b] @ \
            Y[k * b:(k + 1) * b, J * b:(J + 1) * b]
    assert np.abs(C[:n, :n] - r.C).max() <= 1e-12 * (1 + np.abs(C).max())


def test_fp16_error_within_rounding_bound_and_below_bf16():
    n, b = 256, 32
    A = decay(n, 0.08, 23)
    low = 1e30                                   # every kept product LOW
    exact = oracle.spamm(A, A, b, 0.0)
    f16 = oracle.spamm(A, A, b, 0.0, low_tol=low, low_fmt="fp16")
    b16 = oracle.spamm(A, A, b, 0.0, low_tol=low)
    assert f16.Klow == f16.K
    # per element |fl16(x) - x| <= 2^-11 |x| + 2^-14 2^-e (a flushed value is
    # below 2^-14, scaled back); propagate through |dA||A| + |A||dA| + |dA||dA|
    S = oracle.norms(A, b)[-1]
    N = n // b
    D = np.zeros((n, n))
    for I in range(N):
        for J in range(N):
            e = oracle.fp16_exponent(S[I, J])
            blk = np.abs(A[I * b:(I + 1) * b, J * b:(J + 1) * b].astype(np.float64))
            D[I * b:(I + 1) * b, J * b:(J + 1) * b] = 2.0 ** -11 * blk + 2.0 ** (-14 - e)
    Aa = np.abs(A.astype(np.float64))
    bound = D @ Aa + Aa @ D + D @ D
    err16 = np.abs(f16.C - exact.C)
    assert np.all(err16 <= bound * (1 + 1e-9) + 1e-300)
    errb = np.abs(b16.C - exact.C).max()
    assert 0 < err16.max() < errb / 4


# --------------------------------------------------------------------------
# Relative LOW threshold: LOW iff ||A_ik|| ||B_kj|| < theta ||A||_F ||B||_F
# (norm product small relative to ||A|| ||B||, the precision outlook of
# Sec. VI), taken as s_A s_B < (theta^2 s_A0) s_B0 on the stored squared norms.
# --------------------------------------------------------------------------
def exact_sq_norms(P, b):
    """Exact (rational) squared Frobenius norm of every leaf of the padded
    matrix and of the whole matrix: sums of squares of FP32 values, done in
    Fractions (no rounding at all)."""
    from fractions import Fraction
    N = P.shape[0] // b
    leaf = [[sum((Fraction(float(x)) ** 2 for x in P[I * b:(I + 1) * b, J * b:(J + 1) * b].ravel()
                  if x != 0), Fraction(0)) for J in range(N)] for I in range(N)]
    total = sum((leaf[I][J] for I in range(N) for J in range(N)), Fraction(0))
    return leaf, total


@pytest.mark.parametrize("theta,tau", [(1e-2, 1e-6), (1e-3, 1e-8), (3e-2, 0.0)])
def test_relative_low_set_against_exact_norms(theta, tau):
    """The relative LOW class equals the exact-arithmetic classification
    ||A_ik|| ||B_kj|| < theta ||A|| ||B|| (rational squared norms; triples
    within 1e-9 of the threshold are left out)."""
    from fractions import Fraction
    A, B = decay(160, 0.05, 21), decay(160, 0.08, 22, sym=False)
    b = 32
    r = oracle.spamm(A, B, b, tau, want_C=False, low_rel=theta)
    d, np_ = oracle.depth(160, b)
    PA = np.zeros((np_, np_), dtype=np.float32)
    PB = np.zeros((np_, np_), dtype=np.float32)
    PA[:160, :160], PB[:160, :160] = A, B
    sA, SA = exact_sq_norms(PA, b)
    sB, SB = exact_sq_norms(PB, b)
    th2 = Fraction(theta) ** 2
    kept = {int(k) & ~(1 << 63): int(k) >> 63 for k in r.keys}
    N = 1 << d
    checked = 0
    for I in range(N):
        for K in range(N):
            for J in range(N):
                key = (oracle.linear_index(I, J) << 32) | K
                if key not in kept:
                    continue
                lhs, rhs = sA[I][K] * sB[K][J], th2 * SA * SB
                if abs(lhs - rhs) <= Fraction(1, 10 ** 9) * rhs:
                    continue
                assert kept[key] == int(lhs < rhs), (I, K, J)
                checked += 1
    assert checked > 0 and 0 < r.Klow < r.K


def test_relative_low_is_scale_invariant():
    """Scaling A by 2^7 and B by 2^-5 (exact) leaves the relative classes
    unchanged; the same absolute threshold changes them (so a threshold
    that ignored the roots would fail here)."""
    A, B = decay(200, 0.05, 23), decay(200, 0.07, 24, sym=False)
    b, theta = 32, 2e-3
    base = oracle.spamm(A, B, b, 0.0, want_C=False, low_rel=theta)
    As, Bs = (A * np.float32(2.0 ** 7)), (B * np.float32(2.0 ** -5))
    scaled = oracle.spamm(As, Bs, b, 0.0, want_C=False, low_rel=theta)
    assert 0 < base.Klow < base.K
    assert np.array_equal(base.keys, scaled.keys) and base.Klow == scaled.Klow
    # an absolute threshold equal to theta ||A|| ||B|| of the unscaled pair
    sA0 = oracle.norms(A, b)[0][0, 0]
    sB0 = oracle.norms(B, b)[0][0, 0]
    low = theta * np.sqrt(sA0) * np.sqrt(sB0)
    a1 = oracle.spamm(A, B, b, 0.0, want_C=False, low_tol=low)
    a2 = oracle.spamm(As, Bs, b, 0.0, want_C=False, low_tol=low)
    assert a1.Klow != a2.Klow


def test_relative_low_product_and_tiles():
    """C of a relative split product equals the absolute split product at the
    matching threshold when no norm product sits near it, and the per-leaf
    recursion gives the same classes and values."""
    A = decay(192, 0.05, 25)
    b, tau, theta = 32, 1e-7, 1e-3
    r = oracle.spamm(A, A, b, tau, low_rel=theta)
    s = oracle.norms(A, b)
    low = theta * s[0][0, 0]                          # theta ||A||^2
    leaf = s[-1]
    prod = leaf[:, :, None] * leaf[None, :, :]
    assert np.all(np.abs(prod - low * low) > 1e-9 * low * low)
    a = oracle.spamm(A, A, b, tau, low_tol=low)
    assert np.array_equal(r.keys, a.keys) and np.array_equal(r.C, a.C) and 0 < r.Klow < r.K
    N = leaf.shape[0]
    tiles = [(I, J) for I in range(N) for J in range(N)]
    Ct, counts, kl = oracle.spamm_tiles(A, A, b, tau, tiles, threads=2, want_klists=True,
                                        low_rel=theta)
    assert counts.sum() == r.K
    assert int(sum(int((kl[s_, :counts[s_]] >> 30).sum()) for s_ in range(len(tiles)))) == r.Klow
    for s_, (I, J) in enumerate(tiles):
        r0, c0 = I * b, J * b
        blk = r.C[r0:r0 + b, c0:c0 + b]
        assert np.array_equal(Ct[s_][:blk.shape[0], :blk.shape[1]], blk)


def test_relative_low_rejects_bad_arguments():
    A = decay(64, 0.1, 26)
    with pytest.raises(ValueError):
        oracle.spamm(A, A, 32, 0.0, low_tol=1e-3, low_rel=1e-3)
    for bad in (-1e-3, float("inf"), float("nan")):
        with pytest.raises(RuntimeError):
            oracle.spamm(A, A, 32, 0.0, low_rel=bad)
