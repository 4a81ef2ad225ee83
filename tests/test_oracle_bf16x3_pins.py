"""Pins for the oracle's compensated split mode (low_fmt="bf16x3").

LOW products round their operands to bfloat16, as in the plain split mode;
a HIGH product takes each entry x as its two bfloat16 parts, hi = bf16(x)
and lo = bf16(x - hi), and a b as hi_a hi_b + hi_a lo_b + lo_a hi_b (the
three-product bfloat16 method of Henry, Tang and Heinecke, ARITH 2019).

* the parts equal torch's bfloat16 rounding of x and of numpy's float32
  x - hi, and hi + lo recovers x built from known parts;
* on matrices built as A = H + L from known bfloat16 parts (x - hi exact,
  lo exact), the all-HIGH product equals numpy's A B - L_A L_B: the one
  dropped term is lo lo, and a transposed or missing term fails it;
* on random inputs the error against the exact product stays within
  2^-14 sum |a||b| per element, which bfloat16 operands alone exceed;
* the classes are those of the plain split mode, an all-LOW product is the
  plain split mode's, and a mixed product equals the per-leaf sum of numpy
  products with each class's operands;
* the tile recursion and the relative threshold give the same result.
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


def parts_np(A):
    """(hi, lo) by torch's rounding and numpy's float32 subtraction."""
    A = np.asarray(A, dtype=np.float32)
    H = bf16_np(A)
    R = A - H.astype(np.float32)                 # float32 arithmetic
    return H, bf16_np(R)


def built(n, seed, lo_scale=2.0 ** -11):
    """A = H + L with H, L bfloat16 matrices, |L| in [1, 2) 2^-12 |H| ... so
    that bf16(A) = H exactly and A is exact in float32."""
    rng = np.random.default_rng(seed)
    H = bf16_np(rng.uniform(-1, 1, (n, n)).astype(np.float32) *
                np.float32(2.0) ** rng.integers(-6, 6, (n, n)).astype(np.float32))
    u = rng.uniform(1.0, 2.0, (n, n)) * rng.choice([-1.0, 1.0], (n, n))
    L = bf16_np((H * u * lo_scale).astype(np.float32))
    A = (H + L).astype(np.float32)
    assert np.array_equal(A.astype(np.float64), H + L)       # exact in float32
    return A, H, L


def test_parts_match_torch_and_recover_built_values():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(3000).astype(np.float32),
                        (rng.standard_normal(200) * 1e-39).astype(np.float32),   # denormals
                        np.array([1.0, -2.0, 0.0, 3.0e38, 1.00390625, 1.0 - 2.0 ** -24],
                                 dtype=np.float32)])
    # values whose bfloat16 rounding crosses into the next binade (lo < 0)
    x = np.concatenate([x, np.nextafter(np.float32(2.0) ** np.arange(-5, 5, dtype=np.float32),
                                        np.float32(0.0))])
    H, L = parts_np(x)
    got = np.array([oracle.bf16_parts(float(v)) for v in x])
    assert np.array_equal(got[:, 0].view(np.uint64), H.view(np.uint64))
    assert np.array_equal(got[:, 1].view(np.uint64), L.view(np.uint64))
    assert np.any(got[:, 1] < 0) and np.any(got[:, 1] > 0)
    # built values: the parts come back exactly
    A, Hb, Lb = built(40, 1)
    got = np.array([oracle.bf16_parts(float(v)) for v in A.ravel()])
    assert np.array_equal(got[:, 0], Hb.ravel()) and np.array_equal(got[:, 1], Lb.ravel())


@pytest.mark.parametrize("n,b", [(150, 32), (96, 16)])
def test_all_high_product_drops_exactly_lo_lo(n, b):
    A, HA, LA = built(n, 2)
    B, HB, LB = built(n, 3)
    r = oracle.spamm(A, B, b, 0.0, low_fmt="bf16x3")
    assert r.Klow == 0 and r.K > 0
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    want = A64 @ B64 - LA @ LB
    scale = np.abs(A64) @ np.abs(B64)
    assert np.all(np.abs(r.C - want) <= 1e-13 * scale + 1e-300)
    # the dropped term is visible, and neither operand's parts are swapped
    assert np.max(np.abs(r.C - A64 @ B64) / scale) > 1e-8
    assert np.max(np.abs(r.C - (A64 @ B64 - LA @ LB.T)) / scale) > 1e-8
    assert np.max(np.abs(r.C - (HA @ HB + HA @ LB)) / scale) > 1e-5


@pytest.mark.parametrize("seed", [4, 5])
def test_error_within_compensated_bound(seed):
    rng = np.random.default_rng(seed)
    n = 128
    A = (rng.uniform(-1, 1, (n, n)) * 10.0 ** rng.uniform(-3, 3, (n, n))).astype(np.float32)
    B = (rng.uniform(-1, 1, (n, n)) * 10.0 ** rng.uniform(-3, 3, (n, n))).astype(np.float32)
    r = oracle.spamm(A, B, 32, 0.0, low_fmt="bf16x3")
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    exact = A64 @ B64
    bound = 2.0 ** -14 * (np.abs(A64) @ np.abs(B64))
    assert np.all(np.abs(r.C - exact) <= bound)
    # bfloat16 operands alone do not meet it
    r16 = oracle.spamm(A, B, 32, 0.0, low_tol=1e30)
    assert np.any(np.abs(r16.C - exact) > bound)


def test_classes_and_low_products_are_the_plain_split_modes():
    A, B = decay(192, 0.04, 5), decay(192, 0.05, 6, sym=False)
    b, tau, low = 32, 1e-6, 3e-2
    a = oracle.spamm(A, B, b, tau, low_tol=low)
    c = oracle.spamm(A, B, b, tau, low_tol=low, low_fmt="bf16x3")
    assert np.array_equal(a.keys, c.keys) and a.Klow == c.Klow and 0 < c.Klow < c.K
    a = oracle.spamm(A, B, b, 0.0, low_tol=1e30)
    c = oracle.spamm(A, B, b, 0.0, low_tol=1e30, low_fmt="bf16x3")
    assert c.Klow == c.K and np.array_equal(a.C, c.C)


def test_mixed_product_per_leaf():
    n, b, tau, low = 192, 32, 1e-6, 3e-2
    A, B = decay(n, 0.04, 7), decay(n, 0.05, 8, sym=False)
    r = oracle.spamm(A, B, b, tau, low_tol=low, low_fmt="bf16x3")
    assert 0 < r.Klow < r.K
    d, np_ = oracle.depth(n, b)
    N = 1 << d
    PA = np.zeros((np_, np_), dtype=np.float32)
    PB = np.zeros((np_, np_), dtype=np.float32)
    PA[:n, :n] = A
    PB[:n, :n] = B
    HA, LA = parts_np(PA)
    HB, LB = parts_np(PB)
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    C = np.zeros((np_, np_))
    for key in r.keys:
        key = int(key)
        I, J = inv[(key >> 32) & 0x7FFFFFFF]
        k = key & 0xFFFFFFFF
        ia, ka, ja = slice(I * b, I * b + b), slice(k * b, k * b + b), slice(J * b, J * b + b)
        if key >> 63:
            C[ia, ja] += HA[ia, ka] @ HB[ka, ja]                     # bfloat16 operands
        else:
            C[ia, ja] += HA[ia, ka] @ HB[ka, ja] + HA[ia, ka] @ LB[ka, ja] + \
                LA[ia, ka] @ HB[ka, ja]
    assert np.abs(C[:n, :n] - r.C).max() <= 1e-12 * (1 + np.abs(C).max())


def test_tiles_and_relative_threshold():
    A = decay(256, 0.05, 9)
    b, tau = 32, 1e-7
    full = oracle.spamm(A, A, b, tau, low_rel=1e-3, low_fmt="bf16x3")
    assert 0 < full.Klow < full.K
    N = 8
    tiles = [(I, J) for I in range(N) for J in range(N)]
    Ct, counts, _ = oracle.spamm_tiles(A, A, b, tau, tiles, threads=4, low_rel=1e-3,
                                       low_fmt="bf16x3")
    for t, (I, J) in enumerate(tiles):
        assert np.array_equal(Ct[t], full.C[I * b:(I + 1) * b, J * b:(J + 1) * b])
    plain = oracle.spamm(A, A, b, tau, low_rel=1e-3)
    assert np.array_equal(plain.keys, full.keys)
    assert not np.array_equal(plain.C, full.C)
