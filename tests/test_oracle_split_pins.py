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
