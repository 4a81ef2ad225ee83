"""Randomized pins for the oracle (hypothesis, derandomized): the same facts
as the fixed-case pins, over drawn shapes, leaf sizes, decay rates, zero
blocks and tolerances.

* norms: every leaf against math.fsum of its squares within the pairwise
  bound; every parent against the exact sum of its four children's fsum;
* task set: brute-force flat enumeration of the keep test on the leaf norms
  (equal to the recursion by monotonicity), sorted by (linear index, k);
* tau = 0: the product equals numpy's FP64 product;
* truncation: each output leaf within sum over skipped k of ||A_Ik|| ||B_kJ||;
* split precision: the LOW set is the brute-force set {s_A s_B < low_tol^2}
  among kept products, and binary16 LOW operands match per-leaf numpy float16
  products (binary16 subnormals flushed to zero).
"""
import math

import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle

U = 2.0 ** -53
CFG = settings(max_examples=25, deadline=None, derandomize=True,
               suppress_health_check=[HealthCheck.too_slow])


@st.composite
def problems(draw):
    leaf = draw(st.sampled_from([16, 32]))
    n = draw(st.integers(1, 5 * leaf))
    rate = draw(st.floats(0.0, 0.6))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    zero_block = draw(st.booleans())
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    env = np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    A = (rng.uniform(-1, 1, (n, n)) * env).astype(np.float32)
    B = (rng.uniform(-1, 1, (n, n)) * env.T).astype(np.float32)
    if zero_block and n > leaf:
        A[:leaf, leaf:2 * leaf] = 0.0
    tau = draw(st.sampled_from([0.0, 1e-9, 1e-6, 1e-4, 1e-2, 1.0]))
    return A, B, leaf, tau


def padded(A, leaf):
    d, np_ = oracle.depth(A.shape[0], leaf)
    P = np.zeros((np_, np_))
    P[:A.shape[0], :A.shape[0]] = A
    return P, d


@CFG
@given(problems())
def test_norms_against_fsum(p):
    A, _, leaf, _ = p
    P, d = padded(A, leaf)
    tiers = oracle.norms(A, leaf)
    N = 1 << d
    exact = np.zeros((N, N))
    for I in range(N):
        for J in range(N):
            blk = P[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf]
            exact[I, J] = math.fsum((blk * blk).ravel())
    bound = math.ceil(math.log2(leaf * leaf)) * U
    assert np.all(np.abs(tiers[-1] - exact) <= bound * exact)
    for t in range(d - 1, -1, -1):
        m = 1 << t
        ex = exact.reshape(m, N // m, m, N // m).sum(axis=(1, 3))
        slack = (math.ceil(math.log2(leaf * leaf)) + 2 * (d - t)) * U
        assert np.all(np.abs(tiers[t] - ex) <= slack * ex)


@CFG
@given(problems())
def test_task_set_and_product(p):
    A, B, leaf, tau = p
    n = A.shape[0]
    r = oracle.spamm(A, B, leaf, tau)
    sA, sB = oracle.norms(A, leaf)[-1], oracle.norms(B, leaf)[-1]
    N = sA.shape[0]
    want = sorted((oracle.linear_index(I, J) << 32) | K
                  for I in range(N) for K in range(N) for J in range(N)
                  if sA[I, K] > 0 and sB[K, J] > 0 and not (sA[I, K] * sB[K, J] < tau * tau))
    assert [int(k) for k in r.keys] == want
    PA, _ = padded(A, leaf)
    PB, _ = padded(B, leaf)
    if tau == 0.0:
        ref = PA @ PB
        assert np.abs(r.C - ref[:n, :n]).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    exact = (PA @ PB)
    kept = {(int(k) >> 32, int(k) & 0xFFFFFFFF) for k in r.keys}
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    nA, nB = np.sqrt(sA), np.sqrt(sB)
    Cp = np.zeros_like(exact)
    Cp[:n, :n] = r.C
    for l, (I, J) in inv.items():
        skipped = sum(nA[I, k] * nB[k, J] for k in range(N) if (l, k) not in kept)
        diff = np.linalg.norm(exact[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] -
                              Cp[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf])
        assert diff <= skipped * (1 + 1e-9) + 1e-12 * (1 + np.abs(exact).max())


@CFG
@given(problems(), st.sampled_from([1e-3, 1e-2, 1e-1, 1e30]))
def test_split_classes_and_fp16_operands(p, low):
    A, B, leaf, tau = p
    n = A.shape[0]
    r = oracle.spamm(A, B, leaf, tau, low_tol=low, low_fmt="fp16")
    sA, sB = oracle.norms(A, leaf)[-1], oracle.norms(B, leaf)[-1]
    inv = {oracle.linear_index(i, j): (i, j) for i in range(sA.shape[0]) for j in range(sA.shape[0])}
    PA, _ = padded(A, leaf)
    PB, _ = padded(B, leaf)
    C = np.zeros_like(PA)
    for key in r.keys:
        key = int(key)
        I, J = inv[(key >> 32) & 0x7FFFFFFF]
        k = key & 0xFFFFFFFF
        low_c = sA[I, k] * sB[k, J] < low * low
        assert bool(key >> 63) == low_c
        X = PA[I * leaf:(I + 1) * leaf, k * leaf:(k + 1) * leaf]
        Y = PB[k * leaf:(k + 1) * leaf, J * leaf:(J + 1) * leaf]
        if low_c:
            ea, eb = oracle.fp16_exponent(sA[I, k]), oracle.fp16_exponent(sB[k, J])
            hx = (X * 2.0 ** ea).astype(np.float16).astype(np.float64)
            hy = (Y * 2.0 ** eb).astype(np.float16).astype(np.float64)
            X = np.where(np.abs(hx) < 2.0 ** -14, 0.0, hx) * 2.0 ** -ea
            Y = np.where(np.abs(hy) < 2.0 ** -14, 0.0, hy) * 2.0 ** -eb
        C[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] += X @ Y
    assert np.abs(C[:n, :n] - r.C).max() <= 1e-12 * (1 + np.abs(C).max())
