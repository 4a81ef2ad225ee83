"""Pins for epsilon-sparsified trees (Sec. II.C, Eq. epsilon).

* the dropped set against a brute-force reading of the definition
  ||A_IJ||_F < tau / max(||A||_F, ||B||_F) with norms from math.fsum, away
  from rounding ties;
* consistency with the product's test: a product of sparsified operands keeps
  exactly the leaf products of the dense operands and gives the same C
  (a dropped leaf times any leaf of norm <= max(||A||, ||B||) is below tau);
* zero leaves are always dropped, nothing else at tau = 0;
* storage grows linearly in n for exponential decay at fixed tau (the O(n)
  storage of the paper's discussion).
"""
import math

import numpy as np
import pytest

import oracle
import workloads


def decay(n, rate, seed, sym=True):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return A.astype(np.float32)


def fro(M):
    return math.sqrt(math.fsum(float(x) * float(x) for x in np.asarray(M, np.float64).ravel()))


@pytest.mark.parametrize("tau", [1e-3, 1e-5])
def test_dropped_set_bruteforce(tau):
    A = decay(200, 0.05, 0)
    b = 32
    S, keep = oracle.sparsify(A, b, tau)
    nA = fro(A)
    eps = tau / nA
    d, np_ = oracle.depth(200, b)
    P = np.zeros((np_, np_))
    P[:200, :200] = A
    N = 1 << d
    checked = 0
    for I in range(N):
        for J in range(N):
            v = fro(P[I * b:(I + 1) * b, J * b:(J + 1) * b])
            if v == 0.0:
                assert not keep[I, J]
                continue
            if abs(v - eps) <= 1e-12 * eps:
                continue                      # too close to call by this route
            assert keep[I, J] == (v >= eps)
            checked += 1
    assert checked > 0 and 0 < keep.sum() < N * N
    # dropped leaves are zero in the returned matrix, kept ones untouched
    for I in range(N):
        for J in range(N):
            blk = S[I * b:(I + 1) * b, J * b:(J + 1) * b]
            ref = A[I * b:(I + 1) * b, J * b:(J + 1) * b]
            assert np.array_equal(blk, ref if keep[I, J] else np.zeros_like(ref))


@pytest.mark.parametrize("n,b,tau,rate", [(256, 32, 1e-4, 0.3), (300, 16, 1e-6, 0.3),
                                          (500, 64, 1e-5, 0.1), (256, 32, 1e-2, 0.1)])
def test_sparsified_product_equals_dense(n, b, tau, rate):
    A = decay(n, rate, 1)
    S, keep = oracle.sparsify(A, b, tau)
    assert not keep.all()
    dense = oracle.spamm(A, A, b, tau)
    sparse = oracle.spamm(S, S, b, tau)
    assert np.array_equal(sparse.keys, dense.keys)
    assert np.array_equal(sparse.C, dense.C)
    # upper tiers can only shrink
    assert all(ks <= kd for ks, kd in zip(sparse.Kt, dense.Kt))


def test_two_operands_use_the_larger_norm():
    A = decay(256, 0.2, 2, sym=False)
    B = 30.0 * decay(256, 0.25, 3, sym=False)
    tau = 1e-4
    nA2 = float(oracle.norms(A, 32)[0][0, 0])
    nB2 = float(oracle.norms(B, 32)[0][0, 0])
    SA, kA = oracle.sparsify(A, 32, tau, norm2_other=nB2)
    SB, kB = oracle.sparsify(B, 32, tau, norm2_other=nA2)
    dense = oracle.spamm(A, B, 32, tau)
    sparse = oracle.spamm(SA, SB, 32, tau)
    assert np.array_equal(sparse.keys, dense.keys) and np.array_equal(sparse.C, dense.C)
    assert not kA.all()
    # against its own (smaller) norm alone A would drop more leaves, and some
    # of them take part in kept products: the larger norm is needed
    S_self, k_self = oracle.sparsify(A, 32, tau)
    assert k_self.sum() < kA.sum() and (kA & ~k_self).any()
    wrong = oracle.spamm(S_self, SB, 32, tau, want_C=False)
    assert wrong.K < dense.K


def test_tau0_drops_only_zero_leaves():
    A = decay(192, 0.1, 4)
    A[64:96, 0:32] = 0.0
    S, keep = oracle.sparsify(A, 32, 0.0)
    assert np.array_equal(S, A)
    assert not keep[2, 0] and keep.sum() == keep.size - 1 - (keep.size - np.count_nonzero(
        oracle.norms(A, 32)[-1]) - 1)


def test_storage_linear_in_n():
    stored = []
    for n in (1024, 2048, 4096):
        A = workloads.exp_decay(n, 0.1, 0)
        _, keep = oracle.sparsify(A, 32, 1e-8)
        stored.append(int(keep.sum()))
    r1, r2 = stored[1] / stored[0], stored[2] / stored[1]
    assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, stored
    assert stored[2] < 0.15 * (4096 // 32) ** 2
