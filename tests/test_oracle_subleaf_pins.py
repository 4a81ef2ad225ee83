"""Pins for the reading behind sub-leaf culling.

Culling the 32 x 32 sub-blocks inside every kept 64 x 64 leaf product, with
norms from the pyramid of a tree with 32 x 32 leaves, performs exactly the
sub-products that the flat cull of that tree keeps: the stored norms are
monotone up the tree, so a sub-product that passes its own test has parents
that pass theirs.  Checked here by brute force on the oracle's own norms
(independent of any GPU code), including at tau where many leaf products are
kept only partly, and zero blocks; plus the 64 x 64 tier of the leaf-32
pyramid equals the pairwise sums of the four sub-block norms.
"""
import numpy as np
import pytest

import oracle


def decay(n, rate, seed, sym=True):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return A.astype(np.float32)


def keep(sa, sb, tau):
    return sa > 0 and sb > 0 and not (sa * sb < tau * tau)


@pytest.mark.parametrize("n,tau,seed", [(256, 1e-4, 0), (200, 1e-6, 1), (256, 1e-2, 2),
                                        (130, 0.0, 3)])
def test_subleaf_cull_equals_flat_leaf32_cull(n, tau, seed):
    A = decay(n, 0.05, seed)
    B = decay(n, 0.08, seed + 10, sym=False)
    A[64:128, 128:192] = 0.0            # a whole zero 64 x 64 block
    sA, sB = oracle.norms(A, 32), oracle.norms(B, 32)
    d32 = len(sA) - 1
    s32a, s32b = sA[d32], sB[d32]
    s64a, s64b = sA[d32 - 1], sB[d32 - 1]
    N = s32a.shape[0]
    flat, nested, partial = set(), set(), 0
    for I in range(N // 2):
        for K in range(N // 2):
            for J in range(N // 2):
                outer = keep(s64a[I, K], s64b[K, J], tau)
                inner = 0
                for a in range(2):
                    for b in range(2):
                        for c in range(2):
                            i, k, j = 2 * I + a, 2 * K + c, 2 * J + b
                            if keep(s32a[i, k], s32b[k, j], tau):
                                flat.add((i, k, j))
                                if outer:
                                    nested.add((i, k, j))
                                    inner += 1
                partial += outer and 0 < inner < 8
    assert nested == flat
    ref = oracle.spamm(A, B, 32, tau, want_C=False)
    keys = {(oracle.linear_index(i, j) << 32) | k for i, k, j in flat}
    assert keys == {int(x) for x in ref.keys}
    if tau > 0:
        assert partial > 0          # the inner test has work to do at this tau


def test_leaf64_tier_is_parent_of_subblocks():
    A = decay(192, 0.1, 4)
    s = oracle.norms(A, 32)
    d = len(s) - 1
    ch, pa = s[d], s[d - 1]
    for I in range(pa.shape[0]):
        for J in range(pa.shape[1]):
            q = ch[2 * I:2 * I + 2, 2 * J:2 * J + 2]
            assert pa[I, J] == (q[0, 0] + q[0, 1]) + (q[1, 0] + q[1, 1])
