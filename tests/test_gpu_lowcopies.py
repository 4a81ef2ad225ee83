"""The 16-bit leaf copies of split precision (the LOW operands), bit for bit
against the oracle, read back through spamm_tree_matrix16:

* BF16 copies: every element equals oracle.bf16 of the FP32 element;
* FP16 copies: each leaf's exponent equals oracle.fp16_exponent of the
  oracle's squared norm of that leaf, and every element, scaled back by it,
  equals oracle.fp16_scaled (nearest even at x 2^e, results below 2^-14
  flushed to zero);
* both the left-operand copy and the transposed right-operand copy, over the
  whole padded matrix (zero padding included) or, at n = 4133, sampled leaves.

The inputs plant binary16 and bfloat16 ties, values at the edge of the
flush range and leaves scaled over a wide range of binades, so that the
rounding and exponent paths are all exercised; the test checks that they were.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def planted(n, leaf, seed):
    """Random decaying matrix whose leaves are scaled by 2^s, s in [-60, 40];
    every third leaf is a dominant 2^s at its corner plus planted ties and
    flush-edge values relative to the exponent that leaf gets; some leaves
    are zero."""
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-0.01 * np.abs(i[:, None] - i[None, :]))
    N = -(-n // leaf)
    for I in range(N):
        for J in range(N):
            blk = A[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf]
            s = int(rng.integers(-60, 41))
            kind = (I * N + J) % 7
            if kind == 0:
                blk[:] = 0.0
                continue
            if kind in (1, 4) and blk.shape[0] == leaf and blk.shape[1] == leaf:
                # dominant 2^s: squared norm in [4^s, 2 4^s), FP16 exponent 13 - s
                blk[:] *= 2.0 ** (s - 40)
                blk[0, 0] = 2.0 ** s
                e = 13 - s
                ties = [(1 + 2.0 ** -11) * 2.0 ** j for j in range(-14, 0)]
                ties += [(1 + 3 * 2.0 ** -11) * 2.0 ** j for j in range(-14, 0)]
                ties += [1023.5 * 2.0 ** -24, 1022.5 * 2.0 ** -24, 1023.25 * 2.0 ** -24,
                         600.0 * 2.0 ** -24, 511.75 * 2.0 ** -24]
                ties += [(1 + 2.0 ** -8) * 2.0 ** -3, (1 + 3 * 2.0 ** -8) * 2.0 ** -5]
                for m, t in enumerate(ties):
                    r, c = 1 + m // (leaf - 1), 1 + m % (leaf - 1)
                    blk[r, c] = (-1) ** m * t * 2.0 ** -e
            else:
                blk[:] *= 2.0 ** s
    return A.astype(np.float32)


def bits_to_bf16(h):
    return (h.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bits_to_fp16(h):
    return h.view(np.float16).astype(np.float64)


def expected(P, leaf, fmt, S, blocks):
    """Oracle values of the 16-bit copy for the leaves in `blocks`."""
    out = {}
    for (I, J) in blocks:
        blk = P[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf]
        if fmt == "bf16":
            out[(I, J)] = (np.array([oracle.bf16(float(x)) for x in blk.ravel()]).reshape(blk.shape),
                           None)
        else:
            e = oracle.fp16_exponent(float(S[I, J]))
            out[(I, J)] = (np.array([oracle.fp16_scaled(float(x), e)
                                     for x in blk.ravel()]).reshape(blk.shape), e)
    return out


def check(gpu, A, leaf, fmt, blocks=None):
    import torch
    n = A.shape[0]
    d, np_ = oracle.depth(n, leaf)
    N = 1 << d
    P = np.zeros((np_, np_), dtype=np.float32)
    P[:n, :n] = A
    S = oracle.norms(A, leaf)[-1]
    if blocks is None:
        blocks = [(I, J) for I in range(N) for J in range(N)]
    want = expected(P, leaf, fmt, S, blocks)
    t = gpu.build_tree(torch.from_numpy(A).cuda(), leaf, bf16=fmt == "bf16", fp16=fmt == "fp16")
    stats = {"flushed": 0, "ties": 0}
    for copy in (0, 1):
        h, scale = t.matrix16(copy)
        assert h.shape == (np_, np_)
        for (I, J) in blocks:
            vals, e = want[(I, J)]
            hb = h[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf]
            if fmt == "bf16":
                got = bits_to_bf16(hb)
            else:
                assert int(scale[I, J]) == e, (copy, I, J, int(scale[I, J]), e)
                got = bits_to_fp16(hb) * 2.0 ** -e
            bad = np.argwhere(got != vals)
            assert bad.size == 0, (fmt, copy, I, J, bad[:4].tolist(),
                                   [(float(P[I * leaf + r, J * leaf + c]), got[r, c], vals[r, c])
                                    for r, c in bad[:4]])
            if copy == 0:
                x = P[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf].astype(np.float64)
                stats["flushed"] += int(np.count_nonzero((vals == 0) & (x != 0)))
                stats["ties"] += int(np.count_nonzero(vals != x))
    t.free()
    return stats


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("n,leaf,seed", [(320, 32, 1), (333, 32, 2), (256, 64, 3), (300, 64, 4)])
def test_low_copies_bit_exact(gpu, fmt, n, leaf, seed):
    st = check(gpu, planted(n, leaf, seed), leaf, fmt)
    assert st["ties"] > 0                      # some elements were rounded
    if fmt == "fp16":
        assert st["flushed"] > 0               # and some flushed


def test_low_copies_sampled_at_larger_n(gpu):
    """n = 4133 (ragged against 64), cluster-like decay, sampled leaves:
    diagonal, off-diagonal, far corner and padded edge."""
    A = workloads.exp_decay(4133, 0.02, 7)
    N = 128
    rng = np.random.default_rng(11)
    blocks = {(0, 0), (64, 64), (N - 1, N - 1), (0, N - 1), (N - 1, 0), (64, 65), (100, 30)}
    blocks |= {(int(a), int(b)) for a, b in rng.integers(0, N, (12, 2))}
    for fmt in ("bf16", "fp16"):
        check(gpu, A, 64, fmt, sorted(blocks))


def test_matrix16_rejects_trees_without_16bit_copies(gpu):
    import torch
    A = torch.from_numpy(workloads.exp_decay(100, 0.1, 0)).cuda()
    t = gpu.build_tree(A, 32)
    with pytest.raises(gpu.SpammError) as ei:
        t.matrix16(0)
    assert ei.value.code == gpu.SPAMM_E_INVAL
    t.free()
