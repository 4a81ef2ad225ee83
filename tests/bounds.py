"""Elementwise rounding bounds of a GPU product around the oracle's FP64
product on the same task set (Higham's dot-product bound).

For output element (p, q) of leaf (I, J) with K_IJ kept products,
|C_gpu - C_oracle| <= gamma_m * sum_kept |X_ik| |Y_kj| + m 2^-126 s,
gamma_m = m u / (1 - m u), u = 2^-24 (FP32 accumulation), where X, Y are the
operands each product was taken on (FP32 for HIGH products, the rounded
16-bit values for LOW ones) and m = n_b K_IJ + 1 (FP32 and BF16 products) or
(n_b + 1) K_IJ + 1 (FP16 LOW products are summed on their own and added, one
more rounding each).  With compensated HIGH products (low_fmt "bf16x3") a
HIGH product adds three exact terms per k, hi_a hi_b, hi_a lo_b and
lo_a hi_b, bounded together by (|hi_a| + |lo_a|)(|hi_b| + |lo_b|), and
m = 3 n_b K_IJ + 1.  s = max(1, max|X|, max|Y|)^2 covers flushed denormal
products.
"""
import numpy as np

import oracle

U32 = 2.0 ** -24


def padded(A, leaf):
    d, np_ = oracle.depth(A.shape[0], leaf)
    P = np.zeros((np_, np_), dtype=np.float32)
    P[:A.shape[0], :A.shape[0]] = A
    return P, d


def bf16_round(P):
    import torch
    return torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32)).to(torch.bfloat16).to(
        torch.float64).numpy()


def fp16_leaves(P, leaf, S):
    """P (padded FP32) with every leaf rounded through numpy float16 at the
    scale exponent of its squared norm S[I, J] (oracle.fp16_exponent),
    binary16 subnormals flushed to zero."""
    N = P.shape[0] // leaf
    R = np.zeros(P.shape)
    for I in range(N):
        for J in range(N):
            e = oracle.fp16_exponent(S[I, J])
            blk = P[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf].astype(np.float64) * 2.0 ** e
            h = blk.astype(np.float16).astype(np.float64)
            R[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] = \
                np.where(np.abs(h) < 2.0 ** -14, 0.0, h) * 2.0 ** -e
    return R


def class_bound(A, B, leaf, keys, low_fmt="bf16"):
    """Bound on |C_gpu - C_oracle| (n x n) for sorted task keys with their
    class bit (bit 63 = LOW); low_fmt names the LOW operand format."""
    PA, d = padded(A, leaf)
    PB, _ = padded(B, leaf)
    N = 1 << d
    inv = {oracle.linear_index(i, j): (i, j) for i in range(N) for j in range(N)}
    if low_fmt == "bf16x3":
        def parts(P):
            H = bf16_round(P)
            return np.abs(H) + np.abs(bf16_round(P - H.astype(np.float32)))
        ops = {0: (parts(PA), parts(PB))}
    else:
        ops = {0: (np.abs(PA.astype(np.float64)), np.abs(PB.astype(np.float64)))}
    keys = np.asarray(keys, dtype=np.uint64)
    if len(keys) and (keys >> np.uint64(63)).any():
        if low_fmt == "fp16":
            ops[1] = (np.abs(fp16_leaves(PA, leaf, oracle.norms(A, leaf)[-1])),
                      np.abs(fp16_leaves(PB, leaf, oracle.norms(B, leaf)[-1])))
        else:
            ops[1] = (np.abs(bf16_round(PA)), np.abs(bf16_round(PB)))
    M = np.zeros(PA.shape)
    cnt = np.zeros((N, N), dtype=np.int64)
    for key in keys:
        key = int(key)
        I, J = inv[(key >> 32) & 0x7FFFFFFF]
        k = key & 0xFFFFFFFF
        X, Y = ops[key >> 63]
        M[I * leaf:(I + 1) * leaf, J * leaf:(J + 1) * leaf] += (
            X[I * leaf:(I + 1) * leaf, k * leaf:(k + 1) * leaf] @ Y[k * leaf:(k + 1) * leaf,
                                                                  J * leaf:(J + 1) * leaf])
        cnt[I, J] += 1
    per = leaf + 1 if low_fmt == "fp16" else 3 * leaf if low_fmt == "bf16x3" else leaf
    m = per * np.kron(cnt, np.ones((leaf, leaf))) + 1
    gamma = m * U32 / (1 - m * U32)
    scale = max(1.0, float(ops[0][0].max()), float(ops[0][1].max())) ** 2
    n = A.shape[0]
    return (gamma * M + m * 2.0 ** -126 * scale)[:n, :n]
