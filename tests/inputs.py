"""Structured test inputs beyond the seeded workloads: matrices shaped to
reach a code path's limits (no multiply arithmetic here)."""
import numpy as np


def arrow(n, w, seed):
    """Symmetric n x n matrix whose first w rows and columns alone are
    non-zero: uniform noise decaying along the strip, every other group of
    32 strip rows scaled by 1e-4 (so 32 x 32 sub-products inside kept
    64 x 64 leaf products fail the test).  Every output block in the first
    block row and column then takes k over the whole order."""
    rng = np.random.default_rng(seed)
    A = np.empty((n, n), dtype=np.float32)
    A.fill(0.0)                     # touched in row order (faster than zero pages)
    rows = np.where((np.arange(w) // 32) % 2 == 0, 1.0, 1e-4)[:, None]
    strip = (rng.uniform(-1, 1, (w, n)) * np.exp(-np.arange(n) / 3000.0) * rows).astype(np.float32)
    A[:w, :] = strip
    A[:, :w] = strip.T
    corner = strip[:, :w]
    A[:w, :w] = np.triu(corner) + np.triu(corner, 1).T
    return A


def sum_order(b):
    """2b x 2b matrix whose squared leaf norms depend on the summation order:
    leaf (0, 0) holds 1 at (0, 0) and 2^-27 at (1, 0..3) (row-major pairwise
    gives 1 + 2^-52, column-major or sequential orders give 1); leaves (1, 0)
    and (1, 1) hold two entries 2^-27 each (squared norm 2^-53), leaf (0, 1)
    is zero."""
    A = np.zeros((2 * b, 2 * b), dtype=np.float32)
    e = np.float32(2.0 ** -27)
    A[0, 0] = 1.0
    A[1, 0:4] = e
    A[b, 0:2] = e
    A[b + 5, b + 4:b + 6] = e
    return A
