"""SpAMM reference oracle -- test infrastructure only.

A plain FP64 CPU implementation of the sparse approximate matrix multiply,
written from the paper (quadtree depth/padding, Sec. II.A; node norms, product
recursion and SpAMM condition, Sec. II.B; linear index, Sec. III.D.1).  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it; the
GPU library never does, and the two share no code.

The arithmetic lives in ``spamm_oracle.c`` (plain C, -O2, no fast-math,
no FP contraction); this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spamm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OR_OK, OR_EINVAL, OR_ERANGE, OR_ENOMEM = 0, -1, -2, -3


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32, i64, u64, dbl, vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_double, ctypes.c_void_p)
        lib.oracle_depth.argtypes = [i64, i32, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        lib.oracle_depth.restype = ctypes.c_int
        lib.oracle_linear_index.argtypes = [u64, u64]
        lib.oracle_linear_index.restype = u64
        lib.oracle_norms_len.argtypes = [i32]
        lib.oracle_norms_len.restype = i64
        lib.oracle_norms.argtypes = [vp, i64, i32, vp]
        lib.oracle_norms.restype = ctypes.c_int
        lib.oracle_spamm.argtypes = [vp, vp, i64, i32, dbl, vp, vp, i64, vp, vp]
        lib.oracle_spamm.restype = ctypes.c_int
        lib.oracle_spamm_tiles.argtypes = [vp, vp, i64, i32, dbl, vp, i64, vp, vp, vp,
                                           ctypes.c_int]
        lib.oracle_spamm_tiles.restype = ctypes.c_int
        lib.oracle_spamm_split.argtypes = [vp, vp, i64, i32, dbl, dbl, vp, vp, i64, vp, vp, vp]
        lib.oracle_spamm_split.restype = ctypes.c_int
        lib.oracle_spamm_tiles_split.argtypes = [vp, vp, i64, i32, dbl, dbl, vp, i64, vp, vp, vp,
                                                 ctypes.c_int]
        lib.oracle_spamm_tiles_split.restype = ctypes.c_int
        lib.oracle_bf16.argtypes = [ctypes.c_float]
        lib.oracle_bf16.restype = dbl
        lib.oracle_spamm_split_fmt.argtypes = [vp, vp, i64, i32, dbl, dbl, ctypes.c_int, vp, vp,
                                               i64, vp, vp, vp]
        lib.oracle_spamm_split_fmt.restype = ctypes.c_int
        lib.oracle_spamm_tiles_split_fmt.argtypes = [vp, vp, i64, i32, dbl, dbl, ctypes.c_int, vp,
                                                     i64, vp, vp, vp, ctypes.c_int]
        lib.oracle_spamm_tiles_split_fmt.restype = ctypes.c_int
        lib.oracle_spamm_split_rel.argtypes = [vp, vp, i64, i32, dbl, dbl, ctypes.c_int, vp, vp,
                                               i64, vp, vp, vp]
        lib.oracle_spamm_split_rel.restype = ctypes.c_int
        lib.oracle_spamm_tiles_split_rel.argtypes = [vp, vp, i64, i32, dbl, dbl, ctypes.c_int, vp,
                                                     i64, vp, vp, vp, ctypes.c_int]
        lib.oracle_spamm_tiles_split_rel.restype = ctypes.c_int
        lib.oracle_bf16_parts.argtypes = [ctypes.c_float, ctypes.POINTER(dbl),
                                          ctypes.POINTER(dbl)]
        lib.oracle_bf16_parts.restype = None
        lib.oracle_fp16_exponent.argtypes = [dbl]
        lib.oracle_fp16_exponent.restype = ctypes.c_int
        lib.oracle_fp16_scaled.argtypes = [ctypes.c_float, ctypes.c_int]
        lib.oracle_fp16_scaled.restype = dbl
        _lib = lib
    return _lib


def _f32(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A)
    if A.dtype != np.float32 or A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square float32 matrix")
    return A


def depth(n: int, b: int):
    """(d, n_p): quadtree depth and padded size."""
    d = ctypes.c_int32()
    np_ = ctypes.c_int64()
    rc = _load().oracle_depth(n, b, ctypes.byref(d), ctypes.byref(np_))
    if rc:
        raise ValueError(f"oracle_depth({n}, {b}) -> {rc}")
    return d.value, np_.value


def linear_index(i: int, j: int) -> int:
    return int(_load().oracle_linear_index(i, j))


def norms(A: np.ndarray, b: int):
    """Squared Frobenius norms of all tiers: list, tier 0 (root) first, tier t
    as a 2^t x 2^t row-major float64 array."""
    A = _f32(A)
    n = A.shape[0]
    d, _ = depth(n, b)
    out = np.empty(int(_load().oracle_norms_len(d)), dtype=np.float64)
    rc = _load().oracle_norms(A.ctypes.data, n, b, out.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_norms -> {rc}")
    tiers, off = [], 0
    for t in range(d + 1):
        m = 1 << t
        tiers.append(out[off:off + m * m].reshape(m, m))
        off += m * m
    return tiers


LOW_BIT = np.uint64(1) << np.uint64(63)


def bf16(x: float) -> float:
    """x (a float32) rounded to the nearest bfloat16, ties to even."""
    return float(_load().oracle_bf16(x))


def bf16_parts(x: float):
    """(hi, lo) of x (a float32): hi = bf16(x), lo = bf16(x - hi)."""
    hi, lo = ctypes.c_double(), ctypes.c_double()
    _load().oracle_bf16_parts(ctypes.c_float(x), ctypes.byref(hi), ctypes.byref(lo))
    return hi.value, lo.value


def fp16_exponent(S: float) -> int:
    """Scale exponent e of a leaf with squared norm S for binary16 LOW
    operands: every entry of the leaf has |x| 2^e < 2^14 (0 when S = 0)."""
    return int(_load().oracle_fp16_exponent(float(S)))


def fp16_scaled(x: float, e: int) -> float:
    """x (a float32) times 2^e rounded to the nearest binary16 (ties to even),
    zero when that falls below binary16's normal range (2^-14), times 2^-e."""
    return float(_load().oracle_fp16_scaled(x, int(e)))


# LOW operand format; "bf16x3": bfloat16 LOW operands and compensated HIGH
# products (hi_a hi_b + hi_a lo_b + lo_a hi_b of the two bfloat16 parts)
LOW_FMT = {"bf16": 0, "fp16": 1, "bf16x3": 2}


class Result:
    def __init__(self, C, keys, Kt, Klow=0):
        self.C = C          # float64 n x n (or None)
        self.keys = keys    # sorted uint64 (linear_index(I,J) << 32) | K, bit 63 = LOW
        self.Kt = Kt        # kept node triples per tier
        self.Klow = Klow    # kept leaf products classed LOW (split precision)

    @property
    def K(self) -> int:
        return int(self.Kt[-1])


def _split_args(low_tol: float, low_rel: float):
    """(entry point suffix, threshold argument) of a split product: an
    absolute low_tol or a relative low_rel (theta), not both."""
    if low_rel and low_tol:
        raise ValueError("give low_tol or low_rel, not both")
    return ("rel", float(low_rel)) if low_rel else ("fmt", float(low_tol))


def spamm(A: np.ndarray, B: np.ndarray, b: int, tau: float, want_C: bool = True,
          want_keys: bool = True, cap: int | None = None, low_tol: float = 0.0,
          low_fmt: str = "bf16", low_rel: float = 0.0) -> Result:
    """Full recursive SpAMM product in FP64; low_tol > 0 (absolute: LOW iff
    the norm product is below low_tol) or low_rel > 0 (relative: below
    low_rel ||A||_F ||B||_F) selects split precision (LOW products on
    operands rounded to bfloat16, or with low_fmt="fp16" to binary16 at each
    leaf's power-of-two scale; low_fmt="bf16x3" also takes every HIGH
    product from the two bfloat16 parts of its operands, dropping lo lo)."""
    fmt = LOW_FMT[low_fmt]
    kind, thr = _split_args(low_tol, low_rel)
    fn = getattr(_load(), f"oracle_spamm_split_{kind}")
    A, B = _f32(A), _f32(B)
    n = A.shape[0]
    if B.shape[0] != n:
        raise ValueError("shape mismatch")
    d, _ = depth(n, b)
    C = np.empty((n, n), dtype=np.float64) if want_C else None
    Kt = np.zeros(d + 1, dtype=np.int64)
    nk = np.zeros(1, dtype=np.int64)
    kl = np.zeros(1, dtype=np.int64)
    keys = None
    if want_keys:
        if cap is None:
            # count first so the key buffer is exactly sized
            rc = fn(A.ctypes.data, B.ctypes.data, n, b, float(tau), thr, fmt, None, None, 0,
                    nk.ctypes.data, Kt.ctypes.data, kl.ctypes.data)
            if rc:
                raise RuntimeError(f"oracle_spamm -> {rc}")
            cap = int(nk[0])
        keys = np.empty(max(cap, 1), dtype=np.uint64)
    rc = fn(A.ctypes.data, B.ctypes.data, n, b, float(tau), thr, fmt,
            None if C is None else C.ctypes.data, None if keys is None else keys.ctypes.data,
            0 if keys is None else cap, nk.ctypes.data, Kt.ctypes.data, kl.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_spamm -> {rc}")
    if keys is not None:
        keys = keys[:int(nk[0])]
    return Result(C, keys, Kt, int(kl[0]))


def spamm_tiles(A: np.ndarray, B: np.ndarray, b: int, tau: float, tiles,
                threads: int = 1, want_klists: bool = False, low_tol: float = 0.0,
                low_fmt: str = "bf16", low_rel: float = 0.0):
    """Per-tile recursion for the output tiles ``tiles`` ((I, J) pairs).

    Returns (Ctiles [ntiles, b, b] float64, counts [ntiles], klists or None);
    klists[s, :counts[s]] are the kept K values of tile s in ascending order,
    with 1 << 30 added for a LOW product (split precision, low_tol > 0 or
    low_rel > 0 as for spamm; the roots are those of the whole operands).
    """
    kind, thr = _split_args(low_tol, low_rel)
    fn = getattr(_load(), f"oracle_spamm_tiles_split_{kind}")
    A, B = _f32(A), _f32(B)
    n = A.shape[0]
    d, _ = depth(n, b)
    t = np.ascontiguousarray(np.asarray(tiles, dtype=np.int64).reshape(-1, 2))
    m = t.shape[0]
    Ct = np.empty((m, b, b), dtype=np.float64)
    counts = np.zeros(m, dtype=np.int64)
    kl = np.empty((m, 1 << d), dtype=np.int32) if want_klists else None
    rc = fn(A.ctypes.data, B.ctypes.data, n, b, float(tau), thr, LOW_FMT[low_fmt], t.ctypes.data,
            m, Ct.ctypes.data, counts.ctypes.data, None if kl is None else kl.ctypes.data,
            int(threads))
    if rc:
        raise RuntimeError(f"oracle_spamm_tiles -> {rc}")
    return Ct, counts, kl


def sparsify(A: np.ndarray, b: int, tau: float, norm2_other: float = 0.0):
    """Epsilon-sparsification of Sec. II.C (Eq. epsilon), at leaf granularity.

    epsilon = tau / max(||A||_F, ||B||_F): a leaf is dropped (zeroed) when its
    squared norm s is 0 or when s * m < tau^2 with m = max(||A||_F^2,
    norm2_other), all in FP64 on the stored squared norms (the root is that
    of A's full pyramid).  Returns (A with the dropped leaves zeroed, FP32,
    same shape; boolean N x N mask of kept leaves).
    """
    A = _f32(A)
    s = norms(A, b)
    leaf = s[-1]
    m = max(float(s[0][0, 0]), float(norm2_other))
    keep = (leaf > 0.0) & ~(leaf * m < tau * tau)
    n = A.shape[0]
    out = A.copy()
    for I, J in zip(*np.nonzero(~keep)):
        out[I * b:min((I + 1) * b, n), J * b:min((J + 1) * b, n)] = 0.0
    return out, keep
