"""Seeded synthetic inputs for SpAMM, shared by the CPU reference and the GPU path.

This module only draws input matrices; it holds none of the multiply's
arithmetic.  The element generator is a small C library (``gen.c``) so that
the 32750 x 32750 cluster matrix takes seconds, not minutes.

Workloads (the paper's test matrices were Hilbert-ordered water-cluster density
matrices from quantum chemistry, which are not available; these synthetic
matrices have the same structure: decay with distance, clustered by a
space-filling-curve ordering, symmetric, and squared as in purification):

* ``exp_decay``:  a_ij = u_ij * exp(-rate*|i-j|)           (exponential decay)
* ``alg_decay``:  a_ij = u_ij / (|i-j|^power + 1)           (algebraic decay)
* ``molecular_cluster``: molecules uniform in a cube, ordered along a 3-D
  Hilbert curve, ``funcs`` basis functions per molecule at its centre,
  a_ij = u_ij * exp(-rate * r_ij) with r_ij the centre distance.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libspgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, u64, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        fp = ctypes.c_void_p
        lib.spgen_splitmix64_at.argtypes = [u64, u64]
        lib.spgen_splitmix64_at.restype = u64
        lib.spgen_sym_u.argtypes = [u64, i64, i64]
        lib.spgen_sym_u.restype = dbl
        lib.spgen_exp_decay.argtypes = [fp, i64, i64, i64, dbl, u64]
        lib.spgen_alg_decay.argtypes = [fp, i64, i64, i64, dbl, u64]
        lib.spgen_group_decay.argtypes = [fp, i64, i64, i64, fp, fp, i64, u64]
        for f in (lib.spgen_exp_decay, lib.spgen_alg_decay, lib.spgen_group_decay):
            f.restype = None
        _lib = lib
    return _lib


def splitmix64_at(seed: int, idx: int) -> int:
    return int(_load().spgen_splitmix64_at(seed, idx))


def sym_u(seed: int, i: int, j: int) -> float:
    return float(_load().spgen_sym_u(seed, i, j))


def exp_decay(n: int, rate: float, seed: int = 0) -> np.ndarray:
    out = np.empty((n, n), dtype=np.float32)
    _load().spgen_exp_decay(out.ctypes.data, n, 0, n, float(rate), seed)
    return out


def alg_decay(n: int, power: float, seed: int = 0) -> np.ndarray:
    out = np.empty((n, n), dtype=np.float32)
    _load().spgen_alg_decay(out.ctypes.data, n, 0, n, float(power), seed)
    return out


# ---------------------------------------------------------------------------
# 3-D Hilbert ordering (J. Skilling, "Programming the Hilbert curve",
# AIP Conf. Proc. 707, 381 (2004)): axes -> transposed Hilbert index.
# ---------------------------------------------------------------------------
def hilbert_keys(coords: np.ndarray, bits: int) -> np.ndarray:
    """Hilbert index of integer points ``coords`` (m x dims, each < 2**bits)."""
    X = np.array(coords, dtype=np.int64, copy=True)
    m, dims = X.shape
    top = 1 << (bits - 1)
    # Inverse undo of the excess work.
    Q = top
    while Q > 1:
        P = Q - 1
        for i in range(dims):
            hit = (X[:, i] & Q) != 0
            # invert low bits of X0 where bit Q of Xi is set
            X[hit, 0] ^= P
            # otherwise exchange low bits of X0 and Xi
            miss = ~hit
            t = (X[miss, 0] ^ X[miss, i]) & P
            X[miss, 0] ^= t
            X[miss, i] ^= t
        Q >>= 1
    # Gray encode.
    for i in range(1, dims):
        X[:, i] ^= X[:, i - 1]
    t = np.zeros(m, dtype=np.int64)
    Q = top
    while Q > 1:
        hit = (X[:, dims - 1] & Q) != 0
        t[hit] ^= Q - 1
        Q >>= 1
    X ^= t[:, None]
    # Interleave the transposed bits, most significant first.
    key = np.zeros(m, dtype=np.int64)
    for b in range(bits - 1, -1, -1):
        for i in range(dims):
            key = (key << 1) | ((X[:, i] >> b) & 1)
    return key


@dataclass
class Cluster:
    positions: np.ndarray      # molecule centres in Hilbert order (n_mol x 3), Angstrom
    box: float                 # cube side, Angstrom
    order: np.ndarray          # permutation applied to the drawn molecules
    funcs: int                 # basis functions per molecule


def cluster_geometry(n_mol: int, density: float, seed: int = 0, funcs: int = 25,
                     bits: int = 10) -> Cluster:
    """Molecule centres uniform in a cube of the given number density, ordered
    along a 3-D Hilbert curve (coordinates quantised to ``bits`` per axis,
    stable sort, ties by drawing order)."""
    box = (n_mol / density) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(n_mol, 3))
    q = np.floor((1 << bits) * pos / box).astype(np.int64)
    q = np.clip(q, 0, (1 << bits) - 1)
    order = np.argsort(hilbert_keys(q, bits), kind="stable")
    return Cluster(positions=pos[order], box=box, order=order, funcs=funcs)


def molecular_cluster(n_mol: int, density: float = 0.0334, rate: float = 0.6,
                      seed: int = 0, funcs: int = 25) -> np.ndarray:
    geo = cluster_geometry(n_mol, density, seed, funcs)
    diff = geo.positions[:, None, :] - geo.positions[None, :, :]
    r = np.sqrt(np.sum(diff * diff, axis=-1))
    env = np.ascontiguousarray(np.exp(-rate * r), dtype=np.float64)
    n = n_mol * funcs
    group = (np.arange(n, dtype=np.int64) // funcs).astype(np.int32)
    out = np.empty((n, n), dtype=np.float32)
    _load().spgen_group_decay(out.ctypes.data, n, 0, n, group.ctypes.data,
                              env.ctypes.data, n_mol, seed)
    return out


# ---------------------------------------------------------------------------
# Named workloads.  A = B in every case (the matrix square).
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    n: int
    leaf: int
    taus: tuple
    kind: str
    params: dict = field(default_factory=dict)

    @property
    def tau(self) -> float:
        return self.taus[0]

    def matrix(self) -> np.ndarray:
        p = self.params
        if self.kind == "exp":
            return exp_decay(self.n, p["rate"], p.get("seed", 0))
        if self.kind == "alg":
            return alg_decay(self.n, p["power"], p.get("seed", 0))
        if self.kind == "cluster":
            return molecular_cluster(p["n_mol"], p["density"], p["rate"],
                                     p.get("seed", 0), p["funcs"])
        raise ValueError(self.kind)


WORKLOADS = {
    # n=1024 exponential decay 0.1, leaf 32 (depth 5), tau=1e-6
    "expdecay-n1024": Workload("expdecay-n1024", 1024, 32, (1e-6,), "exp",
                               {"rate": 0.1, "seed": 0}),
    # 300 molecules x 25 functions, n=7500 (padded to 8192), leaf 32, tau=1e-8
    "cluster300-n7500": Workload("cluster300-n7500", 7500, 32, (1e-8,), "cluster",
                                 {"n_mol": 300, "density": 0.0334, "rate": 0.6,
                                  "funcs": 25, "seed": 0}),
    # algebraic decay |i-j|^3, n=16384, leaf 64, tau sweep
    "algdecay-n16384": Workload("algdecay-n16384", 16384, 64,
                                (1e-4, 1e-6, 1e-8, 1e-10), "alg",
                                {"power": 3.0, "seed": 0}),
    # 1310 molecules x 25 functions, n=32750 (padded to 32768), leaf 64, tau=1e-8
    "cluster1310-n32750": Workload("cluster1310-n32750", 32750, 64, (1e-8,), "cluster",
                                   {"n_mol": 1310, "density": 0.0334, "rate": 0.6,
                                    "funcs": 25, "seed": 0}),
}


# ---------------------------------------------------------------------------
# Serving mix: a stream of products and squaring chains of uneven size.
# ---------------------------------------------------------------------------
@dataclass
class ServeRequest:
    index: int
    n: int            # order, uniform over SERVE_SIZES
    rate: float       # exponential decay rate, U(0.05, 0.5)
    tau: float        # 1e-6 or 1e-8
    chain_len: int    # 0 (one product C = A A) or 10 squarings X <- X X
    split: bool       # split-BF16 precision (else FP32)
    seed: int         # matrix seed, 1000 + index
    gap: float        # unit-rate exponential inter-arrival gap (scaled by 1 / QPS)


SERVE_SIZES = (512, 1024, 2048, 4096, 8192)
SERVE_LEAF = 32
SERVE_THETA = 1e-4    # split: LOW iff norm product < theta ||A||_F ||B||_F


def serving_mix(count: int = 2000, seed: int = 0, chain_share: float = 0.3,
                split_share: float = 0.5) -> list:
    """Request parameters drawn from one master seed: n uniform over
    SERVE_SIZES, decay rate U(0.05, 0.5), tau in {1e-6, 1e-8}, a share of
    10-step squaring chains, a share in split precision, Poisson arrivals
    (unit-rate exponential gaps).  Request r's matrix uses seed 1000 + r."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.array(SERVE_SIZES), size=count)
    rate = rng.uniform(0.05, 0.5, size=count)
    tau = rng.choice(np.array([1e-6, 1e-8]), size=count)
    chain = rng.random(count) < chain_share
    split = rng.random(count) < split_share
    gap = rng.exponential(1.0, size=count)
    return [ServeRequest(r, int(n[r]), float(rate[r]), float(tau[r]), 10 if chain[r] else 0,
                         bool(split[r]), 1000 + r, float(gap[r])) for r in range(count)]


def spectral_radius(torch, A, iters: int = 64, seed: int = 0) -> float:
    """Largest |eigenvalue| of a symmetric matrix A (a torch tensor on any
    device) by Lanczos with full reorthogonalization: `iters` FP32
    matrix-vector products, the Krylov basis in FP64, the extreme Ritz values
    from the small tridiagonal matrix.  Ritz values lie inside the spectrum,
    so the estimate is a lower bound that converges quickly even when the top
    eigenvalues are clustered (where power iteration stalls)."""
    n = A.shape[0]
    k = min(iters, n)
    g = torch.Generator(device=A.device)
    g.manual_seed(seed)
    Q = torch.zeros((k + 1, n), dtype=torch.float64, device=A.device)
    q = torch.rand(n, generator=g, device=A.device, dtype=torch.float64) - 0.5
    Q[0] = q / q.norm()
    alpha = torch.zeros(k, dtype=torch.float64, device=A.device)
    beta = torch.zeros(k, dtype=torch.float64, device=A.device)
    for j in range(k):
        w = (A @ Q[j].to(A.dtype)).to(torch.float64)
        alpha[j] = Q[j] @ w
        # full reorthogonalization against the basis so far (twice is enough)
        for _ in range(2):
            w = w - Q[:j + 1].T @ (Q[:j + 1] @ w)
        beta[j] = w.norm()
        Q[j + 1] = w / beta[j].clamp_min(1e-300)
    a = alpha.cpu().numpy()
    b = beta.cpu().numpy()
    m = k
    small = np.nonzero(b[:k - 1] <= 1e-12 * max(1.0, float(np.abs(a).max())))[0]
    if len(small):
        m = int(small[0]) + 1             # an invariant subspace was found
    T = np.diag(a[:m]) + np.diag(b[:m - 1], 1) + np.diag(b[:m - 1], -1)
    return float(np.abs(np.linalg.eigvalsh(T)).max())


def serve_matrix(torch, req: ServeRequest, device):
    """Request r's input on `device`: symmetric u ~ U(-1, 1) from a torch
    generator seeded req.seed, times exp(-rate |i - j|).  A squaring chain
    starts from X_0 = A / rho(A) (spectral radius by Lanczos), so its
    eigenvalues lie in [-1, 1] and the ones near +-1 survive every squaring:
    the powers neither vanish nor overflow, as in density-matrix purification,
    where the spectrum is mapped into [0, 1] before squaring."""
    g = torch.Generator(device=device)
    g.manual_seed(req.seed)
    n = req.n
    u = torch.rand((n, n), generator=g, device=device, dtype=torch.float32).mul_(2.0).sub_(1.0)
    A = torch.triu(u)
    A += torch.triu(u, 1).T
    del u
    i = torch.arange(n, device=device, dtype=torch.float32)
    A *= torch.exp((i[:, None] - i[None, :]).abs_().mul_(-req.rate))
    if req.chain_len:
        A /= spectral_radius(torch, A, seed=req.seed)
    return A
