"""Input generators: published RNG vectors, symmetry, decay envelopes and the
Hilbert ordering.  These hold no multiply arithmetic; both sides consume the
same FP32 bytes."""
import itertools
import json
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.json")) as f:
        g = json.load(f)
    got = [workloads.splitmix64_at(g["seed"], i) for i in range(5)]
    assert got == [int(x) for x in g["outputs"]]


def test_sym_u_range_and_symmetry():
    vals = [workloads.sym_u(7, i, j) for i in range(40) for j in range(40)]
    assert min(vals) >= -1.0 and max(vals) < 1.0
    for i in range(40):
        for j in range(40):
            assert workloads.sym_u(7, i, j) == workloads.sym_u(7, j, i)
    assert abs(np.mean(vals)) < 0.1 and 0.25 < np.var(vals) < 0.42


def test_exp_decay_envelope_and_symmetry():
    n, rate = 300, 0.1
    A = workloads.exp_decay(n, rate, seed=0)
    assert A.dtype == np.float32 and np.array_equal(A, A.T)
    i = np.arange(n)
    env = np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    assert np.all(np.abs(A.astype(np.float64)) <= env * (1 + 2.0 ** -23) + 2.0 ** -149)
    # element (i,j) is u(i,j) * envelope rounded once to FP32
    for (r, c) in [(0, 0), (3, 17), (250, 1)]:
        want = np.float32(workloads.sym_u(0, r, c) * np.exp(-rate * abs(r - c)))
        assert A[r, c] == want
    # far entries of n=1024, rate 0.1 are FP32 denormals
    B = workloads.exp_decay(1024, 0.1, seed=0)
    far = np.abs(B[0, 900:])
    assert np.any((far > 0) & (far < np.finfo(np.float32).tiny))
    assert np.array_equal(B, workloads.exp_decay(1024, 0.1, seed=0))
    assert not np.array_equal(B, workloads.exp_decay(1024, 0.1, seed=1))


def test_alg_decay_envelope():
    n = 200
    A = workloads.alg_decay(n, 3.0, seed=0)
    i = np.arange(n)
    env = 1.0 / (np.abs(i[:, None] - i[None, :]).astype(np.float64) ** 3 + 1.0)
    assert np.array_equal(A, A.T)
    assert np.all(np.abs(A.astype(np.float64)) <= env * (1 + 2.0 ** -23))


@pytest.mark.parametrize("dims,bits", [(2, 3), (3, 2), (3, 3)])
def test_hilbert_order_is_a_continuous_curve(dims, bits):
    pts = np.array(list(itertools.product(range(1 << bits), repeat=dims)))
    keys = workloads.hilbert_keys(pts, bits)
    assert np.array_equal(np.sort(keys), np.arange(len(pts)))
    walk = pts[np.argsort(keys)]
    steps = np.abs(np.diff(walk, axis=0)).sum(axis=1)
    assert np.all(steps == 1)        # consecutive cells are face neighbours


def test_cluster_geometry():
    geo = workloads.cluster_geometry(300, 0.0334, seed=0)
    assert geo.box == pytest.approx((300 / 0.0334) ** (1 / 3))
    assert geo.box == pytest.approx(20.79, abs=0.01)
    assert np.all((geo.positions >= 0) & (geo.positions < geo.box))
    q = np.clip(np.floor(1024 * geo.positions / geo.box).astype(np.int64), 0, 1023)
    assert np.all(np.diff(workloads.hilbert_keys(q, 10)) >= 0)
    assert sorted(geo.order.tolist()) == list(range(300))


def test_cluster_matrix_structure():
    A = workloads.molecular_cluster(20, 0.0334, 0.6, seed=3, funcs=5)
    assert A.shape == (100, 100) and np.array_equal(A, A.T)
    geo = workloads.cluster_geometry(20, 0.0334, seed=3, funcs=5)
    p = geo.positions
    for (i, j) in [(0, 1), (0, 7), (13, 99), (50, 51)]:
        r = np.linalg.norm(p[i // 5] - p[j // 5])
        assert A[i, j] == np.float32(workloads.sym_u(3, i, j) * np.exp(-0.6 * r))


def test_spectral_radius_against_eigvalsh():
    """Lanczos estimate of the serving chains' normalisation against LAPACK's
    symmetric eigenvalues (slow and fast decay, and a matrix whose largest
    |eigenvalue| is negative)."""
    import torch
    for n, rate, seed in ((300, 0.05, 1), (700, 0.5, 2), (512, 0.2, 3)):
        req = workloads.ServeRequest(0, n, rate, 1e-6, 0, False, seed, 1.0)
        A = workloads.serve_matrix(torch, req, "cpu")
        rho = float(np.abs(np.linalg.eigvalsh(A.double().numpy())).max())
        assert abs(workloads.spectral_radius(torch, A, seed=seed) - rho) <= 1e-6 * rho
    D = torch.diag(torch.tensor([-3.0, 1.0, 2.0, -0.5]))
    assert abs(workloads.spectral_radius(torch, D) - 3.0) <= 3e-6     # FP32 products


@pytest.mark.parametrize("n,rate,tau", [(512, 0.05, 1e-6), (512, 0.5, 1e-8), (512, 0.5, 1e-6),
                                        (1024, 0.3, 1e-6)])
def test_serving_chains_keep_products_every_step(n, rate, tau):
    """A 10-step squaring chain of the serving mix, run through the oracle,
    keeps leaf products at every step and stays bounded: X_0 = A / rho(A)
    leaves the top eigenvalues at +-1, so the squarings neither vanish nor
    overflow."""
    import torch
    import oracle
    req = workloads.ServeRequest(0, n, rate, tau, 10, False, 1000 + n, 1.0)
    X = workloads.serve_matrix(torch, req, "cpu").numpy()
    kept = []
    for _ in range(req.chain_len):
        ref = oracle.spamm(X, X, workloads.SERVE_LEAF, tau, want_keys=False)
        kept.append(ref.K)
        X = ref.C.astype(np.float32)
    assert min(kept) > 0, kept
    # the top of the spectrum is still near 1 after 2^10-th powers
    assert 0.5 < float(np.abs(np.linalg.eigvalsh(X.astype(np.float64))).max()) < 2.0
