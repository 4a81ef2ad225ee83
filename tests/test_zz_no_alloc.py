"""spamm_multiply_noalloc, the product for callers that cannot allocate device
memory: its task arena lives in the library's fixed per-device block.  It
runs the cull and leaf GEMM of spamm_multiply_opts on the same trees, so C
must equal that entry point's C bit for bit.

* two calls in a row on one stream, the second on a smaller input, each
  against spamm_multiply_opts (the block keeps the first call's contents);
* FP32, BF16 and FP16 split (relative threshold), sub-leaf culling, two
  distinct operands, a single leaf, nothing kept, and the deepest product the
  block holds (256 leaves per dimension);
* a product too deep for the block is refused with SPAMM_E_RANGE.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def decay(n, rate, seed, sym=True):
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    A = rng.uniform(-1, 1, (n, n)) * np.exp(-rate * np.abs(i[:, None] - i[None, :]))
    if sym:
        A = np.triu(A) + np.triu(A, 1).T
    return A.astype(np.float32)


def trees(gpu, A, B, leaf, prec, sub):
    import torch
    kw = dict(bf16=prec in (gpu.PREC_SPLIT_BF16, gpu.PREC_SPLIT_BF16X3),
              fp16=prec == gpu.PREC_SPLIT_FP16, subnorms=sub)
    dA = torch.from_numpy(A).cuda()
    tA = gpu.build_tree(dA, leaf, **kw)
    tB = tA if B is None else gpu.build_tree(torch.from_numpy(B).cuda(), leaf, **kw)
    return dA, tA, tB


def both(gpu, A, B, leaf, tau, prec=0, rel=0.0, sub=False):
    """(C from spamm_multiply_opts, C from spamm_multiply_noalloc, stats)."""
    import torch
    print(f"[noalloc] n={A.shape[0]} leaf={leaf} tau={tau:g} prec={prec} theta={rel:g} "
          f"sub={sub}", flush=True)
    dA, tA, tB = trees(gpu, A, B, leaf, prec, sub)
    C_ref = torch.full_like(dA, float("nan"))
    C_new = torch.full_like(dA, float("nan"))
    st = gpu.multiply_ex(tA, tB, tau, C_ref, precision=prec, low_rel=rel, sub_cull=sub)
    gpu.multiply_noalloc(tA, tB, tau, C_new, precision=prec, low_rel=rel, sub_cull=sub)
    torch.cuda.synchronize()
    return C_ref, C_new, st


def test_two_calls_in_a_row_second_smaller(gpu):
    import torch
    big, small = decay(2048, 0.05, 1), decay(700, 0.1, 2)
    dB, tBig, _ = trees(gpu, big, None, 32, 0, False)
    dS, tSmall, _ = trees(gpu, small, None, 32, 0, False)
    C_big = torch.full_like(dB, float("nan"))
    C_small = torch.full_like(dS, float("nan"))
    print("[noalloc] n=2048 then n=700, leaf 32, one stream", flush=True)
    gpu.multiply_noalloc(tBig, tBig, 1e-6, C_big)
    gpu.multiply_noalloc(tSmall, tSmall, 1e-6, C_small)
    R_big, R_small = torch.empty_like(dB), torch.empty_like(dS)
    st_big = gpu.multiply_ex(tBig, tBig, 1e-6, R_big)
    st_small = gpu.multiply_ex(tSmall, tSmall, 1e-6, R_small)
    torch.cuda.synchronize()
    assert st_big["tasks"] > st_small["tasks"] > 0
    assert torch.equal(C_big.view(torch.int32), R_big.view(torch.int32))
    assert torch.equal(C_small.view(torch.int32), R_small.view(torch.int32))


CASES = {
    "fp32-b32": lambda g: (workloads.exp_decay(1024, 0.1, 0), None, 32, 1e-6, 0, 0.0, False),
    "bf16-rel": lambda g: (decay(900, 0.03, 3), None, 64, 1e-6, g.PREC_SPLIT_BF16, 1e-3, False),
    "fp16-rel": lambda g: (decay(777, 0.05, 4), None, 32, 1e-7, g.PREC_SPLIT_FP16, 1e-3, False),
    "bf16x3-rel": lambda g: (decay(900, 0.03, 10), None, 64, 1e-6, g.PREC_SPLIT_BF16X3, 1e-3,
                             False),
    "bf16x3-rel-b32": lambda g: (decay(600, 0.05, 11), None, 32, 1e-7, g.PREC_SPLIT_BF16X3, 1e-3,
                                 False),
    "subleaf-b64": lambda g: (decay(1500, 0.02, 5), None, 64, 1e-5, 0, 0.0, True),
    "nonsym-b16": lambda g: (decay(400, 0.05, 6, sym=False), decay(400, 0.08, 7, sym=False), 16,
                             1e-5, 0, 0.0, False),
    "single-leaf": lambda g: (decay(40, 0.1, 8), None, 64, 0.0, 0, 0.0, False),
    "nothing-kept": lambda g: (decay(300, 0.1, 9), None, 32, 1e3, 0, 0.0, False),
    "depth8-b32": lambda g: (workloads.exp_decay(8192, 0.1, 0), None, 32, 1e-6, 0, 0.0, False),
}


@pytest.mark.parametrize("name", list(CASES))
def test_equals_multiply_opts(gpu, name):
    import torch
    A, B, leaf, tau, prec, rel, sub = CASES[name](gpu)
    C_ref, C_new, st = both(gpu, A, B, leaf, tau, prec, rel, sub)
    assert not torch.isnan(C_new).any()
    assert torch.equal(C_new.view(torch.int32), C_ref.view(torch.int32))
    if name == "nothing-kept":
        assert st["tasks"] == 0 and torch.count_nonzero(C_new).item() == 0
    else:
        assert st["tasks"] > 0
    if rel:
        assert 0 < st["tasks_low"] < st["tasks"]


def test_too_deep_for_the_block_is_refused(gpu):
    import torch
    A = torch.zeros(4097, 4097, device="cuda")       # leaf 16: 512 leaves per dimension
    A[0, 0] = 1.0
    t = gpu.build_tree(A, 16)
    assert t.depth == 9
    C = torch.empty_like(A)
    with pytest.raises(gpu.SpammError) as ei:
        gpu.multiply_noalloc(t, t, 0.0, C)
    assert ei.value.code == gpu.SPAMM_E_RANGE
    # the ordinary entry point still takes it
    gpu.multiply_ex(t, t, 0.0, C)
    assert C[0, 0].item() == 1.0
