"""MI355X-native SpAMM: quadtree norm build, tier-by-tier cull and an
FP32-MFMA leaf GEMM (one workgroup per block of output leaves; split
precision with BF16 LOW products and FP32 or compensated-BF16 HIGH ones, or
scaled FP16 LOW products; sub-leaf culling) behind the C ABI of
include/spamm.h, plus a continuous-batching server for products and squaring
chains."""
from ._binding import (  # noqa: F401
    HEADER, LIB_PATH, PREC_FP32, PREC_SPLIT_BF16, PREC_SPLIT_BF16X3, PREC_SPLIT_FP16, SPAMM_E_BUSY, SPAMM_E_HIP, SPAMM_E_INVAL,
    SPAMM_E_MISMATCH, SPAMM_E_NOMEM, SPAMM_E_NONFINITE, SPAMM_E_RANGE, SPAMM_OK, SPAMM_PENDING,
    Opts, Plan, Request, TREE_BF16, TREE_FP16, TREE_SUBNORMS, Result, Server, ServerStats, SpammError, Stats, Tree, build_tree, build_tree_output, build_tree_sparse,
    header_functions, load, multiply, multiply_ex, multiply_noalloc, request_footprint, strerror,
    symbolic,
)
