"""ctypes binding of libspamm.so: argument marshalling only.

Every step of the multiply runs in the library's HIP kernels.  PyTorch only
provides device memory and the current stream; tensors must be float32,
contiguous, square and on the current CUDA (HIP) device.  If the library is
not built the import of a function raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspamm.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "spamm.h")

SPAMM_OK = 0
SPAMM_E_INVAL = -1
SPAMM_E_NONFINITE = -2
SPAMM_E_NOMEM = -3
SPAMM_E_HIP = -4
SPAMM_E_RANGE = -5
SPAMM_E_MISMATCH = -6
SPAMM_E_BUSY = -7
SPAMM_PENDING = 1

PREC_FP32 = 0
PREC_SPLIT_BF16 = 1
PREC_SPLIT_FP16 = 2
PREC_SPLIT_BF16X3 = 3     # BF16 LOW products, compensated (three BF16 products) HIGH ones
TREE_BF16 = 1
TREE_SUBNORMS = 2
TREE_FP16 = 4

_lib = None


class SpammError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {code})")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("precision", ctypes.c_int32),
                ("low_tol", ctypes.c_double), ("sub_cull", ctypes.c_int32),
                ("low_rel", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("depth", ctypes.c_int32),
        ("leaf", ctypes.c_int32),
        ("kept", ctypes.c_int64 * 32),
        ("tasks", ctypes.c_int64),
        ("tasks_low", ctypes.c_int64),
        ("block_entries", ctypes.c_int64),
        ("block_entries_low", ctypes.c_int64),
        ("flops", ctypes.c_double),
        ("symbolic_ms", ctypes.c_double),
        ("numeric_ms", ctypes.c_double),
        ("subtasks", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {
            "depth": self.depth, "leaf": self.leaf,
            "kept": [int(self.kept[t]) for t in range(self.depth + 1)],
            "tasks": int(self.tasks), "tasks_low": int(self.tasks_low),
            "block_entries": int(self.block_entries),
            "block_entries_low": int(self.block_entries_low),
            "flops": float(self.flops), "symbolic_ms": float(self.symbolic_ms),
            "numeric_ms": float(self.numeric_ms),
            "subtasks": int(self.subtasks),
        }


class Request(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("leaf", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("tau", ctypes.c_double), ("low_tol", ctypes.c_double),
                ("chain_len", ctypes.c_int32), ("low_rel", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("tasks", ctypes.c_int64), ("tasks_low", ctypes.c_int64),
                ("flops", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("admitted", "completed", "queued", "launches",
                                              "launched_products", "max_batch", "peak_active")] + \
               [(k, ctypes.c_uint64) for k in ("used", "peak_used", "budget")] + \
               [(k, ctypes.c_double) for k in ("sched_cpu_ms", "sched_wall_ms")] + \
               [(k, ctypes.c_int64) for k in ("rounds", "round_steps")]

    def as_dict(self) -> dict:
        return {k: (float(getattr(self, k)) if k.endswith("_ms") else int(getattr(self, k)))
                for k, _ in self._fields_}


def header_functions() -> list:
    """Names of the functions declared in include/spamm.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spamm_[a-z_]+)\s*\(", text)))


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libspamm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_double, ctypes.c_size_t)
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "spamm_build_tree": [vp, i64, i32, vp, pp],
        "spamm_build_tree_ex": [vp, i64, i32, ctypes.c_uint32, vp, pp],
        "spamm_symbolic_ex": [vp, vp, ctypes.POINTER(Opts), vp, pp],
        "spamm_multiply_opts": [vp, vp, ctypes.POINTER(Opts), vp, vp, ctypes.POINTER(Stats)],
        "spamm_tree_free": [vp],
        "spamm_build_tree_sparse": [vp, i64, i32, ctypes.c_uint32, dbl, dbl, vp, pp],
        "spamm_build_tree_output": [vp, vp, ctypes.c_uint32, vp, pp],
        "spamm_tree_storage": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(sz)],
        "spamm_tree_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                            ctypes.POINTER(dbl)],
        "spamm_tree_norms": [vp, i32, vp, sz],
        "spamm_tree_matrix": [vp, i32, vp, sz],
        "spamm_tree_matrix16": [vp, i32, vp, sz, vp, sz],
        "spamm_symbolic": [vp, vp, dbl, vp, pp],
        "spamm_numeric": [vp, vp, vp],
        "spamm_plan_tasks": [vp, vp, sz, ctypes.POINTER(sz)],
        "spamm_plan_subtasks": [vp, vp, sz, ctypes.POINTER(sz)],
        "spamm_plan_stats": [vp, ctypes.POINTER(Stats)],
        "spamm_plan_free": [vp],
        "spamm_multiply": [vp, vp, dbl, vp, vp],
        "spamm_multiply_ex": [vp, vp, dbl, vp, vp, ctypes.POINTER(Stats)],
        "spamm_multiply_noalloc": [vp, vp, ctypes.POINTER(Opts), vp, vp],
        "spamm_server_create": [sz, i32, pp],
        "spamm_request_footprint": [ctypes.POINTER(Request), ctypes.POINTER(sz)],
        "spamm_submit": [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)],
        "spamm_poll": [vp, ctypes.c_uint64, ctypes.POINTER(Result)],
        "spamm_server_info": [vp, ctypes.POINTER(ServerStats)],
        "spamm_server_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.spamm_strerror.argtypes = [ctypes.c_int]
    lib.spamm_strerror.restype = ctypes.c_char_p
    lib.spamm_last_error.argtypes = []
    lib.spamm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != SPAMM_OK:
        lib = load()
        detail = (lib.spamm_last_error() or b"").decode() or lib.spamm_strerror(rc).decode()
        raise SpammError(rc, where, detail)


def strerror(code: int) -> str:
    return load().spamm_strerror(code).decode()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _device_matrix(t, name: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32 or not t.is_cuda or t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be a square float32 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Tree:
    """Quadtree of one operand (packed leaves + FP64 norm pyramid) on the GPU."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        self._plans = 0       # live plans that read this tree
        n, leaf, depth, nrm = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(load().spamm_tree_info(handle, ctypes.byref(n), ctypes.byref(leaf),
                                      ctypes.byref(depth), ctypes.byref(nrm)), "spamm_tree_info")
        self.n, self.leaf, self.depth, self.norm2 = n.value, leaf.value, depth.value, nrm.value

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("tree has been freed")
        return self._h

    @property
    def np(self) -> int:
        return self.leaf << self.depth

    def norms(self, tier: int) -> np.ndarray:
        m = 1 << tier
        out = np.empty((m, m), dtype=np.float64)
        _check(load().spamm_tree_norms(self.handle, tier, out.ctypes.data, out.size),
               "spamm_tree_norms")
        return out

    def matrix(self, copy: int = 0) -> np.ndarray:
        """The padded matrix as held by the tree: copy 0 = left-operand
        leaves, copy 1 = right-operand (transposed) leaves."""
        out = np.empty((self.np, self.np), dtype=np.float32)
        _check(load().spamm_tree_matrix(self.handle, copy, out.ctypes.data, out.size),
               "spamm_tree_matrix")
        return out

    def matrix16(self, copy: int = 0):
        """The 16-bit leaf copies as raw bit patterns (uint16, n_p x n_p) and,
        for FP16 copies, the leaves' scale exponents (int32, N x N; else
        None)."""
        out = np.empty((self.np, self.np), dtype=np.uint16)
        N = self.np // self.leaf
        scale = np.empty((N, N), dtype=np.int32) if getattr(self, "fp16", False) else None
        _check(load().spamm_tree_matrix16(self.handle, copy, out.ctypes.data, out.size,
                                          None if scale is None else scale.ctypes.data,
                                          0 if scale is None else scale.size),
               "spamm_tree_matrix16")
        return out, scale

    def storage(self) -> dict:
        """Leaves stored, leaves in the grid, device bytes held."""
        st, tot, by = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(load().spamm_tree_storage(self.handle, ctypes.byref(st), ctypes.byref(tot),
                                         ctypes.byref(by)), "spamm_tree_storage")
        return {"stored": st.value, "total": tot.value, "bytes": by.value}

    def free(self):
        if self._h is not None:
            if self._plans:
                raise ValueError(f"tree is read by {self._plans} live plan(s); free them first")
            _check(load().spamm_tree_free(self._h), "spamm_tree_free")
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Plan:
    """Kept task list of one product (symbolic multiply result)."""

    def __init__(self, handle, A: Tree, B: Tree):
        self._h = handle
        self._keep = (A, B)   # the plan reads both trees
        for t in {id(A): A, id(B): B}.values():
            t._plans += 1

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan has been freed")
        return self._h

    def stats(self) -> dict:
        st = Stats()
        _check(load().spamm_plan_stats(self.handle, ctypes.byref(st)), "spamm_plan_stats")
        return st.as_dict()

    def tasks(self) -> np.ndarray:
        cnt = ctypes.c_size_t()
        _check(load().spamm_plan_tasks(self.handle, None, 0, ctypes.byref(cnt)), "spamm_plan_tasks")
        out = np.empty(max(cnt.value, 1), dtype=np.uint64)
        _check(load().spamm_plan_tasks(self.handle, out.ctypes.data, out.size, ctypes.byref(cnt)),
               "spamm_plan_tasks")
        return out[:cnt.value]

    def subtasks(self) -> np.ndarray:
        """Sub-leaf culling: the 32 x 32 sub-products the last numeric pass
        performed, as sorted keys on the 32 x 32 grid."""
        cnt = ctypes.c_size_t()
        _check(load().spamm_plan_subtasks(self.handle, None, 0, ctypes.byref(cnt)),
               "spamm_plan_subtasks")
        out = np.empty(max(cnt.value, 1), dtype=np.uint64)
        _check(load().spamm_plan_subtasks(self.handle, out.ctypes.data, out.size,
                                          ctypes.byref(cnt)), "spamm_plan_subtasks")
        return out[:cnt.value]

    def numeric(self, C, stream=None):
        _device_matrix(C, "C")
        _check(load().spamm_numeric(self.handle, ctypes.c_void_p(C.data_ptr()), _stream(stream)),
               "spamm_numeric")
        return C

    def free(self):
        if self._h is not None:
            _check(load().spamm_plan_free(self._h), "spamm_plan_free")
            self._h = None
            for t in {id(t): t for t in self._keep}.values():
                t._plans -= 1

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_tree(A, leaf: int, stream=None, bf16: bool = False, subnorms: bool = False,
               fp16: bool = False) -> Tree:
    """Quadtree of A; bf16=True also keeps BF16 leaf copies (PREC_SPLIT_BF16
    and PREC_SPLIT_BF16X3),
    fp16=True FP16 copies at a per-leaf power-of-two scale (PREC_SPLIT_FP16);
    subnorms=True (leaf 64) also keeps 32 x 32 sub-block norms (sub-leaf
    culling)."""
    A = _device_matrix(A, "A")
    h = ctypes.c_void_p()
    flags = ((TREE_BF16 if bf16 else 0) | (TREE_SUBNORMS if subnorms else 0) |
             (TREE_FP16 if fp16 else 0))
    _check(load().spamm_build_tree_ex(ctypes.c_void_p(A.data_ptr()), A.shape[0], leaf, flags,
                                      _stream(stream), ctypes.byref(h)),
           "spamm_build_tree")
    t = Tree(h)
    t.bf16 = bool(bf16)
    t.fp16 = bool(fp16)
    t.subnorms = bool(subnorms)
    return t


def build_tree_sparse(A, leaf: int, tau: float, norm2_other: float = 0.0, stream=None,
                      bf16: bool = False) -> Tree:
    """Epsilon-sparsified quadtree of A: leaves with norm below
    tau / max(||A||_F, sqrt(norm2_other)) are dropped and not stored."""
    A = _device_matrix(A, "A")
    h = ctypes.c_void_p()
    _check(load().spamm_build_tree_sparse(ctypes.c_void_p(A.data_ptr()), A.shape[0], leaf,
                                          TREE_BF16 if bf16 else 0, float(tau), float(norm2_other),
                                          _stream(stream), ctypes.byref(h)),
           "spamm_build_tree_sparse")
    t = Tree(h)
    t.bf16 = bool(bf16)
    t.subnorms = False
    return t


def build_tree_output(C, plan: "Plan", stream=None, bf16: bool = False,
                      fp16: bool = False) -> Tree:
    """Quadtree of the product C that `plan` computed: only the leaves of C a
    kept product reaches are read and stored (the others are zero)."""
    C = _device_matrix(C, "C")
    h = ctypes.c_void_p()
    flags = (TREE_BF16 if bf16 else 0) | (TREE_FP16 if fp16 else 0)
    _check(load().spamm_build_tree_output(ctypes.c_void_p(C.data_ptr()), plan.handle, flags,
                                          _stream(stream), ctypes.byref(h)),
           "spamm_build_tree_output")
    t = Tree(h)
    t.bf16 = bool(bf16)
    t.fp16 = bool(fp16)
    t.subnorms = False
    return t


def _opts(tau, precision, low_tol, sub_cull=False, low_rel=0.0) -> Opts:
    return Opts(float(tau), int(precision), float(low_tol), 1 if sub_cull else 0, float(low_rel))


def symbolic(A: Tree, B: Tree, tau: float, stream=None, precision: int = PREC_FP32,
             low_tol: float = 0.0, sub_cull: bool = False, low_rel: float = 0.0) -> Plan:
    """Symbolic multiply; split precision classes a product LOW below the
    absolute low_tol, or below low_rel ||A||_F ||B||_F (relative theta,
    evaluated by the library from the trees' roots)."""
    h = ctypes.c_void_p()
    o = _opts(tau, precision, low_tol, sub_cull, low_rel)
    _check(load().spamm_symbolic_ex(A.handle, B.handle, ctypes.byref(o), _stream(stream),
                                    ctypes.byref(h)), "spamm_symbolic")
    return Plan(h, A, B)


def multiply(A: Tree, B: Tree, tau: float, C, stream=None):
    _device_matrix(C, "C")
    if C.shape[0] != A.n:
        raise ValueError("C has the wrong shape")
    _check(load().spamm_multiply(A.handle, B.handle, float(tau), ctypes.c_void_p(C.data_ptr()),
                                 _stream(stream)), "spamm_multiply")
    return C


def multiply_ex(A: Tree, B: Tree, tau: float, C, stream=None, precision: int = PREC_FP32,
                low_tol: float = 0.0, sub_cull: bool = False, low_rel: float = 0.0,
                stats: bool = True):
    """C = A B under the SpAMM condition.  With stats (default) the cull and
    the leaf GEMM are timed and the call synchronizes, returning the stats;
    stats=False enqueues the product asynchronously and returns None."""
    _device_matrix(C, "C")
    if C.shape[0] != A.n:
        raise ValueError("C has the wrong shape")
    st = Stats()
    o = _opts(tau, precision, low_tol, sub_cull, low_rel)
    _check(load().spamm_multiply_opts(A.handle, B.handle, ctypes.byref(o),
                                      ctypes.c_void_p(C.data_ptr()), _stream(stream),
                                      ctypes.byref(st) if stats else None),
           "spamm_multiply_opts")
    return st.as_dict() if stats else None


def multiply_noalloc(A: Tree, B: Tree, tau: float, C, stream=None, precision: int = PREC_FP32,
                     low_tol: float = 0.0, sub_cull: bool = False, low_rel: float = 0.0):
    """C = A B through spamm_multiply_noalloc: the task arena lives in the
    library's fixed per-device block, nothing is allocated (products of depth
    <= 8; calls on one device must not overlap)."""
    _device_matrix(C, "C")
    if C.shape[0] != A.n:
        raise ValueError("C has the wrong shape")
    o = _opts(tau, precision, low_tol, sub_cull, low_rel)
    _check(load().spamm_multiply_noalloc(A.handle, B.handle, ctypes.byref(o),
                                         ctypes.c_void_p(C.data_ptr()), _stream(stream)),
           "spamm_multiply_noalloc")
    return C


# ---- serving -----------------------------------------------------------------

def _request(A_ptr, B_ptr, C_ptr, n, leaf, tau, precision, low_tol, chain_len,
             low_rel=0.0) -> Request:
    return Request(A_ptr, B_ptr, C_ptr, int(n), int(leaf), int(precision), float(tau),
                   float(low_tol), int(chain_len), float(low_rel))


def request_footprint(n: int, leaf: int, tau: float = 0.0, precision: int = PREC_FP32,
                      low_tol: float = 0.0, chain_len: int = 0, distinct_b: bool = False,
                      low_rel: float = 0.0) -> int:
    """Device bytes a server reserves for such a request (host-only check;
    the placeholder pointers are never dereferenced)."""
    r = _request(1, 2 if distinct_b else None, 3, n, leaf, tau, precision, low_tol, chain_len,
                 low_rel)
    out = ctypes.c_size_t()
    _check(load().spamm_request_footprint(ctypes.byref(r), ctypes.byref(out)),
           "spamm_request_footprint")
    return out.value


class Server:
    """Continuous-batching SpAMM server on the current device.

    submit() queues C = A B (or a chain of `chain_len` squarings of A) and
    returns a ticket; poll() returns None while it runs, else the result
    dict.  The tensors of a request are kept referenced until its result has
    been collected.
    """

    def __init__(self, hbm_budget: int, max_slots: int = 8):
        h = ctypes.c_void_p()
        _check(load().spamm_server_create(int(hbm_budget), int(max_slots), ctypes.byref(h)),
               "spamm_server_create")
        self._h = h
        self._keep = {}

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("server has been destroyed")
        return self._h

    def submit(self, A, C, tau: float, leaf: int, B=None, precision: int = PREC_FP32,
               low_tol: float = 0.0, chain_len: int = 0, sync: bool = True,
               low_rel: float = 0.0) -> int:
        """Queue a request; `sync` first waits for the current stream so that
        A and B hold their values when the server's streams read them.
        low_rel is the relative split threshold theta, taken by the library
        against the roots of each product's (each chain step's) operands."""
        import torch
        _device_matrix(A, "A")
        _device_matrix(C, "C")
        if B is not None:
            _device_matrix(B, "B")
        for t in (C, B):
            if t is not None and t.shape != A.shape:
                raise ValueError("A, B and C must have the same shape")
        if sync:
            torch.cuda.current_stream().synchronize()
        r = _request(A.data_ptr(), None if B is None else B.data_ptr(), C.data_ptr(), A.shape[0],
                     leaf, tau, precision, low_tol, chain_len, low_rel)
        t = ctypes.c_uint64()
        _check(load().spamm_submit(self.handle, ctypes.byref(r), ctypes.byref(t)), "spamm_submit")
        self._keep[t.value] = (A, B, C)
        return t.value

    def poll(self, ticket: int):
        res = Result()
        rc = load().spamm_poll(self.handle, int(ticket), ctypes.byref(res))
        if rc == SPAMM_PENDING:
            return None
        _check(rc, "spamm_poll")
        self._keep.pop(int(ticket), None)
        return res.as_dict()

    def wait(self, ticket: int, timeout: float = 60.0) -> dict:
        import time
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() - t0 > timeout:
                raise TimeoutError(f"request {ticket} still pending after {timeout} s")
            time.sleep(50e-6)

    def info(self) -> dict:
        st = ServerStats()
        _check(load().spamm_server_info(self.handle, ctypes.byref(st)), "spamm_server_info")
        return st.as_dict()

    def destroy(self):
        if self._h is not None:
            _check(load().spamm_server_destroy(self._h), "spamm_server_destroy")
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
