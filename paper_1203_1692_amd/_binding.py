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

PREC_FP32 = 0
PREC_SPLIT_BF16 = 1
TREE_BF16 = 1

_lib = None


class SpammError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {code})")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("precision", ctypes.c_int32),
                ("low_tol", ctypes.c_double)]


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
        }


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
        "spamm_tree_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                            ctypes.POINTER(dbl)],
        "spamm_tree_norms": [vp, i32, vp, sz],
        "spamm_tree_matrix": [vp, i32, vp, sz],
        "spamm_symbolic": [vp, vp, dbl, vp, pp],
        "spamm_numeric": [vp, vp, vp],
        "spamm_plan_tasks": [vp, vp, sz, ctypes.POINTER(sz)],
        "spamm_plan_stats": [vp, ctypes.POINTER(Stats)],
        "spamm_plan_free": [vp],
        "spamm_multiply": [vp, vp, dbl, vp, vp],
        "spamm_multiply_ex": [vp, vp, dbl, vp, vp, ctypes.POINTER(Stats)],
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

    def free(self):
        if self._h is not None:
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

    def numeric(self, C, stream=None):
        _device_matrix(C, "C")
        _check(load().spamm_numeric(self.handle, ctypes.c_void_p(C.data_ptr()), _stream(stream)),
               "spamm_numeric")
        return C

    def free(self):
        if self._h is not None:
            _check(load().spamm_plan_free(self._h), "spamm_plan_free")
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_tree(A, leaf: int, stream=None, bf16: bool = False) -> Tree:
    """Quadtree of A; bf16=True also keeps BF16 leaf copies (split precision)."""
    A = _device_matrix(A, "A")
    h = ctypes.c_void_p()
    _check(load().spamm_build_tree_ex(ctypes.c_void_p(A.data_ptr()), A.shape[0], leaf,
                                      TREE_BF16 if bf16 else 0, _stream(stream), ctypes.byref(h)),
           "spamm_build_tree")
    t = Tree(h)
    t.bf16 = bool(bf16)
    return t


def _opts(tau, precision, low_tol) -> Opts:
    return Opts(float(tau), int(precision), float(low_tol))


def relative_low_tol(A: Tree, B: Tree, theta: float) -> float:
    """low_tol for the split class 'norm product < theta ||A||_F ||B||_F'."""
    import math
    return float(theta) * math.sqrt(A.norm2) * math.sqrt(B.norm2)


def symbolic(A: Tree, B: Tree, tau: float, stream=None, precision: int = PREC_FP32,
             low_tol: float = 0.0) -> Plan:
    h = ctypes.c_void_p()
    o = _opts(tau, precision, low_tol)
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
                low_tol: float = 0.0) -> dict:
    """C = A B under the SpAMM condition, timed (synchronizes); returns stats."""
    _device_matrix(C, "C")
    if C.shape[0] != A.n:
        raise ValueError("C has the wrong shape")
    st = Stats()
    o = _opts(tau, precision, low_tol)
    _check(load().spamm_multiply_opts(A.handle, B.handle, ctypes.byref(o),
                                      ctypes.c_void_p(C.data_ptr()), _stream(stream),
                                      ctypes.byref(st)), "spamm_multiply_opts")
    return st.as_dict()
