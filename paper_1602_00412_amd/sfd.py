"""ctypes binding of libsfd.so (include/sfd.h): argument marshalling only.

Every step of the sketch runs in the HIP library; this module converts torch tensors / numpy
arrays to pointers and memory kinds, and error codes to exceptions.  It raises if the library
is not built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsfd.so")

SFD_OK = 0
SFD_E_ARG = -1
SFD_E_INDEX = -2
SFD_E_SHAPE = -3
SFD_E_NOMEM = -4
SFD_E_DEVICE = -5
SFD_E_NOCONVERGE = -6
SFD_E_STATE = -7
SFD_E_TOOBIG = -8
MEM_HOST = 0
MEM_DEVICE = 1
OPT_DELTA = 1
OPT_Q = 2
OPT_MAX_ATTEMPTS = 3
OPT_VERIFY = 4
OPT_STREAM_ID = 5
OPT_PROFILE = 6
OPT_CSC_BANDS = 7
OPT_LANES = 8
OPT_PRECISION = 9
PRECISION_FP32 = 0
PRECISION_BF16 = 1
OPT_ALGORITHM = 10
OPT_CSC_HOT_MIN = 11
OPT_TEST_ZERO_ROW = 12
OPT_TEST_ZERO_ATTEMPTS = 13
OPT_CQR2 = 14
CQR2_OFF = 0
CQR2_FINAL = 1
CQR2_ALL = 2
OPT_AUTOTUNE = 15
OPT_GRAPHS = 16
OPT_PRODUCT_LAUNCH = 17
ALGO_SFD = 0
ALGO_FD = 1
PROF_CLASSES = ["csc_build", "spmm_csr", "spmm_csc", "gram", "chol", "xform", "eig", "vs", "other", "fixup"]

EXPORTS = [
    "sfd_create",
    "sfd_destroy",
    "sfd_reset",
    "sfd_set_option",
    "sfd_set_stream",
    "sfd_append_csr",
    "sfd_sketch",
    "sfd_merge",
    "sfd_get_stats",
    "sfd_get_profile",
    "sfd_start_block",
    "sfd_strerror",
    "sfd_batch_create",
    "sfd_batch_destroy",
    "sfd_batch_reset",
    "sfd_batch_set_option",
    "sfd_batch_set_stream",
    "sfd_batch_get_stats",
    "sfd_batch_append_csr",
    "sfd_batch_sketch",
    "sfd_evaluate",
    "sfd_evaluate_noalloc",
]


class SfdError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [
        ("rows_seen", ctypes.c_int64),
        ("nnz_seen", ctypes.c_int64),
        ("flushes", ctypes.c_int64),
        ("vs_calls", ctypes.c_int64),
        ("attempts", ctypes.c_int64),
        ("vs_rejects", ctypes.c_int64),
        ("live_rows", ctypes.c_int32),
        ("pending_rows", ctypes.c_int32),
        ("pending_nnz", ctypes.c_int64),
        ("last_q", ctypes.c_int32),
        ("last_t", ctypes.c_int32),
        ("last_ln_norm", ctypes.c_double),
        ("last_delta", ctypes.c_double),
        ("last_fro2_buffer", ctypes.c_double),
        ("last_lambda_ell2", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class EvalResult(ctypes.Structure):
    """sfd_eval_t: the accuracy measures of a sketch (Sec. 4)."""
    _fields_ = [
        ("fro2A", ctypes.c_double),
        ("cov_min", ctypes.c_double),
        ("cov_max", ctypes.c_double),
        ("cov_err", ctypes.c_double),
        ("top_k_energy", ctypes.c_double),
        ("proj_num", ctypes.c_double),
        ("proj_err", ctypes.c_double),
        ("steps", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("cov_min_res", ctypes.c_double),
        ("cov_max_res", ctypes.c_double),
        ("top_k_res", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad"}


class Profile(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_int64 * 16),
        ("ms", ctypes.c_double * 16),
        ("bytes", ctypes.c_double * 16),
        ("flops", ctypes.c_double * 16),
        ("calls", ctypes.c_int64 * 16),
    ]

    def as_dict(self) -> dict:
        return {name: {"launches": int(self.launches[i]), "calls": int(self.calls[i]), "ms": float(self.ms[i]),
                       "bytes": float(self.bytes[i]), "flops": float(self.flops[i])}
                for i, name in enumerate(PROF_CLASSES)}


_lib = None


def load(path: str = LIB_PATH):
    """Load libsfd.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built (python -m paper_1602_00412_amd.build)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, u64, dbl, i = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    sig = {
        "sfd_create": (i, [i64, i32, dbl, u64, ctypes.POINTER(vp)]),
        "sfd_destroy": (i, [vp]),
        "sfd_reset": (i, [vp]),
        "sfd_set_option": (i, [vp, i, dbl]),
        "sfd_set_stream": (i, [vp, vp]),
        "sfd_append_csr": (i, [vp, i64, vp, vp, vp, i]),
        "sfd_sketch": (i, [vp, vp, i, ctypes.POINTER(i32)]),
        "sfd_merge": (i, [vp, vp]),
        "sfd_get_stats": (i, [vp, ctypes.POINTER(Stats)]),
        "sfd_get_profile": (i, [vp, ctypes.POINTER(Profile)]),
        "sfd_start_block": (i, [u64, u64, u64, u64, u64, i64, i32, vp]),
        "sfd_strerror": (ctypes.c_char_p, [i]),
        "sfd_batch_create": (i, [i32, i64, i32, dbl, u64, ctypes.POINTER(vp)]),
        "sfd_batch_destroy": (i, [vp]),
        "sfd_batch_reset": (i, [vp]),
        "sfd_batch_set_option": (i, [vp, i, dbl]),
        "sfd_batch_set_stream": (i, [vp, vp]),
        "sfd_batch_get_stats": (i, [vp, i32, ctypes.POINTER(Stats)]),
        "sfd_batch_append_csr": (i, [vp, i32, vp, vp, vp, vp, vp, i]),
        "sfd_batch_sketch": (i, [vp, vp, i]),
        "sfd_evaluate": (i, [i64, i64, vp, vp, vp, vp, i32, i32, i32, u64, vp, ctypes.POINTER(EvalResult)]),
        "sfd_evaluate_noalloc": (i, [i64, i64, vp, vp, vp, vp, i32, i32, i32, u64, vp, ctypes.POINTER(EvalResult)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().sfd_strerror(code).decode()


def _check(code: int, what: str):
    if code != SFD_OK:
        raise SfdError(code, what)


def _ptr_kind(x, dtype):
    """(pointer, memory kind, keep-alive) of a torch tensor or numpy array of ``dtype``."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(x, torch.Tensor):
        want = {np.int64: torch.int64, np.int32: torch.int32, np.float32: torch.float32}[dtype]
        if x.dtype != want:
            raise TypeError(f"expected {want}, got {x.dtype}")
        if not x.is_contiguous():
            x = x.contiguous()
        return x.data_ptr(), (MEM_DEVICE if x.is_cuda else MEM_HOST), x
    a = np.ascontiguousarray(x)
    if a.dtype != dtype:
        raise TypeError(f"expected {np.dtype(dtype)}, got {a.dtype}")
    return a.ctypes.data, MEM_HOST, a


def _out_ptr(out, shape, device: bool):
    """Pointer to a caller-supplied FP32 output buffer of ``shape`` after checking it: a contiguous
    CUDA tensor (device=True) or a C-contiguous writeable numpy array (device=False) with exactly
    that many elements, so the library never writes past it."""
    n = int(np.prod(shape))
    if device:
        import torch

        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
                and out.numel() == n):
            raise TypeError(f"out must be a contiguous CUDA float32 tensor of {n} elements {tuple(shape)}")
        return out.data_ptr()
    if not (isinstance(out, np.ndarray) and out.dtype == np.float32 and out.flags.c_contiguous and out.flags.writeable
            and out.size == n):
        raise TypeError(f"out must be a C-contiguous writeable float32 numpy array of {n} elements {tuple(shape)}")
    return out.ctypes.data


def _torch_stream_handle():
    import torch

    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


class Sketch:
    """A Sparse Frequent Directions stream (sfd_create ... sfd_destroy)."""

    def __init__(self, d: int, ell: int, eps: float = 0.25, seed: int = 0, *, delta=None, q=None,
                 max_attempts=None, verify=None, stream_id=None, csc_bands=None, csc_hot_min=None,
                 precision=None, algorithm=None, cqr2=None, autotune=None, graphs=None, launch=None,
                 use_torch_stream: bool = True):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.sfd_create(int(d), int(ell), float(eps), int(seed), ctypes.byref(h)), "sfd_create")
        self._h = h
        self.d, self.ell = int(d), int(ell)
        for key, val in ((OPT_DELTA, delta), (OPT_Q, q), (OPT_MAX_ATTEMPTS, max_attempts),
                         (OPT_VERIFY, None if verify is None else float(bool(verify))), (OPT_STREAM_ID, stream_id),
                         (OPT_CSC_BANDS, csc_bands), (OPT_CSC_HOT_MIN, csc_hot_min),
                         (OPT_PRECISION, None if precision is None else
                          {"fp32": PRECISION_FP32, "bf16": PRECISION_BF16}.get(precision, precision)),
                         (OPT_ALGORITHM, None if algorithm is None else
                          {"sfd": ALGO_SFD, "fd": ALGO_FD}.get(algorithm, algorithm)),
                         (OPT_CQR2, None if cqr2 is None else
                          {"off": CQR2_OFF, "final": CQR2_FINAL, "all": CQR2_ALL}.get(cqr2, cqr2)),
                         (OPT_AUTOTUNE, None if autotune is None else float(bool(autotune))),
                         (OPT_GRAPHS, None if graphs is None else float(bool(graphs))),
                         (OPT_PRODUCT_LAUNCH, None if launch is None else
                          {"auto": 0, "static": 1, "queue": 2, "stage": 3}.get(launch, launch))):
            if val is not None:
                self.set_option(key, val)
        if use_torch_stream:
            s = _torch_stream_handle()
            if s is not None:
                _check(lib.sfd_set_stream(self._h, ctypes.c_void_p(s)), "sfd_set_stream")

    def set_option(self, key: int, value: float):
        _check(load().sfd_set_option(self._h, int(key), float(value)), "sfd_set_option")

    def append_csr(self, indptr, indices, values):
        """Append rows in CSR form; torch CUDA tensors are read in device memory."""
        p_ptr, p_kind, k1 = _ptr_kind(indptr, np.int64)
        i_ptr, i_kind, k2 = _ptr_kind(indices, np.int32)
        v_ptr, v_kind, k3 = _ptr_kind(values, np.float32)
        if not (p_kind == i_kind == v_kind):
            raise ValueError("indptr, indices and values must live in the same kind of memory")
        nrows = (k1.numel() if hasattr(k1, "numel") else k1.size) - 1
        _check(load().sfd_append_csr(self._h, nrows, p_ptr, i_ptr, v_ptr, p_kind), "sfd_append_csr")
        del k1, k2, k3

    def sketch(self, out=None, device: bool = True):
        """B (ell x d, FP32): a torch CUDA tensor (device=True) or a numpy array."""
        live = ctypes.c_int32()
        if device:
            import torch

            if out is None:
                out = torch.empty((self.ell, self.d), dtype=torch.float32, device="cuda")
            ptr = _out_ptr(out, (self.ell, self.d), True)
            _check(load().sfd_sketch(self._h, ptr, MEM_DEVICE, ctypes.byref(live)), "sfd_sketch")
        else:
            if out is None:
                out = np.empty((self.ell, self.d), dtype=np.float32)
            ptr = _out_ptr(out, (self.ell, self.d), False)
            _check(load().sfd_sketch(self._h, ptr, MEM_HOST, ctypes.byref(live)), "sfd_sketch")
        self.last_live = live.value
        return out

    def merge(self, other: "Sketch"):
        _check(load().sfd_merge(self._h, other._h), "sfd_merge")

    def reset(self):
        _check(load().sfd_reset(self._h), "sfd_reset")

    def stats(self) -> dict:
        s = Stats()
        _check(load().sfd_get_stats(self._h, ctypes.byref(s)), "sfd_get_stats")
        return s.as_dict()

    def profile(self) -> dict:
        p = Profile()
        _check(load().sfd_get_profile(self._h, ctypes.byref(p)), "sfd_get_profile")
        return p.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().sfd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent streams (sfd_batch_create ... sfd_batch_destroy); stream s behaves as a
    Sketch with stream_id = s."""

    def __init__(self, nstreams: int, d: int, ell: int, eps: float = 0.25, seed: int = 0, *, precision=None,
                 lanes=None, autotune=None, graphs=None, use_torch_stream: bool = True):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.sfd_batch_create(int(nstreams), int(d), int(ell), float(eps), int(seed), ctypes.byref(h)),
               "sfd_batch_create")
        self._h = h
        self.nstreams, self.d, self.ell = int(nstreams), int(d), int(ell)
        if precision is not None:
            self.set_option(OPT_PRECISION, {"fp32": PRECISION_FP32, "bf16": PRECISION_BF16}.get(precision, precision))
        if lanes is not None:
            self.set_option(OPT_LANES, lanes)
        if autotune is not None:
            self.set_option(OPT_AUTOTUNE, float(bool(autotune)))
        if graphs is not None:
            self.set_option(OPT_GRAPHS, float(bool(graphs)))
        if use_torch_stream:
            s = _torch_stream_handle()
            if s is not None:
                _check(lib.sfd_batch_set_stream(self._h, ctypes.c_void_p(s)), "sfd_batch_set_stream")

    def set_option(self, key: int, value: float):
        _check(load().sfd_batch_set_option(self._h, int(key), float(value)), "sfd_batch_set_option")

    def append_csr(self, stream_of_seg, seg_row_start, indptr, indices, values):
        """Append a CSR block whose row segments go to the given streams (host segment table)."""
        sos = np.ascontiguousarray(stream_of_seg, dtype=np.int32)
        srs = np.ascontiguousarray(seg_row_start, dtype=np.int64)
        if srs.size != sos.size + 1:
            raise ValueError("seg_row_start needs one more entry than stream_of_seg")
        p_ptr, p_kind, k1 = _ptr_kind(indptr, np.int64)
        i_ptr, i_kind, k2 = _ptr_kind(indices, np.int32)
        v_ptr, v_kind, k3 = _ptr_kind(values, np.float32)
        if not (p_kind == i_kind == v_kind):
            raise ValueError("indptr, indices and values must live in the same kind of memory")
        _check(load().sfd_batch_append_csr(self._h, int(sos.size), sos.ctypes.data, srs.ctypes.data, p_ptr, i_ptr,
                                           v_ptr, p_kind), "sfd_batch_append_csr")
        del k1, k2, k3

    def sketch(self, out=None, device: bool = True):
        """All sketches (nstreams x ell x d, FP32): a torch CUDA tensor or a numpy array."""
        shape = (self.nstreams, self.ell, self.d)
        if device:
            import torch

            if out is None:
                out = torch.empty(shape, dtype=torch.float32, device="cuda")
            _check(load().sfd_batch_sketch(self._h, _out_ptr(out, shape, True), MEM_DEVICE), "sfd_batch_sketch")
        else:
            if out is None:
                out = np.empty(shape, dtype=np.float32)
            _check(load().sfd_batch_sketch(self._h, _out_ptr(out, shape, False), MEM_HOST), "sfd_batch_sketch")
        return out

    def reset(self):
        _check(load().sfd_batch_reset(self._h), "sfd_batch_reset")

    def stats(self, stream: int) -> dict:
        s = Stats()
        _check(load().sfd_batch_get_stats(self._h, int(stream), ctypes.byref(s)), "sfd_batch_get_stats")
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().sfd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def start_block(seed: int, stream_id: int, buffer: int, attempt: int, purpose: int, d: int, ell: int):
    """The FP32 start block G (d x ell) the library draws, as a torch CUDA tensor (sfd_start_block)."""
    import torch

    out = torch.empty((d, ell), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    _check(load().sfd_start_block(seed, stream_id, buffer, attempt, purpose, d, ell, out.data_ptr()), "sfd_start_block")
    return out


def evaluate(indptr, indices, values, d: int, B=None, k: int = 0, steps: int = 0, seed: int = 0,
             noalloc: bool = False) -> dict:
    """cov-err and proj-err of the sketch B (ell x d) against the CSR matrix A (sfd_evaluate, FP64 on
    the GPU).  indptr/indices/values and B are torch CUDA tensors (int64, int32, float32, float32).
    noalloc: call sfd_evaluate_noalloc (work memory from the library's fixed scratch) instead."""
    import torch

    n = int(indptr.numel()) - 1
    for t, dt in ((indptr, torch.int64), (indices, torch.int32), (values, torch.float32)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise TypeError("indptr / indices / values must be contiguous CUDA int64 / int32 / float32 tensors")
    ell, bp = 0, None
    if B is not None:
        if not (B.is_cuda and B.dtype == torch.float32 and B.is_contiguous() and B.dim() == 2 and B.shape[1] == d):
            raise TypeError("B must be a contiguous CUDA float32 tensor of shape (ell, d)")
        ell, bp = int(B.shape[0]), B.data_ptr()
    res = EvalResult()
    name = "sfd_evaluate_noalloc" if noalloc else "sfd_evaluate"
    _check(getattr(load(), name)(n, int(d), indptr.data_ptr(), indices.data_ptr(), values.data_ptr(), bp, ell,
                                 int(k), int(steps), int(seed),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(res)), name)
    return res.as_dict()
