"""ctypes binding of the C ABI declared in include/rpcholqr.h.

Argument marshalling only: every step of the factorization runs in the HIP
kernels of librpcholqr.so.  torch supplies device memory and the stream.
Matrices are float64 CUDA (HIP) tensors in column-major order, i.e. an (m, n)
tensor with strides (1, ld), ld >= m -- for example ``torch.empty(n, m).t()``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "librpcholqr.so")

STATUS = {0: "OK", -1: "EINVAL", -2: "EHIP", -3: "EWORKSPACE", -4: "EUNSUPPORTED"}
INFO = {0: "OK", 1: "ESKETCH", 2: "ECHOL", 3: "ECHOL2"}
FP64, FP32_REFINE, BF16X2_REFINE, A1_FP32 = 0, 1, 2, 3
SMOOTH = 0x100  # OR into precision: sample rows of the smoothed F A (rpcholqr.h, RPCHOLQR_SMOOTH)

# Every function the header declares, with its ctypes signature.
_i64, _u64, _i32, _vp, _sz = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
SIGNATURES = {
    "rpcholqr_max_n": (_i32, []),
    "rpcholqr_workspace_bytes": (_sz, [_i64, _i64, _i64, _i32]),
    "rpcholqr_factor": (_i32, [_i64, _i64, _i64, _u64, _vp, _i64, _vp, _i64, _vp, _i64, _i32, _vp, _sz, _vp, _vp]),
    "rpcholqr_factor_debug": (_i32, [_i64, _i64, _i64, _u64, _vp, _i64, _vp, _i64, _vp, _i64, _i32, _vp, _sz,
                                     _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rpcholqr_factor_noalloc": (_i32, [_i64, _i64, _i64, _u64, _vp, _i64, _vp, _i64, _vp, _i64, _i32, _vp, _vp]),
    "rpcholqr_precond_factor": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _i32, _vp, _sz,
                                       _vp, _vp]),
    "rpcholqr_sample_indices": (_i32, [_i64, _i64, _u64, ctypes.POINTER(_i64)]),
    "rpcholqr_timing_enable": (_i32, [_i32]),
    "rpcholqr_timing_read": (_i32, [ctypes.POINTER(ctypes.c_double), _i32]),
    "rpcholqr_batched_plan_create": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32,
                                            ctypes.POINTER(_vp), ctypes.POINTER(_i64)]),
    "rpcholqr_batched_execute": (_i32, [_vp, _vp, _vp]),
    "rpcholqr_batched_set_tuning": (_i32, [_vp, _i32]),
    "rpcholqr_batched_plan_device_bytes": (_sz, [_vp]),
    "rpcholqr_batched_plan_destroy": (_i32, [_vp]),
    "rpcholqr_factor_batched": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp,
                                       ctypes.POINTER(_i64)]),
}
NSTAGES = 5
STAGES = ("sketch", "passA", "reduce", "cholesky", "passB")


class RpCholQRError(RuntimeError):
    """A call returned a non-OK status, or the device reported a numerical failure."""

    def __init__(self, msg, status=None, code=None, index=None):
        super().__init__(msg)
        self.status, self.code, self.index = status, code, index


_lib = None


def load_library():
    """Loads librpcholqr.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2406_11751_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def max_n() -> int:
    return int(load_library().rpcholqr_max_n())


def workspace_bytes(m: int, n: int, s: int, precision: int = FP64) -> int:
    return int(load_library().rpcholqr_workspace_bytes(m, n, s, precision))


def timing_enable(on: bool = True) -> None:
    rc = load_library().rpcholqr_timing_enable(1 if on else 0)
    if rc != 0:
        raise RpCholQRError(f"rpcholqr_timing_enable returned {STATUS.get(rc, rc)}", status=rc)


def timing_read():
    """(calls, {stage: summed ms}) of the calls timed since the last read."""
    buf = (ctypes.c_double * NSTAGES)()
    calls = load_library().rpcholqr_timing_read(buf, NSTAGES)
    if calls < 0:
        raise RpCholQRError(f"rpcholqr_timing_read returned {STATUS.get(calls, calls)}", status=calls)
    return calls, {STAGES[i]: buf[i] for i in range(NSTAGES)}


def colmajor_empty(m: int, n: int, device, dtype=None):
    """Uninitialized (m, n) column-major tensor with leading dimension m."""
    import torch

    return torch.empty((n, m), dtype=dtype or torch.float64, device=device).t()


def _ld(t, rows):
    import torch

    if t.dtype != torch.float64 or t.dim() != 2 or not t.is_cuda:
        raise ValueError("expected a 2-D float64 device tensor")
    if t.shape[0] != rows:
        raise ValueError(f"expected {rows} rows, got {t.shape[0]}")
    if t.shape[1] > 1 and t.stride(0) != 1:
        raise ValueError("matrix must be column-major (stride (1, ld))")
    return max(t.stride(1), rows) if t.shape[1] > 1 else max(rows, 1)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes, workspace, dev, stream):
    """The caller's workspace if it is large enough, else a new one.  A new one
    used on a caller's stream is marked as in use on that stream, so that the
    caching allocator does not hand its memory to other work before the
    kernels launched there have finished with it."""
    import torch

    if workspace is not None and workspace.numel() * workspace.element_size() >= nbytes:
        return workspace
    workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if stream is not None:
        workspace.record_stream(torch.cuda.ExternalStream(stream, device=dev))
    return workspace


def factor(A, s: int, seed: int, *, Q=None, R=None, workspace=None, info=None, stream=None,
           precision: int = FP64, check: bool = True, debug: bool = False):
    """Thin QR A = Q R by rpCholesky-QR on the GPU.

    Returns (Q, R, info) where info is a device int32 tensor {code, index}.
    With check=True the stream is synchronized and a numerical failure raises
    RpCholQRError.  With debug=True a dict of intermediates (idx, As, Rs, A1,
    G1, R2) is returned as a fourth element.
    """
    import torch

    lib = load_library()
    m, n = A.shape
    dev = A.device
    lda = _ld(A, m)
    if Q is None:
        Q = colmajor_empty(m, n, dev)
    if R is None:
        R = colmajor_empty(n, n, dev)
    ldq, ldr = _ld(Q, m), _ld(R, n)
    wsb = workspace_bytes(m, n, s, precision)
    if wsb == 0:
        raise RpCholQRError(f"unsupported sizes m={m} n={n} s={s} (max n {max_n()})", status=-4)
    workspace = _workspace(wsb, workspace, dev, stream)
    if info is None:
        info = torch.empty(2, dtype=torch.int32, device=dev)
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream)
    common = (m, n, s, seed & (2**64 - 1), _ptr(A), lda, _ptr(Q), ldq, _ptr(R), ldr, precision,
              _ptr(workspace), workspace.numel() * workspace.element_size(), _ptr(info), st)
    extra = None
    if debug:
        extra = dict(idx=torch.empty(s, dtype=torch.int64, device=dev), As=colmajor_empty(s, n, dev),
                     Rs=colmajor_empty(n, n, dev), A1=colmajor_empty(m, n, dev),
                     G1=colmajor_empty(n, n, dev), R2=colmajor_empty(n, n, dev))
        rc = lib.rpcholqr_factor_debug(*common, *(_ptr(extra[k]) for k in ("idx", "As", "Rs", "A1", "G1", "R2")))
    else:
        rc = lib.rpcholqr_factor(*common)
    if rc != 0:
        raise RpCholQRError(f"rpcholqr_factor returned {STATUS.get(rc, rc)}", status=rc)
    if check:
        torch.cuda.synchronize(dev)
        code, index = (int(v) for v in info.cpu().tolist())
        if code != 0:
            raise RpCholQRError(f"numerical failure {INFO.get(code, code)} at column {index}", code=code,
                                index=index)
    return (Q, R, info, extra) if debug else (Q, R, info)


def factor_noalloc(A, s: int, seed: int, *, Q=None, R=None, info=None, stream=None, precision: int = FP64,
                   check: bool = True):
    """rpcholqr_factor_noalloc: as factor(), with the workspace in the library's
    static device array (nothing is allocated by the call).  Returns (Q, R, info)."""
    import torch

    lib = load_library()
    m, n = A.shape
    dev = A.device
    lda = _ld(A, m)
    if Q is None:
        Q = colmajor_empty(m, n, dev)
    if R is None:
        R = colmajor_empty(n, n, dev)
    ldq, ldr = _ld(Q, m), _ld(R, n)
    if info is None:
        info = torch.empty(2, dtype=torch.int32, device=dev)
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream)
    rc = lib.rpcholqr_factor_noalloc(m, n, s, seed & (2**64 - 1), _ptr(A), lda, _ptr(Q), ldq, _ptr(R), ldr,
                                     precision, _ptr(info), st)
    if rc != 0:
        raise RpCholQRError(f"rpcholqr_factor_noalloc returned {STATUS.get(rc, rc)}", status=rc)
    if check:
        torch.cuda.synchronize(dev)
        code, index = (int(v) for v in info.cpu().tolist())
        if code != 0:
            raise RpCholQRError(f"numerical failure {INFO.get(code, code)} at column {index}", code=code,
                                index=index)
    return Q, R, info


def precond_factor(A, Rs, *, Q=None, R=None, workspace=None, info=None, stream=None, precision: int = FP64,
                   check: bool = True):
    """Algorithm "Preconditioned Cholesky-QR" with the given n x n upper
    triangular preconditioner Rs (a device float64 tensor, column-major).
    Returns (Q, R, info) as factor does."""
    import torch

    lib = load_library()
    m, n = A.shape
    if tuple(Rs.shape) != (n, n):
        raise ValueError(f"Rs must be {n} x {n}")
    dev = A.device
    lda, ldrs = _ld(A, m), _ld(Rs, n)
    if Q is None:
        Q = colmajor_empty(m, n, dev)
    if R is None:
        R = colmajor_empty(n, n, dev)
    ldq, ldr = _ld(Q, m), _ld(R, n)
    wsb = workspace_bytes(m, n, n, precision)
    if wsb == 0:
        raise RpCholQRError(f"unsupported sizes m={m} n={n} (max n {max_n()})", status=-4)
    workspace = _workspace(wsb, workspace, dev, stream)
    if info is None:
        info = torch.empty(2, dtype=torch.int32, device=dev)
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream)
    rc = lib.rpcholqr_precond_factor(m, n, _ptr(A), lda, _ptr(Rs), ldrs, _ptr(Q), ldq, _ptr(R), ldr, precision,
                                     _ptr(workspace), workspace.numel() * workspace.element_size(), _ptr(info), st)
    if rc != 0:
        raise RpCholQRError(f"rpcholqr_precond_factor returned {STATUS.get(rc, rc)}", status=rc)
    if check:
        torch.cuda.synchronize(dev)
        code, index = (int(v) for v in info.cpu().tolist())
        if code != 0:
            raise RpCholQRError(f"numerical failure {INFO.get(code, code)} at column {index}", code=code,
                                index=index)
    return Q, R, info


def sample_indices(m: int, s: int, seed: int):
    """The s sampled row indices of factor() for (m, seed), computed on the host
    by the library (numpy int64 array)."""
    import numpy as np

    idx = np.empty(max(s, 0), dtype=np.int64)
    rc = load_library().rpcholqr_sample_indices(m, s, seed & (2**64 - 1),
                                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RpCholQRError(f"rpcholqr_sample_indices returned {STATUS.get(rc, rc)}", status=rc)
    return idx


class BatchedTuning(ctypes.Structure):
    """rpcholqr_batched_tuning (include/rpcholqr.h)."""

    _fields_ = [("nmax", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("m_max", ctypes.c_int64),
                ("pa_rows", ctypes.c_int32), ("pa_max", ctypes.c_int32), ("pb_rows", ctypes.c_int32),
                ("reserved1", ctypes.c_int32)]


TUNING_PATH = os.path.join(HERE, "tuning", "batched_mi355x.json")
_tuning_installed = False


def set_batched_tuning(entries) -> None:
    """Installs the batched launch-shape table (a list of dicts with keys nmax,
    m_max, pa_rows, pa_max, pb_rows); an empty list restores the built-in shapes."""
    global _tuning_installed
    arr = (BatchedTuning * max(len(entries), 1))()
    for i, e in enumerate(entries):
        arr[i] = BatchedTuning(int(e["nmax"]), 0, int(e["m_max"]), int(e["pa_rows"]), int(e["pa_max"]),
                               int(e["pb_rows"]), 0)
    rc = load_library().rpcholqr_batched_set_tuning(ctypes.cast(arr, ctypes.c_void_p), len(entries))
    if rc != 0:
        raise RpCholQRError(f"rpcholqr_batched_set_tuning returned {STATUS.get(rc, rc)}", status=rc)
    _tuning_installed = True


def load_batched_tuning(path: str = TUNING_PATH) -> bool:
    """Installs the table the autotuner wrote (paper_2406_11751_amd/autotune.py), if
    the file exists.  Returns whether a table was installed."""
    import json

    if not os.path.exists(path):
        return False
    with open(path) as f:
        set_batched_tuning(json.load(f)["entries"])
    return True


class BatchedPlan:
    """A batch of independent factorizations planned once and executed any
    number of times (rpcholqr_batched_plan_*).  The plan keeps references to the
    caller's A, Q and R tensors; Q and R are allocated here when not given."""

    def __init__(self, As, s, seeds, *, Qs=None, Rs=None, precision: int = FP64):
        import torch

        lib = load_library()
        if not _tuning_installed:
            load_batched_tuning()
        b = len(As)
        if b < 1:
            raise ValueError("empty batch")
        s = list(s) if hasattr(s, "__len__") else [s] * b
        seeds = list(seeds) if hasattr(seeds, "__len__") else [seeds + i for i in range(b)]
        if Qs is None:
            Qs = [colmajor_empty(A.shape[0], A.shape[1], A.device) for A in As]
        if Rs is None:
            Rs = [colmajor_empty(A.shape[1], A.shape[1], A.device) for A in As]
        self.As, self.Qs, self.Rs = list(As), list(Qs), list(Rs)
        self.batch = b
        self.device = As[0].device
        I64 = ctypes.c_int64 * b
        P = ctypes.c_void_p * b
        m = I64(*[A.shape[0] for A in As])
        n = I64(*[A.shape[1] for A in As])
        sv = I64(*s)
        sd = (ctypes.c_uint64 * b)(*[int(x) & (2**64 - 1) for x in seeds])
        lda = I64(*[_ld(A, A.shape[0]) for A in As])
        ldq = I64(*[_ld(Q, A.shape[0]) for Q, A in zip(Qs, As)])
        ldr = I64(*[_ld(R, A.shape[1]) for R, A in zip(Rs, As)])
        pa = P(*[A.data_ptr() for A in As])
        pq = P(*[Q.data_ptr() for Q in Qs])
        pr = P(*[R.data_ptr() for R in Rs])
        handle = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        with torch.cuda.device(self.device):
            rc = lib.rpcholqr_batched_plan_create(b, m, n, sv, sd, pa, lda, pq, ldq, pr, ldr, precision,
                                                  ctypes.byref(handle), ctypes.byref(bad))
        if rc != 0:
            raise RpCholQRError(f"rpcholqr_batched_plan_create returned {STATUS.get(rc, rc)} "
                                f"(problem {bad.value})", status=rc)
        self._h = handle
        self.device_bytes = int(lib.rpcholqr_batched_plan_device_bytes(handle))

    def execute(self, info=None, stream=None, check: bool = True):
        """Launches the batch; returns the (batch, 2) int32 device info tensor.
        With check=True the stream is synchronized and any failed problem raises."""
        import torch

        if self._h is None:
            raise RuntimeError("plan destroyed")
        if info is None:
            info = torch.empty((self.batch, 2), dtype=torch.int32, device=self.device)
        st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream)
        rc = load_library().rpcholqr_batched_execute(self._h, _ptr(info), st)
        if rc != 0:
            raise RpCholQRError(f"rpcholqr_batched_execute returned {STATUS.get(rc, rc)}", status=rc)
        if check:
            torch.cuda.synchronize(self.device)
            bad = (info[:, 0] != 0).nonzero()
            if bad.numel():
                i = int(bad[0, 0])
                code, index = (int(v) for v in info[i].tolist())
                raise RpCholQRError(f"problem {i}: numerical failure {INFO.get(code, code)} at column {index}",
                                    code=code, index=index)
        return info

    def close(self):
        if getattr(self, "_h", None) is not None:
            import torch

            torch.cuda.synchronize(self.device)
            load_library().rpcholqr_batched_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor_batched(As, s, seeds, *, check: bool = True, precision: int = FP64):
    """Thin QR of every matrix in As.  Returns (Qs, Rs, info)."""
    plan = BatchedPlan(As, s, seeds, precision=precision)
    try:
        info = plan.execute(check=check)
    finally:
        plan.close()
    return plan.Qs, plan.Rs, info
