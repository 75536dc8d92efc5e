"""Python binding of libcqr2.so (MI355X CholeskyQR2): argument marshalling only.

Every step of the factorization runs in the HIP kernels behind the C ABI
declared in ``include/cqr2.h``; torch supplies device memory and the current
stream.  There is no CPU or PyTorch fallback: if the library is not built,
``load()`` raises.

Matrices are column-major: a torch tensor of shape (m, n) with strides
(1, ld), ld >= m (``colmajor()`` converts).
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcqr2.so")

CQR2_ERR_HIP = -100
CQR2_ERR_UNSUPPORTED = -101
CQR2_ERR_TOO_LARGE = -102
CQR2_ERR_NOALLOC_LIMIT = -103
CQR2_NOALLOC_MAX_WORKSPACE = 20 << 20
CQR2_FP64 = 0
CQR2_MIXED_P1_FP32 = 1
CQR2_SHIFTED_CQR3 = 2
CQR2_MAX_INVERSE_DEPTH = 8


def CQR2_INVERSE_DEPTH(d: int) -> int:
    """Flag bits of the partial inverse with depth d (OR onto CQR2_FP64)."""
    return int(d) << 8
NUM_TIMERS = 6
TIMER_NAMES = ("gram", "gram_reduce", "cholinv", "q_pass1", "q_pass2", "upper_product")

# Every symbol include/cqr2.h declares, with (restype, argtypes).
_i64, _u32, _sz, _vp, _i32 = ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int
SIGNATURES = {
    "cqr2_factor": (_i32, [_vp, _i64, _i64, _i64, _vp, _vp, _vp]),
    "cqr2_factor_noalloc": (_i32, [_vp, _i64, _i64, _i64, _vp, _vp, _vp]),
    "cqr2_workspace_size": (_sz, [_i64, _i64, _u32]),
    "cqr2_factor_ex": (_i32, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp, _u32, _vp]),
    "cqr2_gram_workspace_size": (_sz, [_i64, _i64]),
    "cqr2_gram": (_i32, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _sz, _vp]),
    "cqr2_cholinv": (_i32, [_vp, _i64, _i64, _vp, _vp, _i64, _vp, _vp]),
    "cqr2_apply_rinv": (_i32, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp]),
    "cqr2_apply_rinv_f32": (_i32, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp]),
    "cqr2_upper_product": (_i32, [_vp, _vp, _vp, _i64, _i64, _vp]),
    "cqr2_status_string": (ctypes.c_char_p, [_i32]),
    "cqr2_version": (ctypes.c_char_p, []),
    "cqr2_timing_enable": (_i32, [_i32]),
    "cqr2_timing_reset": (_i32, []),
    "cqr2_timing_read": (_i32, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), _i32]),
    "cqr2_problem_check": (_i32, [_vp]),
    "cqr2_lstsq_workspace_size": (_sz, [_i64, _i64, _i64]),
    "cqr2_lstsq": (_i32, [_vp, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp,
                          _vp]),
    "cqr2_batched_workspace_size": (_sz, [_vp, _i32, _u32]),
    "cqr2_factor_batched": (_i32, [_vp, _i32, _vp, _sz, _u32, _vp]),
    "cqr2_server_create": (_i32, [_sz, _sz, _i32, _vp, ctypes.POINTER(_vp)]),
    "cqr2_server_destroy": (_i32, [_vp]),
    "cqr2_server_submit": (_i32, [_vp, _vp, _i64]),
    "cqr2_server_submit_lstsq": (_i32, [_vp, _vp, _vp, _i64, _i64, _vp, _i64, _i64]),
    "cqr2_server_step": (_i32, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "cqr2_server_poll": (_i32, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double), _i32,
                                ctypes.POINTER(ctypes.c_int32)]),
    "cqr2_server_clock": (_i32, [_vp]),
}


class Problem(ctypes.Structure):
    """cqr2_problem: one CholeskyQR2 problem (device pointers, column-major)."""
    _fields_ = [("A", _vp), ("Q", _vp), ("R", _vp), ("m", _i64), ("n", _i64), ("lda", _i64), ("ldq", _i64),
                ("ldr", _i64), ("d_info", _vp)]

_lib = None


class CQR2Error(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = "?"
        if _lib is not None:
            msg = _lib.cqr2_status_string(code).decode()
        super().__init__(f"{where} returned {code}: {msg}")


def load(path: str | None = None):
    """Load libcqr2.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1710_08471_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != 0:
        raise CQR2Error(rc, where)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def colmajor(t, ld: int | None = None):
    """Column-major copy of a 2-D tensor (strides (1, ld)) on the same device."""
    import torch
    m, n = t.shape
    ld = max(ld or m, 1)
    buf = torch.empty((n, ld), dtype=t.dtype, device=t.device)
    out = buf.t()[:m, :]
    out.copy_(t)
    return out


def empty_colmajor(m: int, n: int, dtype=None, device=None, ld: int | None = None):
    import torch
    ld = max(ld or m, 1)
    buf = torch.empty((n, ld), dtype=dtype or torch.float64, device=device)
    return buf.t()[:m, :]


def _ld(t) -> int:
    m, n = t.shape
    if t.stride(0) != 1 and not (m <= 1):
        raise ValueError("tensor must be column-major (stride(0) == 1)")
    return max(t.stride(1) if n > 1 else max(m, 1), 1)


def _require_cuda_f64(t, name):
    import torch
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")


def workspace_size(m: int, n: int, flags: int = CQR2_FP64) -> int:
    return int(load().cqr2_workspace_size(m, n, flags))


def factor(A):
    """(Q, R) = CholeskyQR2(A) with library-managed workspace (cqr2_factor)."""
    import torch
    lib = load()
    _require_cuda_f64(A, "A")
    m, n = A.shape
    lda = _ld(A)
    Q = empty_colmajor(m, n, device=A.device, ld=lda)
    R = empty_colmajor(n, n, device=A.device)
    rc = lib.cqr2_factor(_ptr(A), m, n, lda, _ptr(Q), _ptr(R), _stream())
    _check(rc, "cqr2_factor")
    return Q, R


def factor_noalloc(A, Q=None, R=None):
    """(Q, R) = CholeskyQR2(A) through cqr2_factor_noalloc (the library
    allocates nothing; Q and R are allocated here when None)."""
    lib = load()
    _require_cuda_f64(A, "A")
    m, n = A.shape
    lda = _ld(A)
    if Q is None:
        Q = empty_colmajor(m, n, device=A.device, ld=lda)
    if R is None:
        R = empty_colmajor(n, n, device=A.device)
    if _ld(Q) != lda or _ld(R) != max(n, 1):
        raise ValueError("Q must share A's leading dimension and R must have leading dimension n")
    rc = lib.cqr2_factor_noalloc(_ptr(A), m, n, lda, _ptr(Q), _ptr(R), _stream())
    _check(rc, "cqr2_factor_noalloc")
    return Q, R


def factor_ex(A, Q=None, R=None, work=None, info=None, flags: int = CQR2_FP64):
    """cqr2_factor_ex with caller buffers (allocated here when None)."""
    import torch
    lib = load()
    _require_cuda_f64(A, "A")
    m, n = A.shape
    lda = _ld(A)
    if Q is None:
        Q = empty_colmajor(m, n, device=A.device)
    if R is None:
        R = empty_colmajor(n, n, device=A.device)
    wbytes = workspace_size(m, n, flags)
    if work is None:
        work = torch.empty(max(wbytes, 1), dtype=torch.uint8, device=A.device)
    rc = lib.cqr2_factor_ex(_ptr(A), m, n, lda, _ptr(Q), _ld(Q), _ptr(R), _ld(R), _ptr(work),
                            work.numel() * work.element_size(), _ptr(info), flags, _stream())
    _check(rc, "cqr2_factor_ex")
    return Q, R


def gram(A, W=None, work=None):
    """W = AᵀA (cqr2_gram)."""
    import torch
    lib = load()
    _require_cuda_f64(A, "A")
    m, n = A.shape
    if W is None:
        W = empty_colmajor(n, n, device=A.device)
    wb = int(lib.cqr2_gram_workspace_size(m, n))
    if work is None:
        work = torch.empty(max(wb, 8), dtype=torch.uint8, device=A.device)
    rc = lib.cqr2_gram(_ptr(A), m, n, _ld(A), _ptr(W), _ld(W), _ptr(work),
                       work.numel() * work.element_size(), _stream())
    _check(rc, "cqr2_gram")
    return W


def cholinv(W, info=None):
    """(R, Rinv) = CholInv factors of the SPD matrix W (cqr2_cholinv)."""
    lib = load()
    _require_cuda_f64(W, "W")
    n = W.shape[0]
    R = empty_colmajor(n, n, device=W.device)
    Rinv = empty_colmajor(n, n, device=W.device)
    rc = lib.cqr2_cholinv(_ptr(W), n, _ld(W), _ptr(R), _ptr(Rinv), _ld(R), _ptr(info), _stream())
    _check(rc, "cqr2_cholinv")
    return R, Rinv


def apply_rinv(A, U, Q=None):
    """Q = A U for upper-triangular U (cqr2_apply_rinv); Q may be A (in place)."""
    lib = load()
    _require_cuda_f64(A, "A")
    _require_cuda_f64(U, "U")
    m, n = A.shape
    if Q is None:
        Q = empty_colmajor(m, n, device=A.device)
    rc = lib.cqr2_apply_rinv(_ptr(A), m, n, _ld(A), _ptr(U), _ld(U), _ptr(Q), _ld(Q), _stream())
    _check(rc, "cqr2_apply_rinv")
    return Q


def apply_rinv_f32(A, U, Q=None):
    """Q = fl32(A) fl32(U) in FP32 arithmetic, Q float32 (cqr2_apply_rinv_f32)."""
    import torch
    lib = load()
    _require_cuda_f64(A, "A")
    _require_cuda_f64(U, "U")
    m, n = A.shape
    if Q is None:
        Q = empty_colmajor(m, n, dtype=torch.float32, device=A.device)
    if Q.dtype != torch.float32:
        raise ValueError("Q must be float32")
    rc = lib.cqr2_apply_rinv_f32(_ptr(A), m, n, _ld(A), _ptr(U), _ld(U), _ptr(Q), _ld(Q), _stream())
    _check(rc, "cqr2_apply_rinv_f32")
    return Q


def upper_product(R2, R1, R=None):
    """R = R2 R1 for upper-triangular factors (cqr2_upper_product)."""
    lib = load()
    n = R2.shape[0]
    ld = _ld(R2)
    if _ld(R1) != ld:
        raise ValueError("R2 and R1 must share a leading dimension")
    if R is None:
        R = empty_colmajor(n, n, device=R2.device, ld=ld)
    rc = lib.cqr2_upper_product(_ptr(R2), _ptr(R1), _ptr(R), n, ld, _stream())
    _check(rc, "cqr2_upper_product")
    return R


def timing_enable(on: bool = True):
    load().cqr2_timing_enable(1 if on else 0)


def timing_reset():
    load().cqr2_timing_reset()


def timing_read():
    """{kernel class: (total_ms, launches)} since the last reset."""
    lib = load()
    tot = (ctypes.c_double * NUM_TIMERS)()
    cnt = (ctypes.c_int64 * NUM_TIMERS)()
    _check(lib.cqr2_timing_read(tot, cnt, NUM_TIMERS), "cqr2_timing_read")
    return {TIMER_NAMES[i]: (tot[i], cnt[i]) for i in range(NUM_TIMERS)}


def version() -> str:
    return load().cqr2_version().decode()


def lstsq(A, B, info=None):
    """(X, Q, R): least-squares solution of A X ~= B and the factorization (cqr2_lstsq)."""
    import torch
    lib = load()
    _require_cuda_f64(A, "A")
    _require_cuda_f64(B, "B")
    m, n = A.shape
    if B.dim() == 1:
        B = B[:, None]
    B = B if B.stride(0) == 1 else colmajor(B)
    nrhs = B.shape[1]
    X = empty_colmajor(n, nrhs, device=A.device)
    Q = empty_colmajor(m, n, device=A.device)
    R = empty_colmajor(n, n, device=A.device)
    wb = lib.cqr2_lstsq_workspace_size(m, n, max(nrhs, 1))
    work = torch.empty(max(int(wb), 256), dtype=torch.uint8, device=A.device)
    _check(lib.cqr2_lstsq(_ptr(A), m, n, _ld(A), _ptr(B), m if nrhs == 0 else _ld(B), nrhs, _ptr(X), _ld(X), _ptr(Q),
                          _ld(Q), _ptr(R), _ld(R), _ptr(work), work.numel(), _ptr(info), _stream()), "cqr2_lstsq")
    return X, Q, R


def problem(A, Q, R, info=None) -> Problem:
    """cqr2_problem for column-major device tensors A (m x n), Q (m x n), R (n x n)."""
    m, n = A.shape
    return Problem(A.data_ptr(), Q.data_ptr(), R.data_ptr(), m, n, _ld(A), _ld(Q), _ld(R),
                   info.data_ptr() if info is not None else None)


def factor_batched(As, infos=None):
    """[(Q, R), ...] = CholeskyQR2 of every matrix in `As` (cqr2_factor_batched).

    Problems with n <= 256 share the multi-problem step launches (six, or
    eight when a problem has n > 128); larger ones run the tiled path in turn.
    `infos`: optional int32 device tensor of len(As).
    """
    import torch
    lib = load()
    outs, probs = [], []
    for i, A in enumerate(As):
        _require_cuda_f64(A, "A")
        m, n = A.shape
        Q = empty_colmajor(m, n, device=A.device)
        R = empty_colmajor(n, n, device=A.device)
        outs.append((Q, R))
        probs.append(problem(A, Q, R, infos[i:i + 1] if infos is not None else None))
    arr = (Problem * len(probs))(*probs)
    wb = lib.cqr2_batched_workspace_size(arr, len(probs), CQR2_FP64)
    if wb == 0 and probs:
        for i, p in enumerate(probs):
            _check(lib.cqr2_problem_check(ctypes.byref(p)), f"problem {i}")
    work = torch.empty(max(int(wb), 256), dtype=torch.uint8, device=As[0].device if As else "cuda")
    _check(lib.cqr2_factor_batched(arr, len(probs), _ptr(work), work.numel(), CQR2_FP64, _stream()),
           "cqr2_factor_batched")
    return outs


class Server:
    """Continuous-batching CholeskyQR2 server (cqr2_server_*) on one stream.

    submit() queues a problem with a tag; step() admits what fits and launches
    one multi-problem step; poll() returns (tag, done_ms) of finished requests,
    done_ms being GPU event time since the last clock() call.
    """

    def __init__(self, arena_bytes: int, footprint_budget: int = 0, max_active: int = 256, stream=None):
        import torch
        self._lib = load()
        self._stream = stream or torch.cuda.current_stream()
        h = _vp()
        _check(self._lib.cqr2_server_create(arena_bytes, footprint_budget, max_active,
                                            _vp(self._stream.cuda_stream), ctypes.byref(h)), "cqr2_server_create")
        self._h = h
        self._keep = {}

    def close(self):
        if self._h is not None and self._h.value:
            _check(self._lib.cqr2_server_destroy(self._h), "cqr2_server_destroy")
        self._h = None
        self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def clock(self):
        _check(self._lib.cqr2_server_clock(self._h), "cqr2_server_clock")

    def submit(self, tag: int, A, Q, R, info=None):
        p = problem(A, Q, R, info)
        _check(self._lib.cqr2_server_submit(self._h, ctypes.byref(p), tag), "cqr2_server_submit")
        self._keep[tag] = (A, Q, R, info)   # tensors stay alive until done

    def submit_lstsq(self, tag: int, A, B, X, Q, R, info=None):
        """Queue a least-squares request: A = QR into Q, R and X = R^-1 Qᵀ B."""
        p = problem(A, Q, R, info)
        if B.dim() == 1 or X.dim() == 1:
            raise ValueError("B and X must be 2-D (column-major views)")
        nrhs = B.shape[1]
        _check(self._lib.cqr2_server_submit_lstsq(self._h, ctypes.byref(p), _ptr(B), _ld(B), nrhs, _ptr(X), _ld(X),
                                                  tag), "cqr2_server_submit_lstsq")
        self._keep[tag] = (A, B, X, Q, R, info)

    def step(self):
        act, q = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.cqr2_server_step(self._h, ctypes.byref(act), ctypes.byref(q)), "cqr2_server_step")
        return act.value, q.value

    def poll(self, max_count: int = 4096):
        tags = (ctypes.c_int64 * max_count)()
        ms = (ctypes.c_double * max_count)()
        cnt = ctypes.c_int32()
        _check(self._lib.cqr2_server_poll(self._h, tags, ms, max_count, ctypes.byref(cnt)), "cqr2_server_poll")
        out = [(int(tags[i]), float(ms[i])) for i in range(cnt.value)]
        for t, _ in out:
            self._keep.pop(t, None)
        return out
