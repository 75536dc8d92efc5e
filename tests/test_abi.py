"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before any HIP call."""
import ctypes
import os
import re

import pytest

import paper_1710_08471_amd as cq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cqr2.h")

pytestmark = pytest.mark.skipif(not os.path.exists(cq.LIB_PATH),
                                reason="libcqr2.so not built (run python -m paper_1710_08471_amd.build)")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cqr2_\w+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("cqr2_factor", "cqr2_factor_ex", "cqr2_workspace_size", "cqr2_gram", "cqr2_cholinv",
                 "cqr2_apply_rinv", "cqr2_upper_product", "cqr2_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(cq.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(cq.SIGNATURES), "binding signatures out of sync with header"


def test_version_and_status_strings():
    lib = cq.load()
    assert b"gfx950" in lib.cqr2_version()
    assert lib.cqr2_status_string(0) == b"success"
    assert b"HIP" in lib.cqr2_status_string(cq.CQR2_ERR_HIP)


FAKE = ctypes.c_void_p(0x10000)        # never dereferenced: validation fails first
FAKE2 = ctypes.c_void_p(0x10000000)
NULL = ctypes.c_void_p(0)


def test_factor_argument_errors():
    lib = cq.load()
    f = lib.cqr2_factor
    assert f(FAKE, 10, -1, 10, FAKE2, FAKE2, NULL) == -3            # n < 0
    assert f(FAKE, 3, 5, 5, FAKE2, FAKE2, NULL) == -2               # m < n
    assert f(FAKE, 10, 5, 9, FAKE2, FAKE2, NULL) == -4              # lda < m
    assert f(NULL, 10, 5, 10, FAKE2, FAKE2, NULL) == -1             # A NULL
    assert f(FAKE, 10, 5, 10, NULL, FAKE2, NULL) == -5              # Q NULL
    assert f(FAKE, 10, 5, 10, FAKE2, NULL, NULL) == -6              # R NULL
    assert f(ctypes.c_void_p(0x10004), 10, 5, 10, FAKE2, FAKE2, NULL) == -1   # misaligned
    assert f(FAKE, 10, 5, 10, ctypes.c_void_p(0x10000 + 80), FAKE2, NULL) == -5  # Q overlaps A
    assert f(FAKE, 40000, 20000, 40000, FAKE2, ctypes.c_void_p(0x20000000), NULL) == cq.CQR2_ERR_UNSUPPORTED
    assert f(NULL, 10, 0, 10, NULL, NULL, NULL) == 0                # n == 0: quick return


def test_factor_noalloc_argument_errors():
    # host checks only: nothing reaches the GPU
    lib = cq.load()
    assert lib.cqr2_factor_noalloc(FAKE, 10, 5, 9, FAKE2, ctypes.c_void_p(0x60000000), NULL) == -4
    assert lib.cqr2_factor_noalloc(FAKE, 4, 5, 10, FAKE2, ctypes.c_void_p(0x60000000), NULL) == -2
    assert lib.cqr2_factor_noalloc(NULL, 10, 5, 10, FAKE2, ctypes.c_void_p(0x60000000), NULL) == -1
    assert lib.cqr2_factor_noalloc(FAKE, 10, 5, 10, FAKE, ctypes.c_void_p(0x60000000), NULL) == -5
    assert lib.cqr2_factor_noalloc(FAKE, 10, 0, 10, NULL, NULL, NULL) == 0
    # every n <= 128 problem fits the static scratch; a bigger workspace is refused
    limit = cq.CQR2_NOALLOC_MAX_WORKSPACE
    assert max(lib.cqr2_workspace_size(m, 128, 0) for m in (128, 4096, 1 << 20, 1 << 30)) <= limit
    assert lib.cqr2_workspace_size(1 << 20, 200, 0) > limit
    assert lib.cqr2_factor_noalloc(ctypes.c_void_p(1 << 40), 1 << 20, 200, 1 << 20, ctypes.c_void_p(1 << 41),
                                   ctypes.c_void_p(1 << 42), NULL) == cq.CQR2_ERR_NOALLOC_LIMIT
    assert "no-allocation" in lib.cqr2_status_string(cq.CQR2_ERR_NOALLOC_LIMIT).decode()


def test_factor_ex_argument_errors():
    lib = cq.load()
    f = lib.cqr2_factor_ex
    W = ctypes.c_void_p(0x40000000)
    ws = lib.cqr2_workspace_size(100, 10, 0)
    assert ws > 0
    ok = dict(A=FAKE, m=100, n=10, lda=100, Q=FAKE2, ldq=100, R=ctypes.c_void_p(0x30000000), ldr=10,
              work=W, wb=ws, info=NULL, flags=0)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["A"], a["m"], a["n"], a["lda"], a["Q"], a["ldq"], a["R"], a["ldr"], a["work"], a["wb"],
                 a["info"], a["flags"], NULL)

    assert call(ldq=99) == -6
    assert call(ldr=9) == -8
    assert call(flags=7) == -12
    assert call(flags=3) == -12
    assert call(wb=lib.cqr2_workspace_size(100, 10, 1) - 1, flags=1) == -10
    assert call(work=NULL) == -9
    assert call(work=ctypes.c_void_p(0x40000008)) == -9           # not 256-byte aligned
    assert call(wb=ws - 1) == -10
    assert call(info=ctypes.c_void_p(0x50000002)) == -11
    assert call(R=ctypes.c_void_p(0x10000 + 8)) == -7               # R overlaps A
    assert call(work=ctypes.c_void_p(0x10000000)) == -9             # workspace overlaps Q


def test_workspace_size_contract():
    lib = cq.load()
    assert lib.cqr2_workspace_size(10, 20, 0) == 0       # m < n
    assert lib.cqr2_workspace_size(100, 0, 0) == 0
    assert lib.cqr2_workspace_size(40000, 20000, 0) == 0  # beyond CQR2_MAX_N
    assert lib.cqr2_workspace_size(1000, 200, 0) > 0      # general (tiled) path
    assert lib.cqr2_workspace_size(1000, 20, 1) > 0       # mixed precision (tiled path at any n)
    assert lib.cqr2_workspace_size(1000, 20, 3) == 0      # unknown flag bits
    assert lib.cqr2_workspace_size(1000, 20, 2) == lib.cqr2_workspace_size(1000, 20, 0)   # shifted CQR3
    small = lib.cqr2_workspace_size(4096, 64, 0)
    big = lib.cqr2_workspace_size(1 << 20, 128, 0)
    assert 0 < small < big
    assert small % 256 == 0 and big % 256 == 0
    # depends only on the problem, never on the device
    assert lib.cqr2_workspace_size(1 << 20, 128, 0) == big


def test_step_entry_argument_errors():
    lib = cq.load()
    assert lib.cqr2_gram(FAKE, 10, 5, 9, FAKE2, 5, FAKE2, 1 << 20, NULL) == -4
    assert lib.cqr2_gram(FAKE, 10, 5, 10, FAKE2, 4, FAKE2, 1 << 20, NULL) == -6
    assert lib.cqr2_gram(FAKE, 10, 5, 10, FAKE2, 5, NULL, 1 << 20, NULL) == -7
    assert lib.cqr2_gram(FAKE, 10, 5, 10, FAKE2, 5, ctypes.c_void_p(0x60000000), 8, NULL) == -8
    assert lib.cqr2_cholinv(FAKE, 5, 4, FAKE2, ctypes.c_void_p(0x60000000), 5, NULL, NULL) == -3
    assert lib.cqr2_cholinv(FAKE, 5, 5, FAKE2, FAKE2, 5, NULL, NULL) == -5     # R == Rinv
    assert lib.cqr2_apply_rinv(FAKE, 10, 5, 10, FAKE2, 4, ctypes.c_void_p(0x60000000), 10, NULL) == -6
    assert lib.cqr2_apply_rinv(FAKE, 10, 5, 10, FAKE2, 5, FAKE, 11, NULL) == -8  # in place needs ldq == lda
    # FP32 product of the mixed form: argument checks only (nothing launched)
    q32 = ctypes.c_void_p(0x60000000)
    assert lib.cqr2_apply_rinv_f32(FAKE, 10, 5, 9, FAKE2, 5, q32, 10, NULL) == -4
    assert lib.cqr2_apply_rinv_f32(FAKE, 10, 5, 10, FAKE2, 4, q32, 10, NULL) == -6
    assert lib.cqr2_apply_rinv_f32(FAKE, 10, 5, 10, FAKE2, 5, q32, 9, NULL) == -8
    assert lib.cqr2_apply_rinv_f32(FAKE, 10, 5, 10, FAKE2, 5, ctypes.c_void_p(0x60000002), 10, NULL) == -7
    assert lib.cqr2_apply_rinv_f32(FAKE, 10, 5, 10, FAKE2, 5, FAKE, 10, NULL) == -7   # Q overlaps A
    assert lib.cqr2_apply_rinv_f32(FAKE, 10, 0, 10, FAKE2, 1, q32, 10, NULL) == 0     # n == 0: nothing to do
    assert lib.cqr2_upper_product(FAKE, FAKE2, FAKE, 5, 5, NULL) == -3          # R overlaps R2
    assert lib.cqr2_upper_product(FAKE, FAKE2, ctypes.c_void_p(0x60000000), 5, 4, NULL) == -5


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib
    mod = importlib.import_module("paper_1710_08471_amd")
    saved = mod._lib
    mod._lib = None
    try:
        with pytest.raises(RuntimeError):
            mod.load(str(tmp_path / "missing.so"))
    finally:
        mod._lib = saved


def _problem(**kw):
    import paper_1710_08471_amd as cqm
    base = dict(A=0x10000, Q=0x10000000, R=0x20000000, m=100, n=10, lda=100, ldq=100, ldr=10, d_info=None)
    base.update(kw)
    return cqm.Problem(base["A"], base["Q"], base["R"], base["m"], base["n"], base["lda"], base["ldq"],
                       base["ldr"], base["d_info"])


def test_problem_check_codes():
    lib = cq.load()
    chk = lambda **kw: lib.cqr2_problem_check(ctypes.byref(_problem(**kw)))
    assert chk() == 0
    assert chk(n=-1) == -3
    assert chk(m=5) == -2
    assert chk(lda=99) == -4
    assert chk(ldq=99) == -6
    assert chk(ldr=9) == -8
    assert chk(d_info=0x30000002) == -11
    assert chk(A=None) == -1
    assert chk(A=0x10004) == -1
    assert chk(Q=0x10000 + 80) == -5          # Q overlaps A
    assert chk(R=0x10000000 + 8) == -7        # R overlaps Q
    assert chk(m=40000, n=20000, lda=40000, ldq=40000, ldr=20000, R=0x80000000) == cq.CQR2_ERR_UNSUPPORTED
    assert chk(n=0, A=None, Q=None, R=None) == 0


def test_batched_argument_errors():
    lib = cq.load()
    probs = (cq.Problem * 2)(_problem(), _problem(A=0x40000000, Q=0x50000000, R=0x60000000, m=300, n=129,
                                                   lda=300, ldq=300, ldr=129))
    ws = lib.cqr2_batched_workspace_size(probs, 2, 0)
    assert ws > 0 and ws % 256 == 0
    assert lib.cqr2_batched_workspace_size(probs, 2, 1) == 0            # FP64 only
    assert ws > lib.cqr2_batched_workspace_size(probs, 1, 0) > 0
    W = ctypes.c_void_p(0x70000000)
    f = lib.cqr2_factor_batched
    assert f(probs, -1, W, ws, 0, NULL) == -2
    assert f(probs, 0, W, ws, 0, NULL) == 0                               # nothing to do
    assert f(probs, 2, W, ws, 1, NULL) == -5
    assert f(probs, 2, NULL, ws, 0, NULL) == -3
    assert f(probs, 2, ctypes.c_void_p(0x70000008), ws, 0, NULL) == -3  # not 256-byte aligned
    assert f(probs, 2, W, ws - 1, 0, NULL) == -4
    bad = (cq.Problem * 2)(_problem(), _problem(lda=5))
    assert f(bad, 2, W, ws, 0, NULL) == -1
    assert lib.cqr2_batched_workspace_size(bad, 2, 0) == 0


def test_server_argument_errors():
    lib = cq.load()
    h = ctypes.c_void_p()
    assert lib.cqr2_server_create(0, 0, 8, NULL, ctypes.byref(h)) == -1
    assert lib.cqr2_server_create(1 << 20, 0, 0, NULL, ctypes.byref(h)) == -3
    assert lib.cqr2_server_create(1 << 20, 0, 5000, NULL, ctypes.byref(h)) == -3
    assert lib.cqr2_server_create(1 << 20, 0, 8, NULL, None) == -5
    assert lib.cqr2_server_submit(NULL, ctypes.byref(_problem()), 0) == -1
    assert lib.cqr2_server_step(NULL, None, None) == -1
    assert lib.cqr2_server_clock(NULL) == -1
    assert lib.cqr2_server_destroy(NULL) == -1


def test_lstsq_argument_errors():
    lib = cq.load()
    f = lib.cqr2_lstsq
    A, B, X = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x1000000), ctypes.c_void_p(0x2000000)
    Q, R, W = ctypes.c_void_p(0x3000000), ctypes.c_void_p(0x4000000), ctypes.c_void_p(0x5000000)
    ws = lib.cqr2_lstsq_workspace_size(100, 10, 2)
    assert ws > lib.cqr2_workspace_size(100, 10, 0) and ws % 256 == 0
    assert lib.cqr2_lstsq_workspace_size(10, 20, 1) == 0
    ok = dict(A=A, m=100, n=10, lda=100, B=B, ldb=100, k=2, X=X, ldx=10, Q=Q, ldq=100, R=R, ldr=10, W=W, wb=ws,
              info=NULL)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["A"], a["m"], a["n"], a["lda"], a["B"], a["ldb"], a["k"], a["X"], a["ldx"], a["Q"], a["ldq"],
                 a["R"], a["ldr"], a["W"], a["wb"], a["info"], NULL)

    assert call(n=-1) == -3
    assert call(m=5) == -2
    assert call(ldb=99) == -6
    assert call(k=-1) == -7
    assert call(ldx=9) == -9
    assert call(ldq=99) == -11
    assert call(ldr=9) == -13
    assert call(B=NULL) == -5
    assert call(X=ctypes.c_void_p(0x10000 + 8)) == -8          # X overlaps A
    assert call(R=ctypes.c_void_p(0x3000000 + 8)) == -12       # R overlaps Q
    assert call(W=ctypes.c_void_p(0x5000008)) == -14
    assert call(wb=ws - 1) == -15
    assert call(info=ctypes.c_void_p(0x6000002)) == -16


def test_inverse_depth_flags():
    lib = cq.load()
    d = cq.CQR2_INVERSE_DEPTH
    ws0 = lib.cqr2_workspace_size(5000, 600, 0)
    # the block substitution's m x (widest block) buffer is added on the tiled path
    assert lib.cqr2_workspace_size(5000, 600, d(1)) > ws0
    assert lib.cqr2_workspace_size(5000, 600, d(cq.CQR2_MAX_INVERSE_DEPTH)) > ws0
    # no recursion level at n <= 128: the flag changes nothing there
    assert lib.cqr2_workspace_size(5000, 100, d(2)) == lib.cqr2_workspace_size(5000, 100, 0)
    assert lib.cqr2_workspace_size(5000, 600, d(cq.CQR2_MAX_INVERSE_DEPTH + 1)) == 0
    assert lib.cqr2_workspace_size(5000, 600, d(1) | cq.CQR2_MIXED_P1_FP32) == 0
    assert lib.cqr2_workspace_size(5000, 600, d(1) | cq.CQR2_SHIFTED_CQR3) == 0
    f = lib.cqr2_factor_ex
    W = ctypes.c_void_p(0x40000000)
    for flags in (d(9), d(1) | 1, d(2) | 2, 3 | d(1)):
        assert f(FAKE, 100, 10, 100, FAKE2, 100, ctypes.c_void_p(0x30000000), 10, W, 1 << 30, NULL, flags,
                 NULL) == -12
