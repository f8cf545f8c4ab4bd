"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_1707_02244_amd as cs
from paper_1707_02244_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cscirc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cs2?_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_declares_expected_calls():
    syms = declared_symbols()
    for name in ["cs_circ_apply", "cs_circ_apply_T", "cs_ista_solve", "cs_admm_solve"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = cs.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == declared_symbols()


def test_version():
    assert cs.version() >= 100


NULL = ctypes.c_void_p(0)
FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every case below fails validation first


@pytest.mark.parametrize("n,d", [(0, 4), (100, 4), (32, 4), (1 << 27, 4), (4096, 3), (4096, 6),
                                 (4096, 32), (4096, 0), (4096, -4)])
def test_bad_sizes_rejected(n, d):
    lib = cs.load()
    st = lib.cs_circ_apply(FAKE, n, d, FAKE, FAKE, NULL)
    assert st == _lib.CS_EINVAL
    assert lib.cs_last_error()
    st = lib.cs_ista_solve(FAKE, n, d, FAKE, 0.1, 0.1, 5, FAKE, NULL, NULL)
    assert st == _lib.CS_EINVAL


def test_unrolled_rejects_square_operator():
    """d = 1 is a valid operator and solver size, but the unrolled solver
    takes d >= 2: rejected before anything is enqueued."""
    lib = cs.load()
    assert lib.cs_unrolled_ista_fwd(FAKE, 4096, 1, 2, FAKE, FAKE, FAKE, 5, 0, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert b"d >= 2" in lib.cs_last_error()


def test_unrolled_rejects_largest_size():
    """n = 2^26 is a valid operator and solver size; the unrolled solver
    takes n <= 2^25."""
    lib = cs.load()
    assert lib.cs_unrolled_ista_fwd(FAKE, 1 << 26, 4, 2, FAKE, FAKE, FAKE, 5, 0, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert b"2^25" in lib.cs_last_error()


@pytest.mark.parametrize("n,L,same", [(4096, 0, False), (4096, -3, False), (256, 257, False), (1 << 14, 4097, False),
                                      (4096, 5, True), (1000, 5, False), (32, 5, False)])
def test_box_blur_generator_bad_arguments(n, L, same):
    """The C B generator validates n, the order L and aliasing on the host,
    before anything is enqueued."""
    lib = cs.load()
    out = FAKE if same else ctypes.c_void_p(0x2000)
    assert lib.cs_box_blur_generator(FAKE, n, L, out, NULL) == _lib.CS_EINVAL
    assert lib.cs_last_error()
    assert lib.cs_box_blur_generator(NULL, 4096, 5, out, NULL) == _lib.CS_EINVAL
    assert lib.cs_box_blur_generator(FAKE, 4096, 5, NULL, NULL) == _lib.CS_EINVAL


def test_direct_products_reject_small_n():
    """n = 2^6 and 2^7 are valid for the FFT operators but not for the direct
    products (n >= 2^8)."""
    lib = cs.load()
    assert lib.cs_circ_apply_direct(FAKE, 128, 4, FAKE, FAKE, NULL) == _lib.CS_EINVAL
    assert b"n >= 256" in lib.cs_last_error()


def test_null_pointers_rejected():
    lib = cs.load()
    assert lib.cs_circ_apply(NULL, 4096, 4, FAKE, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_circ_apply(FAKE, 4096, 4, NULL, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_circ_apply_T(FAKE, 4096, 4, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert lib.cs_circ_norm_bound(FAKE, 4096, NULL, NULL) == _lib.CS_EINVAL
    assert lib.cs_ista_solve(FAKE, 4096, 4, NULL, 0.1, 0.1, 5, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert lib.cs_admm_solve(FAKE, 4096, 4, FAKE, 0.1, 1.0, 5, 0, FAKE, NULL, FAKE, NULL, NULL) == _lib.CS_EINVAL


@pytest.mark.parametrize("lam,tau,iters", [(-1.0, 0.1, 5), (0.1, 0.0, 5), (0.1, -1.0, 5), (0.1, 0.1, -1),
                                           (float("nan"), 0.1, 5), (0.1, float("inf"), 5)])
def test_bad_ista_scalars_rejected(lam, tau, iters):
    lib = cs.load()
    assert lib.cs_ista_solve(FAKE, 4096, 4, FAKE, lam, tau, iters, FAKE, NULL, NULL) == _lib.CS_EINVAL


@pytest.mark.parametrize("lam,rho,iters", [(-1.0, 1.0, 5), (0.1, 0.0, 5), (0.1, -2.0, 5), (0.1, 1.0, -3),
                                           (0.1, float("nan"), 5)])
def test_bad_admm_scalars_rejected(lam, rho, iters):
    lib = cs.load()
    assert lib.cs_admm_solve(FAKE, 4096, 4, FAKE, lam, rho, iters, 0, FAKE, FAKE, FAKE, NULL, NULL) == _lib.CS_EINVAL


def test_objective_trace_arguments_checked_first():
    """With a trace requested, argument errors are still reported before any
    device work."""
    lib = cs.load()
    assert lib.cs_ista_solve(FAKE, 4096, 4, FAKE, 0.1, 0.1, -1, FAKE, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_admm_solve(FAKE, 4096, 4, FAKE, 0.1, -1.0, 5, 0, FAKE, FAKE, FAKE, FAKE, NULL) == _lib.CS_EINVAL


def test_timing_read_unknown_name():
    lib = cs.load()
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    assert lib.cs_timing_read(b"no_such_kernel", ctypes.byref(n), ctypes.byref(ms)) == _lib.CS_EINVAL


def test_package_has_no_oracle_dependency():
    """The product package never imports the oracle."""
    pkg = os.path.dirname(cs.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(root, f)).read()
                assert "oracle" not in text.lower(), f


@pytest.mark.parametrize("rows,cols", [(8, 64), (64, 8), (48, 64), (64, 8192), (16384, 64)])
def test_bad_2d_shapes_rejected(rows, cols):
    lib = cs.load()
    assert lib.cs2_apply(FAKE, NULL, rows, cols, FAKE, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs2_admm_solve(FAKE, NULL, rows, cols, FAKE, 0.1, 1.0, 5, 0, FAKE, FAKE, FAKE, NULL, NULL) == _lib.CS_EINVAL


def test_bad_2d_arguments_rejected():
    lib = cs.load()
    assert lib.cs2_apply(NULL, NULL, 64, 64, FAKE, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs2_apply(FAKE, NULL, 64, 64, NULL, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs2_ista_solve(FAKE, NULL, 64, 64, FAKE, -1.0, 0.1, 5, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert lib.cs2_ista_solve(FAKE, NULL, 64, 64, FAKE, 0.1, 0.0, 5, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert lib.cs2_admm_solve(FAKE, NULL, 64, 64, FAKE, 0.1, 0.0, 5, 0, FAKE, FAKE, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert lib.cs2_admm_solve(FAKE, NULL, 64, 64, FAKE, 0.1, 1.0, -2, 0, FAKE, FAKE, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert b"rows" in lib.cs_last_error() or b"iters" in lib.cs_last_error()


@pytest.mark.parametrize("n,d", [(1000, 4), (4096, 3), (4096, 1), (128, 2)])
def test_direct_products_reject_bad_sizes(n, d):
    """The direct products validate like the FFT operators: nothing is
    enqueued for a size the library does not support."""
    lib = _lib.load()
    assert lib.cs_circ_apply_direct(FAKE, n, d, FAKE, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_circ_apply_T_direct(FAKE, n, d, FAKE, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_last_error() != b""


def test_direct_products_reject_null_pointers():
    lib = _lib.load()
    assert lib.cs_circ_apply_direct(NULL, 4096, 4, FAKE, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_circ_apply_direct(FAKE, 4096, 4, NULL, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_circ_apply_direct(FAKE, 4096, 4, FAKE, NULL, NULL) == _lib.CS_EINVAL
    assert lib.cs_circ_apply_T_direct(FAKE, 4096, 4, NULL, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_circ_apply_T_direct(FAKE, 4096, 4, FAKE, NULL, NULL) == _lib.CS_EINVAL


def test_workspace_bytes_layout():
    """The block of one (n, d) plan: barrier area (counters and error flag),
    scalars, six twiddle tables, the spectrum buffer and the c_hat and
    y_hat tables, each part rounded up to 64 complex values."""
    lib = cs.load()
    up = lambda v: (v + 63) // 64 * 64
    for n in (64, 256, 4096, 1 << 17, 1 << 22, 1 << 26):
        N = n // 2
        L = N.bit_length() - 1
        N1 = 1 << ((L - 1) // 2) if L % 2 else 1 << (L // 2 - 1)
        N2 = N // N1
        lo = (L + 1) // 2
        bar_words = 256 * 32 + 32
        parts = [up(bar_words // 2), 64, up(N1), up(N2), up(1 << lo), up(N >> lo), up(N1), up(N2),
                 up(N), up(N + 1), up(N + 1)]
        for d in (1, 2, 4, 8, 16):
            for mode in (0, 1, 2):
                assert lib.cs_workspace_bytes(n, d, mode) == 8 * sum(parts)
    assert lib.cs_workspace_bytes(1 << 22, 4, 3) == 0
    assert lib.cs_workspace_bytes(1000, 4, 1) == 0
    assert lib.cs_workspace_bytes(4096, 3, 1) == 0
    assert lib.cs_workspace_bytes(1 << 27, 4, 1) == 0


def test_bad_workspace_rejected():
    lib = cs.load()
    # misaligned: rejected before any device query
    assert lib.cs_set_workspace(ctypes.c_void_p(0x1000 + 8), 1 << 20) == _lib.CS_EINVAL
    assert b"aligned" in lib.cs_last_error()
    # smaller than the smallest plan
    assert lib.cs_set_workspace(ctypes.c_void_p(0x1000), 1024) == _lib.CS_EINVAL
    assert b"smallest" in lib.cs_last_error()


def _arr(vals, ctype):
    a = (ctype * len(vals))(*vals)
    return ctypes.cast(a, ctypes.c_void_p), a


@pytest.mark.parametrize("ns,ds,offs", [
    ([1 << 9], [4], [0]),                  # n below 2^10
    ([1 << 19], [4], [0]),                 # n above 2^18
    ([3000], [4], [0]),                    # not a power of two
    ([4096], [16], [0]),                   # d outside {2, 4, 8}
    ([4096], [3], [0]),
    ([4096, 4096], [4, 4], [0, 1]),        # odd off_n
    ([4096, 4096], [4, 4], [0, 2048]),     # overlapping n-length slices
    ([4096], [4], [-2]),                   # negative offset
])
def test_batched_bad_layout_rejected(ns, ds, offs):
    """The batched calls validate the host arrays (sizes, per-signal
    decimations, offsets, overlap) before any device call."""
    lib = cs.load()
    n_p, n_k = _arr(ns, ctypes.c_int64)
    d_p, d_k = _arr(ds, ctypes.c_int32)
    o_p, o_k = _arr(offs, ctypes.c_int64)
    m_p, m_k = _arr([0] * len(ns), ctypes.c_int64)
    cnt = len(ns)
    assert lib.cs_ista_solve_batched(cnt, n_p, d_p, o_p, m_p, FAKE, FAKE, FAKE, FAKE, 5, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_last_error()
    assert lib.cs_admm_solve_batched(cnt, n_p, d_p, o_p, m_p, FAKE, FAKE, FAKE, FAKE, 5, 0,
                                     FAKE, FAKE, FAKE, NULL) == _lib.CS_EINVAL


def test_batched_null_and_count_checks():
    lib = cs.load()
    n_p, n_k = _arr([4096], ctypes.c_int64)
    d_p, d_k = _arr([4], ctypes.c_int32)
    o_p, o_k = _arr([0], ctypes.c_int64)
    assert lib.cs_ista_solve_batched(-1, n_p, d_p, o_p, o_p, FAKE, FAKE, FAKE, FAKE, 5, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_ista_solve_batched(1, n_p, NULL, o_p, o_p, FAKE, FAKE, FAKE, FAKE, 5, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_ista_solve_batched(1, n_p, d_p, o_p, o_p, FAKE, FAKE, FAKE, FAKE, -1, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_ista_solve_batched(1, n_p, d_p, o_p, o_p, FAKE, FAKE, NULL, FAKE, 5, FAKE, NULL) == _lib.CS_EINVAL
    assert lib.cs_admm_solve_batched(1, n_p, d_p, o_p, o_p, FAKE, FAKE, FAKE, FAKE, 5, 0,
                                     FAKE, NULL, FAKE, NULL) == _lib.CS_EINVAL
    # count = 0 is a no-op, whatever the pointers
    assert lib.cs_ista_solve_batched(0, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 5, NULL, NULL) == _lib.CS_OK
    assert lib.cs_admm_solve_batched(0, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 5, 1,
                                     NULL, NULL, NULL, NULL) == _lib.CS_OK
    assert lib.cs_batched_schedule(None, 0) == _lib.CS_EINVAL


@pytest.mark.parametrize("n,omega,alpha,rho,sigma,tau,iters", [
    (1000, [0, 1], 0.1, 1.0, 1.0, 1.0, 5),           # n not a power of two
    (1 << 23, [0, 1], 0.1, 1.0, 1.0, 1.0, 5),        # n above 2^22
    (128, [0, 1], 0.1, 1.0, 1.0, 1.0, 5),            # n below 2^8 (this call's minimum)
    (4096, [0, 4096], 0.1, 1.0, 1.0, 1.0, 5),        # index out of range
    (4096, [-1, 3], 0.1, 1.0, 1.0, 1.0, 5),
    (4096, [7, 3, 7], 0.1, 1.0, 1.0, 1.0, 5),        # repeated index
    (4096, [1, 2], -0.1, 1.0, 1.0, 1.0, 5),          # alpha < 0
    (4096, [1, 2], 0.1, 0.0, 1.0, 1.0, 5),           # rho <= 0
    (4096, [1, 2], 0.1, 1.0, -1.0, 1.0, 5),          # sigma <= 0
    (4096, [1, 2], 0.1, 1.0, 1.0, 0.0, 5),           # tau <= 0
    (4096, [1, 2], 0.1, 1.0, 1.0, 1.0, -1),          # iters < 0
])
def test_cpadmm_bad_arguments_rejected(n, omega, alpha, rho, sigma, tau, iters):
    """The circulant ADMM with a row set validates sizes, the index set and
    the scalars on the host before any device call."""
    lib = cs.load()
    om = (ctypes.c_int64 * len(omega))(*omega)
    st = lib.cs_cpadmm_solve(FAKE, n, ctypes.cast(om, ctypes.c_void_p), len(omega), FAKE, alpha, rho, sigma, tau,
                             iters, FAKE, FAKE, FAKE, FAKE, FAKE, NULL)
    assert st == _lib.CS_EINVAL
    assert lib.cs_last_error()


def test_cpadmm_null_and_count_rejected():
    lib = cs.load()
    om = (ctypes.c_int64 * 2)(1, 2)
    omp = ctypes.cast(om, ctypes.c_void_p)
    assert lib.cs_cpadmm_solve(FAKE, 4096, NULL, 2, FAKE, 0.1, 1.0, 1.0, 1.0, 5, FAKE, FAKE, FAKE, FAKE, FAKE,
                               NULL) == _lib.CS_EINVAL
    assert lib.cs_cpadmm_solve(FAKE, 4096, omp, 0, FAKE, 0.1, 1.0, 1.0, 1.0, 5, FAKE, FAKE, FAKE, FAKE, FAKE,
                               NULL) == _lib.CS_EINVAL
    assert lib.cs_cpadmm_solve(FAKE, 4096, omp, 2, FAKE, 0.1, 1.0, 1.0, 1.0, 5, FAKE, NULL, FAKE, FAKE, FAKE,
                               NULL) == _lib.CS_EINVAL
