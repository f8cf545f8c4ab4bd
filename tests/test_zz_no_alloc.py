"""The allocation-free ISTA entry point (cs_ista_solve_noalloc) against the
allocating one (cs_ista_solve), both called through the C ABI on the same
inputs: two calls in a row, the second with a smaller input; the size limit
is enforced before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import workloads
from oracle import problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402
from paper_1707_02244_amd import _lib  # noqa: E402

DEV = torch.device("cuda:0")


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)


def case(n, d, k, seed, iters):
    pr = problem.build(workloads.signal(n, d, k, seed))
    c, y = g(pr.c), g(pr.y)
    lib = cs.load()
    x_ref = torch.empty(n, device=DEV)
    x_na = torch.full((n,), 7.0, device=DEV)
    assert lib.cs_ista_solve(P(c), n, d, P(y), float(pr.lam), float(pr.tau), iters, P(x_ref), None,
                             stream()) == _lib.CS_OK, lib.cs_last_error()
    assert lib.cs_ista_solve_noalloc(P(c), n, d, P(y), float(pr.lam), float(pr.tau), iters, P(x_na),
                                     stream()) == _lib.CS_OK, lib.cs_last_error()
    torch.cuda.synchronize()
    cs.check_device()
    a = x_na.cpu().numpy().astype(np.float64)
    b = x_ref.cpu().numpy().astype(np.float64)
    e = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    print("noalloc n=%d d=%d iters=%d: rel diff to cs_ista_solve %.2e" % (n, d, iters, e))
    assert e <= 1e-6, e
    return e


def test_noalloc_matches_allocating_entry_point_two_calls():
    # two calls in a row on the shared scratch array, the second smaller
    case(1 << 20, 4, 1 << 12, 11, 60)
    case(1 << 12, 8, 32, 12, 80)
    # and back to a mid size (twiddles of another n rewritten in place)
    case(1 << 16, 2, 256, 13, 40)


def test_noalloc_rejects_sizes_beyond_its_limit():
    lib = cs.load()
    n = 1 << 21
    c = torch.zeros(n, device=DEV)
    y = torch.zeros(n // 4, device=DEV)
    x = torch.zeros(n, device=DEV)
    st = lib.cs_ista_solve_noalloc(P(c), n, 4, P(y), 0.1, 0.1, 5, P(x), stream())
    assert st == _lib.CS_EINVAL
    assert b"allocation-free" in lib.cs_last_error()
