"""GPU parity of the direct (FFT-free) products y = A x and x = A^T r against
the FP64 oracle, through the C ABI.

Each output is one FP32 inner product accumulated in input order, so its
rounding error grows with the number of nonzero terms: about u sqrt(n)
relative for dense random inputs (u = 2^-24; 5e-6 at n = 8192), far less for
the sparse signals of the workloads.  Tolerances: relative l2 <= 1e-4 for
dense inputs, 1e-5 for sparse ones, and agreement with the FFT path within
the sum of both paths' tolerances.
"""
import numpy as np
import pytest

import workloads
from oracle import problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# m < outputs per workgroup, several input tiles, every decimation
DENSE_CASES = [(256, 2), (512, 16), (2048, 8), (8192, 4), (4096, 2), (8192, 16)]


@pytest.mark.parametrize("n,d", DENSE_CASES)
def test_direct_vs_dense_oracle(n, d):
    pr = problem.build(workloads.signal(n, d, max(2, n // 256), 900 + n + d))
    A = pr.A()
    rng = np.random.default_rng(n + d)
    x = rng.standard_normal(n).astype(np.float32)
    r = rng.standard_normal(n // d).astype(np.float32)
    c = g(pr.c)
    y = h(cs.circ_apply_direct(c, d, g(x)))
    xt = h(cs.circ_apply_T_direct(c, d, g(r)))
    assert rel(y, A @ x.astype(np.float64)) <= 1e-4
    assert rel(xt, A.T @ r.astype(np.float64)) <= 1e-4


@pytest.mark.parametrize("n,d", [(1 << 16, 4), (1 << 16, 2), (1 << 17, 16)])
def test_direct_sparse_vs_fft_oracle(n, d):
    """Workload-like inputs (sparse x, its measurements y) against the FP64
    FFT oracle, and against the FFT path on the GPU."""
    pr = problem.build(workloads.signal(n, d, n // 256, 950 + d))
    op = pr.op()
    c, xg = g(pr.c), g(pr.x_true)
    y = h(cs.circ_apply_direct(c, d, xg))
    assert rel(y, op.A(pr.x_true.astype(np.float64))) <= 1e-5
    assert rel(y, h(cs.circ_apply(c, d, xg))) <= 2e-5
    r = pr.y.astype(np.float32)
    xt = h(cs.circ_apply_T_direct(c, d, g(r)))
    assert rel(xt, op.AT(r.astype(np.float64))) <= 1e-4
    assert rel(xt, h(cs.circ_apply_T(c, d, g(r)))) <= 1.1e-4


def test_direct_adjoint_identity():
    n, d = 1 << 14, 8
    rng = np.random.default_rng(3)
    c = g(rng.standard_normal(n) / np.sqrt(n // d))
    x = rng.standard_normal(n)
    r = rng.standard_normal(n // d)
    lhs = float(np.dot(h(cs.circ_apply_direct(c, d, g(x))), r.astype(np.float32)))
    rhs = float(np.dot(x.astype(np.float32), h(cs.circ_apply_T_direct(c, d, g(r)))))
    assert abs(lhs - rhs) <= 1e-4 * max(abs(lhs), 1.0)


def test_direct_impulse_gives_generator_samples():
    """A e_0 = (c_0, c_d, c_2d, ...); A^T e_0 = (c_0, c_{n-1}, ..., c_1)."""
    n, d = 1024, 4
    c_np = np.arange(1, n + 1, dtype=np.float32) / n
    c = g(c_np)
    e = np.zeros(n, np.float32)
    e[0] = 1.0
    y = h(cs.circ_apply_direct(c, d, g(e)))
    assert np.array_equal(y, c_np[::d].astype(np.float64))
    e1 = np.zeros(n // d, np.float32)
    e1[0] = 1.0
    xt = h(cs.circ_apply_T_direct(c, d, g(e1)))
    assert np.array_equal(xt, c_np[(-np.arange(n)) % n].astype(np.float64))


def test_direct_bad_arguments():
    c = g(np.ones(1024))
    with pytest.raises(cs.CsError):
        cs.circ_apply_direct(c, 3, g(np.ones(1024)), g(np.ones(341)))
    with pytest.raises(cs.CsError):
        cs.circ_apply_T_direct(g(np.ones(1000)), 4, g(np.ones(250)))


def test_direct_headline_size():
    """The products the direct baseline times (n = 2^22, m = 2^20, d = 4, the
    headline's c, x and y) against the FP64 FFT oracle, every output.  FP32
    accumulation in input order of N terms errs by about u sqrt(N) relative
    (u = 2^-24): N = 2^14 nonzeros of x for A x, N = m for A^T y; the bound
    is three times that."""
    pr = problem.build(workloads.large_signal())
    n, d = pr.n, pr.d
    op = pr.op()
    c = g(pr.c)
    u = 2.0 ** -24
    y = h(cs.circ_apply_direct(c, d, g(pr.x_true)))
    k = int(np.count_nonzero(pr.x_true))
    assert rel(y, op.A(pr.x_true.astype(np.float64))) <= 3 * u * np.sqrt(k)
    xt = h(cs.circ_apply_T_direct(c, d, g(pr.y)))
    assert rel(xt, op.AT(pr.y.astype(np.float64))) <= 3 * u * np.sqrt(n // d)
