"""GPU parity at the edges of the size range: d = 1 (A = C: every row kept,
m = n), where every alias class is a single bin, and the smallest lengths
n = 2^6, 2^7 for every d.  Operators, ISTA and ADMM iterates against the
dense FP64 oracle (Alg. 1 and Alg. 2 with A written out) and at a larger
size against the FFT oracle; the objective trace against the oracle's
objective.
Tolerances as in the other parity tests: relative l2 1e-4 per iterate,
1e-5 per trace entry, operators to the FP32 transform error."""
import numpy as np
import pytest

import workloads
from oracle import dense, fftref, problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")
IT_TOL = 1e-4
F_TOL = 1e-5


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def square():
    pr = problem.build(workloads.signal(4096, 1, 40, 4242))
    return pr, pr.A()


@pytest.mark.parametrize("n", [256, 4096, 1 << 16, 1 << 21])
def test_square_operators(n):
    rng = np.random.default_rng(n)
    c = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    op = fftref.Operator(c.astype(np.float64), 1)
    y = h(cs.circ_apply(g(c), 1, g(x)))
    xt = h(cs.circ_apply_T(g(c), 1, g(x)))
    assert rel(y, op.A(x.astype(np.float64))) <= 1e-5
    assert rel(xt, op.AT(x.astype(np.float64))) <= 1e-5


def test_square_dense_operator_matches(square):
    pr, A = square
    x = pr.x_true.astype(np.float64)
    assert A.shape == (4096, 4096)
    assert rel(h(cs.circ_apply(g(pr.c), 1, g(pr.x_true))), A @ x) <= 1e-5


def test_square_ista_iterates(square):
    pr, A = square
    y = pr.y.astype(np.float64)
    T = 100
    _, hist = dense.ista(A, y, float(pr.lam), float(pr.tau), T, record=True)
    for t in (1, 2, 5, 25, 100):
        got = h(cs.ista_solve(g(pr.c), 1, g(pr.y), pr.lam, pr.tau, t))
        assert rel(got, hist[t - 1]) <= IT_TOL, t


def test_square_admm_iterates(square):
    pr, A = square
    y = pr.y.astype(np.float64)
    rho, T = 1.0, 100
    _, hist = dense.admm(A, y, float(pr.lam), rho, T, record=True)
    for t in (1, 2, 5, 25, 100):
        got = [h(v) for v in cs.admm_solve(g(pr.c), 1, g(pr.y), pr.lam, rho, t)]
        for name, a_, b_ in zip("xzu", got, hist[t - 1]):
            assert rel(a_, b_) <= IT_TOL, (t, name)


def test_square_traces(square):
    pr, A = square
    y = pr.y.astype(np.float64)
    lam, tau, T = float(pr.lam), float(pr.tau), 60
    _, hi = dense.ista(A, y, lam, tau, T, record=True)
    _, ha = dense.admm(A, y, lam, 0.5, T, record=True)
    oi, oa = torch.empty(T, device=DEV), torch.empty(T, device=DEV)
    cs.ista_solve(g(pr.c), 1, g(pr.y), pr.lam, pr.tau, T, obj=oi)
    cs.admm_solve(g(pr.c), 1, g(pr.y), pr.lam, 0.5, T, obj=oa)
    ri = np.array([dense.objective(A, y, lam, x) for x in hi])
    ra = np.array([dense.objective(A, y, lam, r[0]) for r in ha])
    assert np.max(np.abs(h(oi) - ri) / ri) <= F_TOL
    assert np.max(np.abs(h(oa) - ra) / ra) <= F_TOL


def test_square_large_first_iterates():
    """n = 2^20, d = 1: the first iterates against the FFT oracle."""
    pr = problem.build(workloads.signal(1 << 20, 1, 2000, 77))
    op = pr.op()
    y = pr.y.astype(np.float64)
    _, hist = fftref.ista(op, y, float(pr.lam), float(pr.tau), 5, record=True)
    for t in (1, 2, 5):
        got = h(cs.ista_solve(g(pr.c), 1, g(pr.y), pr.lam, pr.tau, t))
        assert rel(got, hist[t - 1][1]) <= IT_TOL, t
    _, ha = fftref.admm(op, y, float(pr.lam), 1.0, 5, record=True)
    got = [h(v) for v in cs.admm_solve(g(pr.c), 1, g(pr.y), pr.lam, 1.0, 5)]
    for name, a_, b_ in zip("xzu", got, ha[-1][1:]):
        assert rel(a_, b_) <= IT_TOL, name


def test_square_persistent_path_unsupported(square):
    """d = 1 runs on the two-launch schedule; asking for the persistent one
    is refused rather than silently rerouted."""
    pr, _ = square
    cs.set_solver_path(cs.PATH_PERSISTENT)
    try:
        with pytest.raises(cs.CsError):
            cs.ista_solve(g(pr.c), 1, g(pr.y), pr.lam, pr.tau, 5)
    finally:
        cs.set_solver_path(cs.PATH_AUTO)
    cs.check_device()


@pytest.mark.parametrize("n,d", [(64, 1), (64, 2), (64, 4), (64, 16), (128, 1), (128, 4), (128, 8), (128, 16)])
def test_smallest_sizes(n, d):
    """n = 2^6 and 2^7 (8-point rows, 4-point columns): operators, ISTA and
    ADMM iterates against the dense oracle."""
    pr = problem.build(workloads.signal(n, d, 3, 31 * n + d))
    A = pr.A()
    x = pr.x_true.astype(np.float64)
    assert rel(h(cs.circ_apply(g(pr.c), d, g(pr.x_true))), A @ x) <= 1e-5
    r = pr.y.astype(np.float64)
    assert rel(h(cs.circ_apply_T(g(pr.c), d, g(pr.y))), A.T @ r) <= 1e-5
    _, hi = dense.ista(A, r, float(pr.lam), float(pr.tau), 50, record=True)
    _, ha = dense.admm(A, r, float(pr.lam), 1.0, 50, record=True)
    for t in (1, 5, 50):
        assert rel(h(cs.ista_solve(g(pr.c), d, g(pr.y), pr.lam, pr.tau, t)), hi[t - 1]) <= IT_TOL, t
        got = [h(v) for v in cs.admm_solve(g(pr.c), d, g(pr.y), pr.lam, 1.0, t)]
        for name, a_, b_ in zip("xzu", got, ha[t - 1]):
            assert rel(a_, b_) <= IT_TOL, (t, name)


@pytest.mark.timeout(900)
def test_largest_size():
    """n = 2^26, d = 4 (4096-point columns in 4-column blocks): operators,
    the first ISTA and ADMM iterates and their trace entries against the FFT
    oracle."""
    pr = problem.build(workloads.signal(1 << 26, 4, 1 << 16, 2026))
    op = pr.op()
    y = pr.y.astype(np.float64)
    c, yg = g(pr.c), g(pr.y)
    assert rel(h(cs.circ_apply(c, 4, g(pr.x_true))), op.A(pr.x_true.astype(np.float64))) <= 1e-5
    assert rel(h(cs.circ_apply_T(c, 4, yg)), op.AT(y)) <= 1e-5
    lam, tau = float(pr.lam), float(pr.tau)
    _, hi = fftref.ista(op, y, lam, tau, 2, record=True)
    obj = torch.empty(2, device=DEV)
    x = h(cs.ista_solve(c, 4, yg, pr.lam, pr.tau, 2, obj=obj))
    assert rel(x, hi[-1][1]) <= IT_TOL
    ref = [fftref.objective(op, y, lam, v) for _, v in hi]
    assert np.max(np.abs(h(obj) - ref) / ref) <= F_TOL
    _, ha = fftref.admm(op, y, lam, 1.0, 2, record=True)
    got = [h(v) for v in cs.admm_solve(c, 4, yg, pr.lam, 1.0, 2)]
    for name, a_, b_ in zip("xzu", got, ha[-1][1:]):
        assert rel(a_, b_) <= IT_TOL, name
    cs.check_device()
