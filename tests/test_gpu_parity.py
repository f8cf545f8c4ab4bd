"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (derivation in the design notes):
  * operators (one forward and one inverse n-point FP32 FFT): relative l2
    error <= 1e-5, max-abs error <= 5e-5 * max |reference|;
  * solver iterates: relative l2 error <= 1e-4 for every compared iterate;
  * final objective, evaluated in FP64 by the oracle on both iterates:
    relative difference <= 1e-5.
"""
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
OP_TOL = 1e-5
IT_TOL = 1e-4
OBJ_TOL = 1e-5


@pytest.fixture(params=["two_pass", "persistent"])
def path(request):
    """Run a solver test under both schedules (two launches per iteration, or
    one persistent cooperative launch), then check the device error flag."""
    cs.set_solver_path(cs.PATH_TWO_PASS if request.param == "two_pass" else cs.PATH_PERSISTENT)
    yield request.param
    cs.check_device()
    cs.set_solver_path(cs.PATH_AUTO)


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check_elementwise(got, ref, tol=OP_TOL):
    assert rel(got, ref) <= tol, rel(got, ref)
    assert np.max(np.abs(got - ref)) <= 5 * tol * max(np.max(np.abs(ref)), 1e-30)


# ----------------------------------------------------------------------------
# Operators A x, A^T r, the norm bound
# ----------------------------------------------------------------------------
OP_CASES = [(256, 2), (256, 16), (1024, 4), (4096, 4), (4096, 8), (8192, 16), (1 << 16, 4), (1 << 17, 2)]


@pytest.mark.parametrize("n,d", OP_CASES)
def test_circ_apply_and_transpose(n, d):
    rng = np.random.default_rng(n * 31 + d)
    m = n // d
    c = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    r = rng.standard_normal(m).astype(np.float32)
    if n <= 8192:
        A = dense.dense_A(c.astype(np.float64), d)
        y_ref, xt_ref = A @ x.astype(np.float64), A.T @ r.astype(np.float64)
    else:
        op = fftref.Operator(c.astype(np.float64), d)
        y_ref, xt_ref = op.A(x.astype(np.float64)), op.AT(r.astype(np.float64))
    y = h(cs.circ_apply(g(c), d, g(x)))
    xt = h(cs.circ_apply_T(g(c), d, g(r)))
    check_elementwise(y, y_ref)
    check_elementwise(xt, xt_ref)
    # adjoint identity in FP32
    lhs, rhs = float(y @ r.astype(np.float64)), float(x.astype(np.float64) @ xt)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(y) * np.linalg.norm(r)


@pytest.mark.parametrize("n", [256, 4096, 1 << 20])
def test_norm_bound(n):
    rng = np.random.default_rng(n)
    c = rng.standard_normal(n).astype(np.float32)
    ref = fftref.Operator(c.astype(np.float64), 1).max_chat_sq()
    got = float(h(cs.circ_norm_bound(g(c)))[0])
    assert abs(got - ref) <= 1e-5 * ref


def test_apply_structured_inputs():
    """Delta input: C e_j is c shifted by j (first column convention)."""
    n, d = 4096, 4
    rng = np.random.default_rng(5)
    c = rng.standard_normal(n).astype(np.float32)
    x = np.zeros(n, np.float32)
    x[7] = 1.0
    y = h(cs.circ_apply(g(c), d, g(x)))
    ref = np.roll(c.astype(np.float64), 7)[::d]
    check_elementwise(y, ref)
    # zero input gives exact zeros
    assert np.all(h(cs.circ_apply(g(c), d, g(np.zeros(n)))) == 0.0)


# ----------------------------------------------------------------------------
# Solvers at the parity configuration (n = 4096, m = 1024, d = 4, k = 40)
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def parity_signal():
    pr = problem.build(workloads.parity_signal())
    A = pr.A()
    return pr, A


def test_ista_per_iterate_parity_signal(parity_signal, path):
    pr, A = parity_signal
    y = pr.y.astype(np.float64)
    lam, tau = float(pr.lam), float(pr.tau)
    _, hist = dense.ista(A, y, lam, tau, 100, record=True)
    c, yg = g(pr.c), g(pr.y)
    worst = 0.0
    for t in range(1, 101):
        x = h(cs.ista_solve(c, pr.d, yg, pr.lam, pr.tau, t))
        e = rel(x, hist[t - 1])
        worst = max(worst, e)
        assert e <= IT_TOL, (t, e)
    print("ista parity_signal worst per-iterate rel err (t<=100): %.3e" % worst)


def test_ista_final_objective_parity_signal(parity_signal, path):
    pr, A = parity_signal
    y = pr.y.astype(np.float64)
    lam, tau = float(pr.lam), float(pr.tau)
    T = workloads.PARITY_PARAMS["ista_iters"]
    xo = dense.ista(A, y, lam, tau, T)
    x = h(cs.ista_solve(g(pr.c), pr.d, g(pr.y), pr.lam, pr.tau, T))
    fo, fg = dense.objective(A, y, lam, xo), dense.objective(A, y, lam, x)
    assert abs(fg - fo) <= OBJ_TOL * fo, (fg, fo)
    assert rel(x, xo) <= IT_TOL


def test_admm_per_iterate_parity_signal(parity_signal, path):
    pr, A = parity_signal
    y = pr.y.astype(np.float64)
    lam = float(pr.lam)
    rho = workloads.PARITY_PARAMS["rho"]
    _, hist = dense.admm(A, y, lam, rho, 100, record=True)
    c, yg = g(pr.c), g(pr.y)
    worst = 0.0
    for t in range(1, 101):
        x, z, u = (h(v) for v in cs.admm_solve(c, pr.d, yg, pr.lam, rho, t))
        ex, ez, eu = rel(x, hist[t - 1][0]), rel(z, hist[t - 1][1]), rel(u, hist[t - 1][2])
        worst = max(worst, ex, ez)
        assert ex <= IT_TOL and ez <= IT_TOL, (t, ex, ez)
        assert eu <= 10 * IT_TOL, (t, eu)
    print("admm parity_signal worst per-iterate rel err (t<=100): %.3e" % worst)


def test_admm_final_objective_parity_signal(parity_signal, path):
    pr, A = parity_signal
    y = pr.y.astype(np.float64)
    lam = float(pr.lam)
    rho = workloads.PARITY_PARAMS["rho"]
    T = workloads.PARITY_PARAMS["admm_iters"]
    (xo, zo, uo) = dense.admm(A, y, lam, rho, T)
    x, z, u = (h(v) for v in cs.admm_solve(g(pr.c), pr.d, g(pr.y), pr.lam, rho, T))
    fo, fg = dense.objective(A, y, lam, zo), dense.objective(A, y, lam, z)
    assert abs(fg - fo) <= OBJ_TOL * fo, (fg, fo)
    assert rel(z, zo) <= IT_TOL and rel(x, xo) <= IT_TOL


# ----------------------------------------------------------------------------
# Other decimations and sizes (dense oracle), ADMM with rho != 1
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n,d,k", [(256, 2, 4), (512, 16, 3), (2048, 8, 12), (8192, 4, 60)])
def test_solvers_other_shapes(n, d, k, path):
    pr = problem.build(workloads.signal(n, d, k, 100 + n + d))
    A = pr.A()
    y = pr.y.astype(np.float64)
    lam, tau = float(pr.lam), float(pr.tau)
    c, yg = g(pr.c), g(pr.y)
    for T in (1, 7, 40):
        xo = dense.ista(A, y, lam, tau, T)
        assert rel(h(cs.ista_solve(c, d, yg, pr.lam, pr.tau, T)), xo) <= IT_TOL
    rho = 2.5
    for T in (1, 7, 40):
        (xo, zo, uo) = dense.admm(A, y, lam, rho, T)
        x, z, u = (h(v) for v in cs.admm_solve(c, d, yg, pr.lam, rho, T))
        assert rel(x, xo) <= IT_TOL and rel(z, zo) <= IT_TOL


# ----------------------------------------------------------------------------
# Degenerate and edge cases
# ----------------------------------------------------------------------------
def test_zero_iterations(path):
    n, d = 4096, 4
    c = g(np.ones(n))
    y = g(np.ones(n // d))
    x = g(np.full(n, 3.0))
    cs.ista_solve(c, d, y, 0.1, 0.1, 0, x=x)
    assert np.all(h(x) == 0.0)
    x, z, u = g(np.full(n, 3.0)), g(np.full(n, 4.0)), g(np.full(n, 5.0))
    cs.admm_solve(c, d, y, 0.1, 1.0, 0, x=x, z=z, u=u)
    assert np.all(h(x) == 0.0) and np.all(h(z) == 0.0) and np.all(h(u) == 0.0)
    x, z, u = g(np.full(n, 3.0)), g(np.full(n, 4.0)), g(np.full(n, 5.0))
    cs.admm_solve(c, d, y, 0.1, 1.0, 0, x=x, z=z, u=u, warm=True)
    assert np.all(h(z) == 4.0) and np.all(h(u) == 5.0)


def test_lambda_at_lam_max_gives_zero(parity_signal, path):
    pr, A = parity_signal
    lmax = problem.lam_max(pr.c, pr.d, pr.y)
    lam = np.float32(lmax * 1.001)
    x = h(cs.ista_solve(g(pr.c), pr.d, g(pr.y), lam, pr.tau, 20))
    assert np.count_nonzero(x) == 0


def test_lambda_zero_is_least_squares_gradient(parity_signal, path):
    """lam = 0: one ISTA step from 0 is tau A^T y exactly (no threshold)."""
    pr, A = parity_signal
    x = h(cs.ista_solve(g(pr.c), pr.d, g(pr.y), 0.0, pr.tau, 1))
    ref = float(pr.tau) * (A.T @ pr.y.astype(np.float64))
    check_elementwise(x, ref)


def test_admm_warm_start_continues(parity_signal, path):
    pr, A = parity_signal
    c, yg = g(pr.c), g(pr.y)
    x20, z20, u20 = (h(v) for v in cs.admm_solve(c, pr.d, yg, pr.lam, 1.0, 20))
    x, z, u = cs.admm_solve(c, pr.d, yg, pr.lam, 1.0, 10)
    x, z, u = cs.admm_solve(c, pr.d, yg, pr.lam, 1.0, 10, x=x, z=z, u=u, warm=True)
    assert rel(h(z), z20) <= 1e-6 and rel(h(u), u20) <= 1e-6 and rel(h(x), x20) <= 1e-6


def test_deterministic(parity_signal, path):
    pr, A = parity_signal
    c, yg = g(pr.c), g(pr.y)
    a = h(cs.ista_solve(c, pr.d, yg, pr.lam, pr.tau, 50))
    b = h(cs.ista_solve(c, pr.d, yg, pr.lam, pr.tau, 50))
    assert np.array_equal(a, b)
    a = [h(v) for v in cs.admm_solve(c, pr.d, yg, pr.lam, 1.0, 30)]
    b = [h(v) for v in cs.admm_solve(c, pr.d, yg, pr.lam, 1.0, 30)]
    assert all(np.array_equal(p, q) for p, q in zip(a, b))


def test_bad_arguments_on_device():
    n, d = 4096, 4
    c = g(np.ones(n))
    with pytest.raises(cs.CsError):
        cs.ista_solve(c, d, g(np.ones(n // d)), -1.0, 0.1, 5)
    with pytest.raises(cs.CsError):
        cs.admm_solve(c, d, g(np.ones(n // d)), 0.1, 0.0, 5)
    with pytest.raises(ValueError):
        cs.circ_apply(c, d, g(np.ones(n - 1)))


# ----------------------------------------------------------------------------
# Full size (n = 2^22, m = 2^20, d = 4), the benchmark's launch configuration
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def large_signal():
    pr = problem.build(workloads.large_signal())
    return pr, pr.op()


def test_large_signal_ista_first_iterates(large_signal, path):
    pr, op = large_signal
    y = pr.y.astype(np.float64)
    lam, tau = float(pr.lam), float(pr.tau)
    _, hist = fftref.ista(op, y, lam, tau, 3, record=True)
    c, yg = g(pr.c), g(pr.y)
    for t in (1, 2, 3):
        x = h(cs.ista_solve(c, pr.d, yg, pr.lam, pr.tau, t))
        assert rel(x, hist[t - 1][1]) <= IT_TOL, t


def test_large_signal_admm_first_iterates(large_signal, path):
    pr, op = large_signal
    y = pr.y.astype(np.float64)
    lam = float(pr.lam)
    _, hist = fftref.admm(op, y, lam, 1.0, 3, record=True)
    c, yg = g(pr.c), g(pr.y)
    for t in (1, 2, 3):
        x, z, u = (h(v) for v in cs.admm_solve(c, pr.d, yg, pr.lam, 1.0, t))
        assert rel(x, hist[t - 1][1]) <= IT_TOL and rel(z, hist[t - 1][2]) <= IT_TOL, t


def test_large_signal_operator_full_size(large_signal):
    pr, op = large_signal
    y = h(cs.circ_apply(g(pr.c), pr.d, g(pr.x_true)))
    check_elementwise(y, pr.y.astype(np.float64), tol=OP_TOL)


def test_large_signal_full_run_objective_decreases(large_signal, path):
    """At the benchmark's iteration counts the oracle cannot follow every
    iterate; the GPU iterates must still drive the FP64 objective down
    monotonically (ISTA with tau <= 1/||A||^2 cannot increase it)."""
    pr, op = large_signal
    y = pr.y.astype(np.float64)
    lam = float(pr.lam)
    c, yg = g(pr.c), g(pr.y)
    f = [fftref.objective(op, y, lam, np.zeros(pr.n))]
    for T in (10, 50, workloads.LARGE_PARAMS["ista_iters"]):
        f.append(fftref.objective(op, y, lam, h(cs.ista_solve(c, pr.d, yg, pr.lam, pr.tau, T))))
    assert all(b < a for a, b in zip(f, f[1:])), f
    x, z, u = cs.admm_solve(c, pr.d, yg, pr.lam, 1.0, workloads.LARGE_PARAMS["admm_iters"])
    fz = fftref.objective(op, y, lam, h(z))
    assert fz < f[1]


def test_paths_agree(parity_signal):
    """The persistent launch and the two-launch schedule run the same
    arithmetic in the same order: their iterates agree to FP32 round-off."""
    pr, A = parity_signal
    c, yg = g(pr.c), g(pr.y)
    out = {}
    for p in (cs.PATH_TWO_PASS, cs.PATH_PERSISTENT):
        cs.set_solver_path(p)
        out[p] = (h(cs.ista_solve(c, pr.d, yg, pr.lam, pr.tau, 60)),
                  [h(v) for v in cs.admm_solve(c, pr.d, yg, pr.lam, 1.0, 40)])
    cs.check_device()
    cs.set_solver_path(cs.PATH_AUTO)
    a, b = out[cs.PATH_TWO_PASS], out[cs.PATH_PERSISTENT]
    assert rel(b[0], a[0]) <= 1e-6
    assert all(rel(q, p) <= 1e-6 for p, q in zip(a[1], b[1]))
