"""GPU edge cases: the largest supported n (two-launch schedule only), closed
forms of degenerate operators, the smallest sizes, and the batched solver's
degenerate inputs."""
import numpy as np
import pytest

import workloads
from oracle import fftref, problem

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
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.mark.parametrize("n,d", [(1 << 25, 4), (1 << 24, 2), (1 << 24, 16), (1 << 23, 4)])
def test_largest_n_operator_and_first_iterates(n, d):
    """n = 2^23 .. 2^25: beyond the persistent solver's range, so the
    two-launch schedule runs (4096-point rows at 2^23 and 2^24 with 512
    threads, 8192-point rows and 2048-point columns with 1024 at 2^25; d = 2
    and 4 hold three or more classes per row-pass thread, d = 16 fewer);
    operators and the first ISTA / ADMM iterates against the FFT oracle."""
    rng = np.random.default_rng(n.bit_length() * 100 + d)
    m = n // d
    c = (rng.standard_normal(n) / np.sqrt(m)).astype(np.float32)
    x = np.zeros(n, np.float32)
    k = n >> 10
    x[rng.choice(n, k, replace=False)] = rng.standard_normal(k)
    op = fftref.Operator(c.astype(np.float64), d)
    yref = op.A(x.astype(np.float64))
    cg = g(c)
    y = h(cs.circ_apply(cg, d, g(x)))
    assert rel(y, yref) <= 1e-5
    y32 = yref.astype(np.float32)
    r = h(cs.circ_apply_T(cg, d, g(y32)))
    assert rel(r, op.AT(y32.astype(np.float64))) <= 1e-5
    lam = np.float32(0.01 * np.abs(r).max())
    tau = np.float32(1.0 / op.max_chat_sq())
    _, hist = fftref.ista(op, y32.astype(np.float64), float(lam), float(tau), 2, record=True)
    for t in (1, 2):
        xt = h(cs.ista_solve(cg, d, g(y32), lam, tau, t))
        assert rel(xt, hist[t - 1][1]) <= 1e-4, t
    (xa, za, ua) = fftref.admm(op, y32.astype(np.float64), float(lam), 1.0, 1)
    x1, z1, u1 = (h(v) for v in cs.admm_solve(cg, d, g(y32), lam, 1.0, 1))
    assert rel(x1, xa) <= 1e-4 and rel(z1, za) <= 1e-4


@pytest.mark.parametrize("path", ["two_pass", "persistent"])
@pytest.mark.parametrize("d", [2, 4, 16])
def test_identity_generator_closed_form(path, d):
    """c = e0 makes A = P (plain decimation) with c_hat = 1 and tau = 1: ISTA
    reaches x = soft(P^T y, lam) in one step and stays there; ADMM's x-update
    is (P^T y + rho (z - u)) / (1 + rho) on kept samples and z - u elsewhere."""
    n = 4096
    c = np.zeros(n, np.float32)
    c[0] = 1.0
    rng = np.random.default_rng(d)
    y = rng.standard_normal(n // d).astype(np.float32)
    lam = np.float32(0.3)
    up = np.zeros(n)
    up[::d] = y
    want = np.sign(up) * np.maximum(np.abs(up) - lam, 0.0)
    cs.set_solver_path(cs.PATH_TWO_PASS if path == "two_pass" else cs.PATH_PERSISTENT)
    try:
        for T in (1, 7):
            x = h(cs.ista_solve(g(c), d, g(y), lam, 1.0, T))
            assert np.max(np.abs(x - want)) <= 1e-6 * np.abs(up).max(), T
        # ADMM, one step from zero: x = P^T y / (1 + rho), z = soft(x, lam / rho)
        rho = np.float32(0.5)
        x1, z1, u1 = (h(v) for v in cs.admm_solve(g(c), d, g(y), lam, rho, 1))
        xw = up / (1.0 + float(rho))
        zw = np.sign(xw) * np.maximum(np.abs(xw) - float(lam) / float(rho), 0.0)
        assert np.max(np.abs(x1 - xw)) <= 1e-6 * np.abs(up).max()
        assert np.max(np.abs(z1 - zw)) <= 1e-6 * np.abs(up).max()
        cs.check_device()
    finally:
        cs.set_solver_path(cs.PATH_AUTO)


@pytest.mark.parametrize("n,d", [(256, 2), (256, 16), (512, 8)])
def test_smallest_sizes_both_schedules(n, d):
    pr = problem.build(workloads.signal(n, d, 3, 60 + n + d))
    A = pr.A()
    from oracle import dense
    y = pr.y.astype(np.float64)
    _, hist = dense.ista(A, y, float(pr.lam), float(pr.tau), 30, record=True)
    for path in (cs.PATH_TWO_PASS, cs.PATH_PERSISTENT):
        cs.set_solver_path(path)
        try:
            x = h(cs.ista_solve(g(pr.c), d, g(pr.y), pr.lam, pr.tau, 30))
        finally:
            cs.set_solver_path(cs.PATH_AUTO)
        assert rel(x, hist[-1]) <= 1e-4
    cs.check_device()


def test_batched_degenerate_inputs():
    """No signals; one signal; zero iterations (x = 0)."""
    d = 4
    empty = torch.empty(0, device=DEV)
    cs.ista_solve_batched(np.zeros(0, np.int64), d, empty, empty, empty, empty, 10, empty)
    sig = workloads.signal(1 << 12, d, 16, 5)
    pr = problem.build(sig)
    ns = np.array([sig.n], np.int64)
    lam = g(np.array([pr.lam])); tau = g(np.array([pr.tau]))
    x = torch.full((sig.n,), 3.0, device=DEV)
    cs.ista_solve_batched(ns, d, g(pr.c), g(pr.y), lam, tau, 0, x)
    assert float(h(x).max()) == 0.0
    cs.ista_solve_batched(ns, d, g(pr.c), g(pr.y), lam, tau, 25, x)
    ref = h(cs.ista_solve(g(pr.c), d, g(pr.y), pr.lam, pr.tau, 25))
    assert rel(h(x), ref) <= 1e-5
    cs.check_device()
