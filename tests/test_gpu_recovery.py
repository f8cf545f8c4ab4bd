"""The recovery-time study (Section 6) on the GPU against the FP64 oracle:
n = 2^15, m = n/2, k = n/10, lambda = 1e-4, target MSE 1e-4.  At several
iteration counts the GPU iterate (ISTA x, ADMM z, circulant-ADMM z) matches
the oracle's to relative l2 1e-4 up to t = 100 (the per-iterate gate) and
1e-3 beyond; its MSE = ||x - x*||^2 / n then differs from the oracle's by at
most (2 ||e|| ||delta|| + ||delta||^2) / n with e the oracle's error x - x*
and ||delta|| <= tol ||x||, which the test checks; and whether the target is met
agrees wherever the oracle's MSE is farther from the target than that bound."""
import numpy as np
import pytest

import workloads
from oracle import cpadmm, fftref, problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")
PRM = workloads.RECOVERY_PARAMS
IT_TOL = 1e-4     # per-iterate gate for t <= 100
LONG_TOL = 1e-3   # t > 100: FP32 round-off accumulates along the slow directions
                  # (measured up to 1e-4 at t = 2500 for the circulant ADMM)


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def mse(a, b):
    return float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))


def check(tag, t, got, ref, truth):
    """Iterate parity and the MSE bound it implies (see the module text)."""
    got = np.asarray(got, np.float64)
    nr = np.linalg.norm(ref)
    tol = IT_TOL if t <= 100 else LONG_TOL
    e_it = float(np.linalg.norm(got - ref) / nr)
    mg, mo = mse(got, truth), mse(ref, truth)
    dmax = tol * nr
    bound = (2.0 * np.linalg.norm(ref - truth) * dmax + dmax * dmax) / len(ref)
    print("%s t=%d: iterate rel err %.2e, MSE %.4e (oracle %.4e, bound on the difference %.1e)"
          % (tag, t, e_it, mg, mo, bound))
    assert e_it <= tol, (tag, t, e_it)
    assert abs(mg - mo) <= bound, (tag, t, mg, mo, bound)
    if abs(mo - PRM["target_mse"]) > bound:
        assert (mg <= PRM["target_mse"]) == (mo <= PRM["target_mse"]), (tag, t)


@pytest.fixture(scope="module")
def setup():
    sig = workloads.recovery_signal()
    pr = problem.build(sig, 0.01)
    return sig, pr


@pytest.mark.timeout(600)
def test_admm_reaches_target_like_the_oracle(setup):
    sig, pr = setup
    checks = [100, 500, 1000, 1100, 1200]
    ref = {}

    def cb(t, x, z, u):
        if t in checks:
            ref[t] = z.copy()
    fftref.admm(pr.op(), pr.y.astype(np.float64), PRM["lam"], PRM["rho"], max(checks), callback=cb)
    c, y = g(pr.c), g(pr.y)
    for t in checks:
        z = cs.admm_solve(c, pr.d, y, PRM["lam"], PRM["rho"], t)[1].cpu().numpy()
        check("ADMM", t, z, ref[t], sig.x_true)
    assert mse(ref[max(checks)], sig.x_true) <= PRM["target_mse"]


@pytest.mark.timeout(600)
def test_ista_mse_like_the_oracle(setup):
    sig, pr = setup
    checks = [10, 100, 1000, 3000]
    ref = {}

    def cb(t, x):
        if t in checks:
            ref[t] = x.copy()
    fftref.ista(pr.op(), pr.y.astype(np.float64), PRM["lam"], PRM["ista_tau"], max(checks), callback=cb)
    c, y = g(pr.c), g(pr.y)
    for t in checks:
        x = cs.ista_solve(c, pr.d, y, PRM["lam"], PRM["ista_tau"], t).cpu().numpy()
        check("ISTA", t, x, ref[t], sig.x_true)


@pytest.mark.timeout(600)
def test_cpadmm_mse_like_the_oracle():
    sig, omega = workloads.recovery_random_rows()
    y, _ = cpadmm.problem(sig, omega, 0.01)
    checks = [10, 100, 1000, 2500]
    ref = {}

    def cb(t, x, v, z, mu, nu):
        if t in checks:
            ref[t] = z.copy()
    cpadmm.fft_cpadmm(sig.c.astype(np.float64), omega, y.astype(np.float64), PRM["lam"], PRM["rho"], PRM["sigma"],
                      PRM["cp_tau"], max(checks), callback=cb)
    for t in checks:
        z = cs.cpadmm_solve(g(sig.c), omega, g(y), PRM["lam"], PRM["rho"], PRM["sigma"], PRM["cp_tau"], t)[2]
        check("CPADMM", t, z.cpu().numpy(), ref[t], sig.x_true)
