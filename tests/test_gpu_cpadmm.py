"""GPU parity of the circulant ADMM with an arbitrary row set (Section 4.3,
Alg. 3) against the FP64 oracle (oracle/cpadmm.py), element by element on the
same float32 inputs: per iterate x, v, z, mu, nu at relative l2 1e-4, the
final objective 1/2 ||y - P C z||^2 + alpha ||z||_1 at 1e-5 (both evaluated by
the oracle in FP64), the closed form of the first iterates for C = I, and the
timed shape (n = 2^22, m = n/2 random rows)."""
import sys
import time

import numpy as np
import pytest

import workloads
from oracle import cpadmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")
IT_TOL = 1e-4
OBJ_TOL = 1e-5
NAMES = ("x", "v", "z", "mu", "nu")


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.abs(a).max())
    return float(np.linalg.norm(a - b) / nb)


def run_gpu(sig, omega, y, alpha, prm, iters):
    out = cs.cpadmm_solve(g(sig.c), omega, g(y), float(alpha), prm["rho"], prm["sigma"], prm["tau"], iters)
    return [h(t) for t in out]


def oracle_hist(sig, omega, y, alpha, prm, iters, keep, tag=None):
    hist = {}
    t0 = time.perf_counter()

    def cb(t, *state):
        if t in keep:
            hist[t] = [s.copy() for s in state]
        if tag and t % 25 == 0:
            print("[oracle %s] t=%d (%.0fs)" % (tag, t, time.perf_counter() - t0), file=sys.stderr, flush=True)
    cpadmm.fft_cpadmm(sig.c.astype(np.float64), omega, y.astype(np.float64), float(alpha), prm["rho"], prm["sigma"],
                      prm["tau"], iters, callback=cb)
    return hist


@pytest.mark.parametrize("n,m,k,seed,rho,sigma,tau", [
    (256, 128, 6, 1, 1.0, 1.0, 1.0),
    (4096, 2048, 40, 2, 1.0, 1.0, 1.0),
    (4096, 1000, 30, 3, 0.7, 0.4, 1.3),
    (1 << 15, 1 << 14, 300, 4, 1.0, 0.5, 1.0),
    (1 << 18, 100000, 2000, 5, 2.0, 1.0, 0.8),
])
def test_cpadmm_iterates_vs_oracle(n, m, k, seed, rho, sigma, tau):
    sig, omega = workloads.random_rows_signal(n, m, k, seed)
    y, alpha = cpadmm.problem(sig, omega, 0.01)
    prm = dict(rho=rho, sigma=sigma, tau=tau)
    checks = [1, 2, 3, 5, 10, 25, 60]
    ref = oracle_hist(sig, omega, y, alpha, prm, max(checks), set(checks))
    worst = 0.0
    for t in checks:
        got = run_gpu(sig, omega, y, alpha, prm, t)
        for name, a, b in zip(NAMES, got, ref[t]):
            e = rel(a, b)
            worst = max(worst, e)
            assert e <= IT_TOL, (n, t, name, e)
    print("cpadmm n=%d m=%d: worst iterate rel err %.2e (t <= %d)" % (n, m, worst, max(checks)))


def test_cpadmm_identity_generator_closed_form():
    """c = e0 (C = I): x(1) = 0, v(1) = D P^T y, z(1) = 0, mu(1) = tau v(1),
    nu(1) = 0; x(2) = rho (1 + tau) v(1) / (rho + sigma)."""
    n = 256
    c = np.zeros(n, np.float32)
    c[0] = 1.0
    omega = np.array([1, 4, 9, 15, 100, 255], np.int64)
    y = np.array([2.0, -1.0, 0.5, 3.0, -0.25, 1.5], np.float32)
    rho, sigma, tau, alpha = 0.5, 0.25, 0.8, 0.1
    sig = workloads.Signal1D(n=n, d=0, k=0, c=c, x_true=np.zeros(n, np.float32), support=np.zeros(0, np.int64))
    prm = dict(rho=rho, sigma=sigma, tau=tau)
    x1, v1, z1, mu1, nu1 = run_gpu(sig, omega, y, alpha, prm, 1)
    py = cpadmm.scatter(omega, y.astype(np.float64), n)
    v1_ref = py / (1.0 + rho)
    # x(1) = 0 exactly (the transforms of zero spectra); v(1) and mu(1) are
    # time-domain products of the inputs; x(2) passes through two FP32
    # transforms: the operators' tolerance (relative l2 1e-5, largest error
    # 5e-5 of the largest entry)
    assert not x1.any() and not z1.any() and not nu1.any()
    assert np.allclose(v1, v1_ref, rtol=1e-6, atol=0)
    assert np.allclose(mu1, tau * v1_ref, rtol=1e-6, atol=0)
    x2 = run_gpu(sig, omega, y, alpha, prm, 2)[0]
    x2_ref = rho * (1.0 + tau) * v1_ref / (rho + sigma)
    assert rel(x2, x2_ref) <= 1e-5
    assert np.abs(x2 - x2_ref).max() <= 5e-5 * np.abs(x2_ref).max()


def test_cpadmm_zero_iterations():
    sig, omega = workloads.random_rows_signal(1024, 300, 5, 8)
    y, alpha = cpadmm.problem(sig, omega, 0.01)
    out = run_gpu(sig, omega, y, alpha, dict(rho=1.0, sigma=1.0, tau=1.0), 0)
    assert all(not a.any() for a in out)


def test_cpadmm_rejects_repeated_rows():
    sig, omega = workloads.random_rows_signal(1024, 300, 5, 9)
    y, alpha = cpadmm.problem(sig, omega, 0.01)
    bad = omega.copy()
    bad[1] = bad[0]
    with pytest.raises(cs.CsError):
        cs.cpadmm_solve(g(sig.c), bad, g(y), float(alpha), 1.0, 1.0, 1.0, 5)


@pytest.mark.timeout(900)
def test_cpadmm_timed_shape():
    """n = 2^22, m = n/2 random rows, k = n/10 (the random-row workload the
    benchmark times): iterates at t = 1, 2, 5, 10, 25, 50, 100 and the final
    objective on z(100)."""
    prm = workloads.RANDOM_ROWS_PARAMS
    sig, omega = workloads.random_rows_large()
    y, alpha = cpadmm.problem(sig, omega, prm["alpha_frac"])
    T = prm["iters"]
    checks = [1, 2, 5, 10, 25, 50, T]
    ref = oracle_hist(sig, omega, y, alpha, prm, T, set(checks), tag="n=2^22 CPADMM")
    worst = 0.0
    for t in checks:
        got = run_gpu(sig, omega, y, alpha, prm, t)
        for name, a, b in zip(NAMES, got, ref[t]):
            e = rel(a, b)
            worst = max(worst, e)
            assert e <= IT_TOL, (t, name, e)
    zg, zo = got[2], ref[T][2]
    c64, y64 = sig.c.astype(np.float64), y.astype(np.float64)
    fg = cpadmm.objective(c64, omega, y64, float(alpha), zg)
    fo = cpadmm.objective(c64, omega, y64, float(alpha), zo)
    ef = abs(fg - fo) / fo
    print("cpadmm n=2^22: worst iterate rel err %.2e (t <= %d), F(z(%d)) rel err %.2e" % (worst, T, T, ef))
    assert ef <= OBJ_TOL
