"""Pins for the circulant ADMM oracle with a random row set (Section 4.3,
Alg. 3): the two inverses B and D against dense solves, the FFT form
against the dense form, a closed form for the first iterates with C = I,
and the limit against the LASSO optimality conditions and against Alg. 2 on
the same A.  Planted mistakes in the update must fail."""
import numpy as np
import pytest

import workloads
from oracle import cpadmm, dense


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _instance(n=256, m=128, k=6, seed=3, alpha_frac=0.05):
    sig, omega = workloads.random_rows_signal(n, m, k, seed)
    c = sig.c.astype(np.float64)
    A = cpadmm.dense_A(c, omega)
    y = A @ sig.x_true.astype(np.float64)
    alpha = alpha_frac * float(np.max(np.abs(A.T @ y)))
    return c, omega, y, alpha, A


def test_B_is_diagonal_in_frequency():
    rng = np.random.default_rng(1)
    n, rho, sigma = 128, 0.7, 0.3
    c = rng.standard_normal(n)
    q = rng.standard_normal(n)
    C = dense.dense_C(c)
    ref = np.linalg.solve(rho * C.T @ C + sigma * np.eye(n), q)
    assert _rel(cpadmm._FFT(c, rho, sigma).B(q), ref) < 1e-12


def test_D_diagonal():
    n, rho = 64, 0.4
    omega = np.array([0, 3, 7, 20, 41, 63])
    P = np.zeros((len(omega), n))
    P[np.arange(len(omega)), omega] = 1.0
    ref = np.linalg.inv(P.T @ P + rho * np.eye(n))
    assert np.allclose(np.diag(cpadmm.d_diag(omega, n, rho)), ref, rtol=0, atol=1e-15)
    y = np.arange(1.0, 7.0)
    assert np.array_equal(cpadmm.scatter(omega, y, n), P.T @ y)


def test_fft_form_matches_dense_form():
    c, omega, y, alpha, _ = _instance()
    args = (c, omega, y, alpha, 1.3, 0.6, 1.1, 40)
    (_, hd) = cpadmm.dense_cpadmm(*args, record=True)
    (_, hf) = cpadmm.fft_cpadmm(*args, record=True)
    for a, b in zip(hd, hf):
        for p, q in zip(a[1:], b[1:]):
            assert _rel(q, p) < 1e-11 or np.linalg.norm(p) == 0


def check_first_iterates(run):
    """c = e0 (C = I): from zeros, x(1) = 0, v(1) = D P^T y, z(1) = 0,
    mu(1) = tau v(1), nu(1) = 0; then x(2) = rho (1 + tau) v(1) / (rho + sigma)."""
    n = 16
    c = np.zeros(n)
    c[0] = 1.0
    omega = np.array([1, 4, 9, 15])
    y = np.array([2.0, -1.0, 0.5, 3.0])
    alpha, rho, sigma, tau = 0.1, 0.5, 0.25, 0.8
    (_, h) = run(c, omega, y, alpha, rho, sigma, tau, 2, record=True)
    v1 = cpadmm.scatter(omega, y, n) / (1.0 + rho)
    t1, x1, vv1, z1, mu1, nu1 = h[0]
    assert np.all(x1 == 0) and np.all(z1 == 0) and np.all(nu1 == 0)
    assert np.allclose(vv1, v1, rtol=0, atol=1e-15) and np.allclose(mu1, tau * v1, rtol=0, atol=1e-15)
    x2 = rho * (1.0 + tau) * v1 / (rho + sigma)
    assert np.allclose(h[1][1], x2, rtol=0, atol=1e-14)


def test_first_iterates_closed_form():
    check_first_iterates(cpadmm.dense_cpadmm)
    check_first_iterates(cpadmm.fft_cpadmm)


def check_limit(run, iters=6000):
    """The limit solves the LASSO for A = P C (random rows): the optimality
    conditions hold, and z equals the limit of Alg. 2 on the same A."""
    c, omega, y, alpha, A = _instance()
    (x, v, z, mu, nu) = run(c, omega, y, alpha, 1.0, 1.0, 1.0, iters)
    g = A.T @ (y - A @ z)
    on = z != 0
    assert np.all(np.abs(g[~on]) <= alpha * (1 + 1e-6))
    assert np.all(np.abs(g[on] - alpha * np.sign(z[on])) <= alpha * 1e-6)
    _, zz, _ = dense.admm(A, y, alpha, 1.0, 6000)
    assert _rel(z, zz) < 1e-6
    assert _rel(x, z) < 1e-6


def test_limit_is_the_lasso_minimiser():
    check_limit(cpadmm.fft_cpadmm)


def test_every_dth_row_gives_alg2_problem():
    """Omega = rows 0, d, 2d, ...: the same LASSO as Alg. 2 with the
    decimating P, so both limits agree."""
    n, d = 256, 4
    sig = workloads.signal(n, d, 5, 9)
    c = sig.c.astype(np.float64)
    omega = np.arange(0, n, d)
    A = dense.dense_A(c, d)
    assert np.array_equal(A, cpadmm.dense_A(c, omega))
    y = A @ sig.x_true.astype(np.float64)
    alpha = 0.05 * float(np.max(np.abs(A.T @ y)))
    (_, _, z, _, _) = cpadmm.fft_cpadmm(c, omega, y, alpha, 1.0, 1.0, 1.0, 6000)
    _, zz, _ = dense.admm(A, y, alpha, 1.0, 6000)
    assert _rel(z, zz) < 1e-6


# planted mistakes ------------------------------------------------------------
def _mut_no_mu_in_x(c, omega, y, alpha, rho, sigma, tau, iters, record=False):
    """Alg. 3's x-update read literally (C^T v, the multiplier not folded in)."""
    op = cpadmm._FFT(c, rho, sigma)
    n = op.n
    py, dd = cpadmm.scatter(omega, y, n), cpadmm.d_diag(omega, n, rho)
    x = v = z = mu = nu = np.zeros(n)
    hist = []
    for t in range(iters):
        x = op.B(rho * op.T(v) + sigma * (z - nu))
        cx = op(x)
        v = dd * (rho * cx - rho * mu + py)
        z = dense.soft(x + nu, alpha / sigma)
        mu = mu + tau * (v - cx)
        nu = nu + tau * (x - z)
        hist.append((t + 1, x, v, z, mu, nu))
    return ((x, v, z, mu, nu), hist) if record else (x, v, z, mu, nu)


def _mut_D_without_rho(c, omega, y, alpha, rho, sigma, tau, iters, record=False):
    """D = (P^T P)^{-1} on Omega, rho^{-1} elsewhere (1 in place of 1 + rho)."""
    orig = cpadmm.d_diag
    try:
        def bad(om, n, r):
            dd = np.full(n, 1.0 / r)
            dd[np.asarray(om)] = 1.0
            return dd
        cpadmm.d_diag = bad
        return cpadmm.fft_cpadmm(c, omega, y, alpha, rho, sigma, tau, iters, record)
    finally:
        cpadmm.d_diag = orig


def _mut_mu_sign(c, omega, y, alpha, rho, sigma, tau, iters, record=False):
    return cpadmm.fft_cpadmm(c, omega, y, alpha, rho, sigma, -tau, iters, record)


@pytest.mark.parametrize("mut", [_mut_no_mu_in_x, _mut_D_without_rho, _mut_mu_sign])
def test_planted_mistakes_fail(mut):
    with pytest.raises(AssertionError):
        check_first_iterates(mut)
        check_limit(mut, iters=3000)
