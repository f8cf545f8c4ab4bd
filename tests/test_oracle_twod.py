"""Pins for the 2-D oracle: the dense definition against brute force and
closed forms, the FFT operator against the dense one, Lam against the
eigenvalues of A A^T, Woodbury against a dense solve, a separable kernel
against the Kronecker product of two 1-D operators, and ADMM iterates."""
import numpy as np
import pytest

import workloads
from oracle import dense, fftref, twod


def brute_conv(k, x):
    """Periodic 2-D convolution by explicit loops."""
    n1, n2 = k.shape
    out = np.zeros((n1, n2))
    for i in range(n1):
        for j in range(n2):
            s = 0.0
            for a in range(n1):
                for b in range(n2):
                    s += k[(i - a) % n1, (j - b) % n2] * x[a, b]
            out[i, j] = s
    return out


def rand_case(n1, n2, seed, psf=True):
    rng = np.random.default_rng(seed)
    s = rng.choice([-1.0, 1.0], (n1, n2))
    h = workloads.gaussian_psf(n1, n2, sigma=0.8, half=1) if psf else None
    return s, h, rng


def test_conv_matrix_is_the_convolution():
    rng = np.random.default_rng(3)
    k = rng.standard_normal((4, 6))
    x = rng.standard_normal((4, 6))
    np.testing.assert_allclose(twod.conv_matrix(k) @ x.ravel(), brute_conv(k, x).ravel(), rtol=0, atol=1e-12)


def test_impulse_kernel_is_a_cyclic_shift():
    k = np.zeros((5, 8))
    k[1, 3] = 1.0
    x = np.arange(40.0).reshape(5, 8)
    np.testing.assert_array_equal(twod.conv_matrix(k) @ x.ravel(), np.roll(x, (1, 3), axis=(0, 1)).ravel())


def test_decimation_keeps_the_even_grid():
    x = np.arange(64.0).reshape(8, 8)
    np.testing.assert_array_equal(twod.dec_matrix(8, 8, 2, 2) @ x.ravel(), x[::2, ::2].ravel())


def test_psf_is_normalised_and_symmetric():
    h = workloads.gaussian_psf(32, 32)
    assert abs(h.sum() - 1.0) < 1e-14
    # h(-a, -b) = h(a, b): real, symmetric spectrum
    np.testing.assert_allclose(h, np.roll(h[::-1, ::-1], (1, 1), axis=(0, 1)), atol=1e-15)
    assert np.max(np.abs(np.fft.fft2(h).imag)) < 1e-14


@pytest.mark.parametrize("n1,n2", [(16, 16), (8, 16), (16, 4)])
def test_fft_operator_matches_dense(n1, n2):
    """P16: the FFT operator against the dense 2-D definition (3x3 PSF)."""
    s, h, rng = rand_case(n1, n2, 11)
    A = twod.dense_A2(s, h, 2, 2)
    op = twod.Operator2D(s, h, 2, 2)
    for _ in range(3):
        x = rng.standard_normal(n1 * n2)
        r = rng.standard_normal(op.m)
        np.testing.assert_allclose(op.A(x), A @ x, rtol=0, atol=1e-12 * np.abs(A @ x).max())
        np.testing.assert_allclose(op.AT(r), A.T @ r, rtol=0, atol=1e-12 * np.abs(A.T @ r).max())


def test_lambda_are_the_eigenvalues_of_AAT():
    """P16: Lam (the 2x2 alias average of |g_hat|^2) is the spectrum of A A^T."""
    s, h, _ = rand_case(16, 16, 5)
    A = twod.dense_A2(s, h, 2, 2)
    ev = np.sort(np.linalg.eigvalsh(A @ A.T))
    lam = np.sort(twod.Operator2D(s, h, 2, 2).Lam().ravel())
    assert np.max(np.abs(ev - lam)) <= 1e-12 * ev.max()


def test_separable_kernel_is_a_kronecker_product():
    """s[i, j] = a[i] b[j], no blur: A = A_1(a) kron A_1(b) with the 1-D
    operators of the paper (keep every second row of each circulant)."""
    rng = np.random.default_rng(8)
    a, b = rng.standard_normal(8), rng.standard_normal(16)
    op = twod.Operator2D(np.outer(a, b), None, 2, 2)
    K = np.kron(dense.dense_A(a, 2), dense.dense_A(b, 2))
    x = rng.standard_normal(8 * 16)
    np.testing.assert_allclose(op.A(x), K @ x, rtol=0, atol=1e-12 * np.abs(K @ x).max())


def test_woodbury_matches_dense_solve():
    s, h, rng = rand_case(16, 8, 21)
    A = twod.dense_A2(s, h, 2, 2)
    op = twod.Operator2D(s, h, 2, 2)
    q = rng.standard_normal(op.n)
    for rho in (0.3, 1.0, 4.0):
        ref = np.linalg.solve(A.T @ A + rho * np.eye(op.n), q)
        np.testing.assert_allclose(op.woodbury_solve(rho, q), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_admm_iterates_match_dense():
    s, h, rng = rand_case(16, 16, 2)
    A = twod.dense_A2(s, h, 2, 2)
    op = twod.Operator2D(s, h, 2, 2)
    x = np.zeros(op.n)
    x[rng.choice(op.n, 6, replace=False)] = rng.lognormal(0, 1, 6)
    y = A @ x
    lam = 0.01 * np.abs(A.T @ y).max()
    (xd, zd, ud), hd = dense.admm(A, y, lam, 1.0, 40, record=True)
    (xf, zf, uf), hf = twod.admm(op, y, lam, 1.0, 40, record=True)
    # dense records (x, z, u); the FFT reference records (t, x, z, u)
    for rd, rf in zip(hd, hf):
        assert np.max(np.abs(rd[0] - rf[1])) <= 1e-11 * max(np.abs(rd[0]).max(), 1e-30)
        assert np.max(np.abs(rd[1] - rf[2])) <= 1e-11 * max(np.abs(rd[1]).max(), 1e-30)
    assert np.abs(zf).max() > 0


def test_planted_alias_factor_is_caught():
    """Dropping the 1/(d1 d2) of Lam breaks the eigenvalue pin."""
    s, h, _ = rand_case(16, 16, 5)
    A = twod.dense_A2(s, h, 2, 2)
    ev = np.sort(np.linalg.eigvalsh(A @ A.T))
    op = twod.Operator2D(s, h, 2, 2)
    bad = np.sort((np.abs(op.ghat) ** 2).reshape(2, 8, 2, 8).sum(axis=(0, 2)).ravel())
    assert np.max(np.abs(ev - bad)) > 1e-3 * ev.max()


def test_problem_build_rounding():
    sc = workloads.draw_2d(np.random.default_rng(4), 16, 16, 5, sigma=0.8, half=1)
    pr = twod.build(sc, 0.005)
    op = pr.op()
    assert pr.y.dtype == np.float32 and pr.y.shape == (8, 8)
    y64 = op.A(sc.x_true.astype(np.float64))
    assert np.max(np.abs(pr.y.ravel() - y64)) <= 1e-6 * np.abs(y64).max()
    assert np.float32(0.005 * np.abs(op.AT(pr.y.astype(np.float64).ravel())).max()) == pr.lam
