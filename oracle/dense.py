"""Dense FP64 oracle: the method's definitions written out with an explicit A.

Test infrastructure only (see the package docstring).  Sizes: n up to ~8192
(A is m x n doubles; ADMM factors the n x n matrix A^T A + rho I).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def dense_C(c):
    """Circulant with first column c: C[i, j] = c[(i - j) mod n].

    Section 4.2 defines a circulant by shifts of one generating vector; the
    generator is taken as the first column (reading of the index convention).
    """
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return c[(i - j) % n]


def dense_P(n, d):
    """Row selector P (m x n), P[r, r*d] = 1: keeps every d-th row (Section 4.3,
    partial circulant A = P C with a deterministic, evenly spaced Omega)."""
    m = n // d
    P = np.zeros((m, n))
    P[np.arange(m), np.arange(m) * d] = 1.0
    return P


def dense_A(c, d):
    """A = P C, i.e. A[r, j] = c[(r*d - j) mod n] (Section 4.3)."""
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    m = n // d
    r = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    return c[(r * d - j) % n]


def soft(v, gamma):
    """Soft threshold eta_gamma of Eq. 4: sgn(v)(|v| - gamma) where
    |v| > gamma (strict), 0 otherwise."""
    v = np.asarray(v, dtype=np.float64)
    return np.where(np.abs(v) > gamma, np.sign(v) * (np.abs(v) - gamma), 0.0)


def objective(A, y, lam, x):
    """LASSO objective, Eq. 3 halved: 1/2 ||y - A x||^2 + lam ||x||_1."""
    r = y - A @ x
    return 0.5 * float(r @ r) + lam * float(np.abs(x).sum())


def ista(A, y, lam, tau, iters, record=False):
    """ISTA, Alg. 1: x(0) = 0; r = y - A x; Delta = tau A^T r;
    x = eta_{tau*lam}(x + Delta).  Returns x(iters) and, if record, the list
    of x(1..iters)."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x = np.zeros(A.shape[1])
    hist = []
    for _ in range(iters):
        r = y - A @ x                      # residual
        delta = tau * (A.T @ r)            # gradient step
        x = soft(x + delta, tau * lam)     # soft threshold
        if record:
            hist.append(x.copy())
    return (x, hist) if record else x


def admm(A, y, lam, rho, iters, record=False, x0=None, z0=None, u0=None):
    """ADMM, Alg. 2 (scaled dual u): B = (A^T A + rho I)^-1 (here a Cholesky
    factor of the dense matrix, never formed as an inverse);
      x(t) = B (A^T y + rho (z(t-1) - u(t-1)))
      z(t) = eta_{lam/rho}(x(t) + u(t-1))
      u(t) = u(t-1) + x(t) - z(t)
    with x(0) = z(0) = u(0) = 0 unless a warm start is given.
    Returns (x, z, u) after `iters` steps and, if record, the list of triples.
    """
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = A.shape[1]
    M = A.T @ A + rho * np.eye(n)
    fac = scipy.linalg.cho_factor(M)
    aty = A.T @ y
    x = np.zeros(n) if x0 is None else np.asarray(x0, np.float64).copy()
    z = np.zeros(n) if z0 is None else np.asarray(z0, np.float64).copy()
    u = np.zeros(n) if u0 is None else np.asarray(u0, np.float64).copy()
    hist = []
    for _ in range(iters):
        x = scipy.linalg.cho_solve(fac, aty + rho * (z - u))
        z = soft(x + u, lam / rho)
        u = u + x - z
        if record:
            hist.append((x.copy(), z.copy(), u.copy()))
    return ((x, z, u), hist) if record else (x, z, u)
