"""Circulant ADMM with a random row selection (Section 4.3, Alg. 3) in the
FP64 oracle (test infrastructure).

The sensing matrix is A = P C: C is the n x n circulant with first column c,
P keeps the rows in Omega (any set of m indices, drawn at random in the
paper).  Section 4.3 splits the LASSO as

    min 1/2 ||y - P v||^2 + alpha ||z||_1   s.t.  v = C x,  z = x

and forms the augmented Lagrangian

    L = 1/2 ||y - P v||^2 + alpha ||z||_1 + sigma nu^T (x - z)
        + sigma/2 ||x - z||^2 + rho mu^T (v - C x) + rho/2 ||v - C x||^2.

Minimising L in x, then in (v, z) (separable given x), then moving the
scaled multipliers mu, nu along the constraint residuals gives, from
mu = nu = z = v = 0 (the paper's initial condition):

    x(t)  = B (rho C^T (v(t-1) + mu(t-1)) + sigma (z(t-1) - nu(t-1))),
            B = (rho C^T C + sigma I)^{-1}
    v(t)  = D (rho C x(t) - rho mu(t-1) + P^T y),   D = (P^T P + rho I)^{-1}
    z(t)  = eta_{alpha/sigma}(x(t) + nu(t-1))
    mu(t) = mu(t-1) + tau (v(t) - C x(t))
    nu(t) = nu(t-1) + tau (x(t) - z(t))

with tau in (0, (1 + sqrt 5)/2) (the convergence range the paper quotes).
Readings of the printed algorithm (each derived from L above):

* The x-update needs C^T (v + mu); Alg. 3 writes C^T v and ends each
  iteration with "v = v + mu", i.e. it stores v + mu in v.  Here v and mu
  are kept apart and v + mu is formed where the x-update needs it.
* D: P^T P + rho I is diagonal with 1 + rho on Omega and rho elsewhere (the
  text prints "P^T P - rho I" and calls both matrices circulant).
* One step size tau for both multipliers (tau_1 = tau_2).
* The per-work-item listings that follow Alg. 3 disagree with it on the
  multiplier updates; the derivation from L is followed instead.

`dense_*` build C, B and D as explicit matrices (B by a dense solve) for
small n; `fft_*` apply C, C^T and B through numpy's FFT (C and B are
circulant, diagonalised by the DFT); the tests pin one against the other.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import dense


def scatter(omega, y, n):
    """P^T y: y placed at the rows in Omega, zeros elsewhere."""
    out = np.zeros(n)
    out[np.asarray(omega)] = np.asarray(y, np.float64)
    return out


def d_diag(omega, n, rho):
    """The diagonal of D = (P^T P + rho I)^{-1}: 1/(1 + rho) on Omega, 1/rho
    elsewhere."""
    dd = np.full(n, 1.0 / rho)
    dd[np.asarray(omega)] = 1.0 / (1.0 + rho)
    return dd


def _iterate(Cop, CTop, Bop, omega, y, alpha, rho, sigma, tau, iters, record, callback=None):
    n = Cop.n
    py = scatter(omega, y, n)
    dd = d_diag(omega, n, rho)
    x = np.zeros(n)
    v = np.zeros(n)
    z = np.zeros(n)
    mu = np.zeros(n)
    nu = np.zeros(n)
    hist = []
    for t in range(1, iters + 1):
        x = Bop(rho * CTop(v + mu) + sigma * (z - nu))
        cx = Cop(x)
        v = dd * (rho * cx - rho * mu + py)
        z = dense.soft(x + nu, alpha / sigma)
        mu = mu + tau * (v - cx)
        nu = nu + tau * (x - z)
        if record:
            hist.append((t, x.copy(), v.copy(), z.copy(), mu.copy(), nu.copy()))
        if callback is not None:
            callback(t, x, v, z, mu, nu)
    out = (x, v, z, mu, nu)
    return (out, hist) if record else out


class _Dense:
    def __init__(self, c, rho, sigma):
        self.C = dense.dense_C(c)
        self.n = self.C.shape[0]
        M = rho * self.C.T @ self.C + sigma * np.eye(self.n)
        self.fac = scipy.linalg.cho_factor(M)

    def __call__(self, x):
        return self.C @ x

    def T(self, v):
        return self.C.T @ v

    def B(self, q):
        return scipy.linalg.cho_solve(self.fac, q)


def dense_cpadmm(c, omega, y, alpha, rho, sigma, tau, iters, record=False, callback=None):
    """Alg. 3 with explicit C and a Cholesky factor of rho C^T C + sigma I
    (n up to a few thousand).  Returns (x, v, z, mu, nu) after `iters`."""
    op = _Dense(np.asarray(c, np.float64), rho, sigma)
    return _iterate(op, op.T, op.B, omega, y, alpha, rho, sigma, tau, iters, record, callback)


class _FFT:
    def __init__(self, c, rho, sigma):
        c = np.asarray(c, np.float64)
        self.n = c.shape[0]
        self.chat = np.fft.rfft(c)
        self.binv = 1.0 / (rho * np.abs(self.chat) ** 2 + sigma)   # eigenvalues of B

    def __call__(self, x):
        return np.fft.irfft(self.chat * np.fft.rfft(x), self.n)

    def T(self, v):
        return np.fft.irfft(np.conj(self.chat) * np.fft.rfft(v), self.n)

    def B(self, q):
        return np.fft.irfft(self.binv * np.fft.rfft(q), self.n)


def fft_cpadmm(c, omega, y, alpha, rho, sigma, tau, iters, record=False, callback=None):
    """Alg. 3 with C, C^T and B applied through the FFT (any n)."""
    op = _FFT(c, rho, sigma)
    return _iterate(op, op.T, op.B, omega, y, alpha, rho, sigma, tau, iters, record, callback)


def dense_A(c, omega):
    """A = P C for the rows in Omega (in the order given)."""
    return dense.dense_C(c)[np.asarray(omega)]


def problem(sig, omega, alpha_frac):
    """The rounded problem of a random-row draw: y = P C x* in FP64 rounded
    to float32, alpha = alpha_frac max |A^T y| in FP64 on the rounded y,
    rounded to float32 (the same rule as the decimating problem)."""
    c = np.asarray(sig.c, np.float64)
    op = _FFT(c, 1.0, 1.0)
    y = op(np.asarray(sig.x_true, np.float64))[np.asarray(omega)].astype(np.float32)
    aty = op.T(scatter(omega, y.astype(np.float64), len(c)))
    alpha = np.float32(alpha_frac * float(np.max(np.abs(aty))))
    return y, alpha


def objective(c, omega, y, alpha, x):
    """1/2 ||y - P C x||^2 + alpha ||x||_1 through the FFT."""
    op = _FFT(c, 1.0, 1.0)
    r = np.asarray(y, np.float64) - op(x)[np.asarray(omega)]
    return 0.5 * float(r @ r) + alpha * float(np.abs(x).sum())
