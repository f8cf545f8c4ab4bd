"""FFT-based FP64 oracle for sizes where a dense A cannot be stored.

Test infrastructure only (see the package docstring).  Every operator here is
the plain definition evaluated with numpy's FFT as a library primitive:

* C x is the circular convolution of c and x, and the DFT turns circular
  convolution into a pointwise product (Section 4.2: circulants are
  diagonalised by the Fourier matrix);
* P keeps entries 0, d, 2d, ... (time-domain slicing), P^T zero-fills;
* ADMM's (A^T A + rho I)^{-1} is applied with the Woodbury identity
      (A^T A + rho I)^{-1} = rho^{-1} [I - A^T (rho I_m + A A^T)^{-1} A],
  where A A^T = P C C^T P^T is an m x m circulant whose eigenvalues are
      Lam[k'] = (1/d) sum_{l<d} |c_hat[k' + l m]|^2,
  so (rho I + A A^T)^{-1} is a pointwise division in the m-point DFT domain.
  Pinned against a dense solve in the tests.

Agreement with dense.py is a test at n <= 8192.
"""
from __future__ import annotations

import numpy as np


class Operator:
    """A = P C with C's first column c and decimation d (Section 4.3)."""

    def __init__(self, c, d):
        self.c = np.asarray(c, dtype=np.float64)
        self.n = self.c.shape[0]
        self.d = int(d)
        assert self.n % self.d == 0
        self.m = self.n // self.d
        self.chat = np.fft.rfft(self.c)            # half spectrum of c

    # --- the sensing operator and its transpose --------------------------
    def C(self, x):
        """C x: circular convolution of c and x."""
        return np.fft.irfft(self.chat * np.fft.rfft(x), self.n)

    def CT(self, v):
        """C^T v: circular correlation with c (conjugate spectrum)."""
        return np.fft.irfft(np.conj(self.chat) * np.fft.rfft(v), self.n)

    def A(self, x):
        """A x = P C x (Eq. 1)."""
        return self.C(x)[:: self.d]

    def AT(self, r):
        """A^T r = C^T P^T r: zero-fill r onto rows 0, d, 2d, ..., then C^T."""
        up = np.zeros(self.n)
        up[:: self.d] = r
        return self.CT(up)

    # --- spectral quantities ---------------------------------------------
    def full_spectrum(self):
        return np.fft.fft(self.c)

    def Lam(self):
        """Eigenvalues of A A^T in m-point DFT order:
        Lam[k'] = (1/d) sum_l |c_hat[k' + l m]|^2."""
        a = np.abs(self.full_spectrum()) ** 2
        return a.reshape(self.d, self.m).mean(axis=0)

    def max_chat_sq(self):
        """max_k |c_hat[k]|^2 over all n DFT bins: an upper bound on ||A||_2^2."""
        return float(np.max(np.abs(self.full_spectrum()) ** 2))

    def woodbury_solve(self, rho, q):
        """(A^T A + rho I)^{-1} q via Woodbury with the circulant A A^T."""
        Aq = self.A(q)
        t = np.fft.ifft(np.fft.fft(Aq) / (rho + self.Lam())).real
        return (q - self.AT(t)) / rho


def soft(v, gamma):
    """Soft threshold eta_gamma of Eq. 4 (strict '>')."""
    return np.where(np.abs(v) > gamma, np.sign(v) * (np.abs(v) - gamma), 0.0)


def objective(op, y, lam, x):
    """1/2 ||y - A x||^2 + lam ||x||_1 (Eq. 3 halved)."""
    r = y - op.A(x)
    return 0.5 * float(r @ r) + lam * float(np.abs(x).sum())


def ista(op, y, lam, tau, iters, record=False, record_every=1, callback=None):
    """ISTA, Alg. 1, with the operator applied through the FFT:
    x(0)=0; r = y - A x; x = eta_{tau*lam}(x + tau A^T r)."""
    y = np.asarray(y, dtype=np.float64)
    x = np.zeros(op.n)
    hist = []
    for t in range(1, iters + 1):
        r = y - op.A(x)
        x = soft(x + tau * op.AT(r), tau * lam)
        if record and (t % record_every == 0):
            hist.append((t, x.copy()))
        if callback is not None:
            callback(t, x)
    return (x, hist) if record else x


def admm(op, y, lam, rho, iters, record=False, record_every=1,
         x0=None, z0=None, u0=None, callback=None):
    """ADMM, Alg. 2, with B = (A^T A + rho I)^{-1} applied by Woodbury."""
    y = np.asarray(y, dtype=np.float64)
    n = op.n
    aty = op.AT(y)
    x = np.zeros(n) if x0 is None else np.asarray(x0, np.float64).copy()
    z = np.zeros(n) if z0 is None else np.asarray(z0, np.float64).copy()
    u = np.zeros(n) if u0 is None else np.asarray(u0, np.float64).copy()
    hist = []
    for t in range(1, iters + 1):
        x = op.woodbury_solve(rho, aty + rho * (z - u))
        z = soft(x + u, lam / rho)
        u = u + x - z
        if record and (t % record_every == 0):
            hist.append((t, x.copy(), z.copy(), u.copy()))
        if callback is not None:
            callback(t, x, z, u)
    return ((x, z, u), hist) if record else (x, z, u)
