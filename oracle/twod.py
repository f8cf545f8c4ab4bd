"""2-D partial-circulant sensing with a blur (FP64; test infrastructure only).

Model.  An n1 x n2 image x is blurred by a point-spread function h and
sensed by a second 2-D kernel s, both acting by periodic (circular)
convolution, then decimated on the grid (d1 i, d2 j):

    y = P C H x,   (K x)[i, j] = sum_{a, b} k[(i - a) mod n1, (j - b) mod n2] x[a, b]

for K = C (kernel s) and K = H (kernel h).  Writing a blur as a circulant
acting on the vectorised image is how Section 7 brings deblurring into the
partial-circulant framework (there with a 1-D box blur); here the blur and
the sensing kernel are 2-D, so C H is doubly block circulant and the 2-D DFT
diagonalises it with eigenvalues g_hat = DFT2(s) * DFT2(h) (the 2-D form of
Section 4.2's diagonalisation).  Decimation folds the n1 x n2 spectrum onto
the m1 x m2 grid (m_i = n_i / d_i), so A A^T is an m1 x m2 doubly block
circulant with eigenvalues

    Lam[k1', k2'] = 1/(d1 d2) * sum_{l1 < d1, l2 < d2} |g_hat[k1' + l1 m1, k2' + l2 m2]|^2,

which is what makes ADMM's (A^T A + rho I)^{-1} (Alg. 2) exact and cheap by
the Woodbury identity, as in 1-D.

Vectors are flattened row-major (index i * n2 + j), so the generic solvers
and the objective of `fftref` (ista, admm, objective) run on `Operator2D`
unchanged.

dense_A2 is the definition written out as an explicit matrix (pin P16 checks
the FFT operator against it and Lam against the eigenvalues of A A^T).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.fft as sfft

from . import fftref

_WORKERS = -1   # scipy.fft: all cores


def conv_matrix(k):
    """Dense matrix of periodic 2-D convolution by kernel k (n1 x n2):
    K[(i, j), (a, b)] = k[(i - a) mod n1, (j - b) mod n2]."""
    k = np.asarray(k, np.float64)
    n1, n2 = k.shape
    i = np.arange(n1)
    j = np.arange(n2)
    di = (i[:, None] - i[None, :]) % n1          # (i, a)
    dj = (j[:, None] - j[None, :]) % n2          # (j, b)
    K = k[di[:, None, :, None], dj[None, :, None, :]]   # [i, j, a, b]
    return K.reshape(n1 * n2, n1 * n2)


def dec_matrix(n1, n2, d1, d2):
    """P: keeps pixel (d1 i, d2 j) as output i * (n2/d2) + j."""
    m1, m2 = n1 // d1, n2 // d2
    P = np.zeros((m1 * m2, n1 * n2))
    for i in range(m1):
        for j in range(m2):
            P[i * m2 + j, (d1 * i) * n2 + d2 * j] = 1.0
    return P


def dense_A2(s, h, d1, d2):
    """A = P C H as a dense matrix (h = None: no blur)."""
    s = np.asarray(s, np.float64)
    n1, n2 = s.shape
    A = conv_matrix(s)
    if h is not None:
        A = A @ conv_matrix(h)
    return dec_matrix(n1, n2, d1, d2) @ A


class Operator2D:
    """A = P C H through the 2-D FFT, on flattened vectors."""

    def __init__(self, s, h, d1, d2):
        s = np.asarray(s, np.float64)
        self.n1, self.n2 = s.shape
        self.d1, self.d2 = d1, d2
        self.m1, self.m2 = self.n1 // d1, self.n2 // d2
        self.n = self.n1 * self.n2
        self.m = self.m1 * self.m2
        g = sfft.fft2(s, workers=_WORKERS)
        if h is not None:
            g = g * sfft.fft2(np.asarray(h, np.float64), workers=_WORKERS)
        self.ghat = g                     # full n1 x n2 eigenvalues of C H

    def _img(self, x):
        return np.asarray(x, np.float64).reshape(self.n1, self.n2)

    def G(self, x):
        """C H x (periodic convolution by s * h)."""
        X = sfft.fft2(self._img(x), workers=_WORKERS)
        return sfft.ifft2(self.ghat * X, workers=_WORKERS).real.ravel()

    def GT(self, v):
        X = sfft.fft2(self._img(v), workers=_WORKERS)
        return sfft.ifft2(np.conj(self.ghat) * X, workers=_WORKERS).real.ravel()

    def up(self, r):
        """P^T r: r (m1 x m2) onto pixels (d1 i, d2 j), zeros elsewhere."""
        u = np.zeros((self.n1, self.n2))
        u[:: self.d1, :: self.d2] = np.asarray(r, np.float64).reshape(self.m1, self.m2)
        return u.ravel()

    def A(self, x):
        return self.G(x).reshape(self.n1, self.n2)[:: self.d1, :: self.d2].ravel()

    def AT(self, r):
        return self.GT(self.up(r))

    def Lam(self):
        """Eigenvalues of A A^T on the m1 x m2 DFT grid."""
        a = np.abs(self.ghat) ** 2
        return a.reshape(self.d1, self.m1, self.d2, self.m2).mean(axis=(0, 2))

    def max_chat_sq(self):
        """max |g_hat|^2: an upper bound on ||A||_2^2 (same role as in 1-D)."""
        return float(np.max(np.abs(self.ghat) ** 2))

    def woodbury_solve(self, rho, q):
        """(A^T A + rho I)^{-1} q = (q - A^T (rho I + A A^T)^{-1} A q) / rho."""
        aq = self.A(q).reshape(self.m1, self.m2)
        t = sfft.ifft2(sfft.fft2(aq, workers=_WORKERS) / (rho + self.Lam()), workers=_WORKERS).real
        return (q - self.AT(t.ravel())) / rho


@dataclasses.dataclass
class Problem2D:
    n1: int
    n2: int
    d1: int
    d2: int
    s: np.ndarray       # float32 (n1, n2)
    h: np.ndarray       # float32 (n1, n2) or None
    y: np.ndarray       # float32 (m1, m2)
    x_true: np.ndarray  # float32 (n1, n2)
    lam: np.float32
    tau: np.float32

    def op(self):
        return Operator2D(self.s.astype(np.float64), None if self.h is None else self.h.astype(np.float64),
                          self.d1, self.d2)


def build(scene, lam_frac):
    """Problem from a workloads.Scene2D draw: y = A x* in FP64 rounded to
    float32; lam = frac ||A^T y||_inf and tau = 1/max|g_hat|^2 in FP64 on the
    rounded data, rounded to float32 (the same rule as in 1-D)."""
    op = Operator2D(scene.s.astype(np.float64), scene.h.astype(np.float64), scene.d1, scene.d2)
    y = op.A(scene.x_true.astype(np.float64)).astype(np.float32)
    lam = np.float32(lam_frac * float(np.max(np.abs(op.AT(y.astype(np.float64))))))
    tau = np.float32(1.0 / op.max_chat_sq())
    return Problem2D(n1=scene.n1, n2=scene.n2, d1=scene.d1, d2=scene.d2, s=scene.s, h=scene.h,
                     y=y.reshape(op.m1, op.m2), x_true=scene.x_true, lam=lam, tau=tau)


# the solvers and objective of the 1-D reference are generic in the operator
ista = fftref.ista
admm = fftref.admm
objective = fftref.objective
