"""Problem instances: from a seeded draw to the float32 data both sides solve.

Test infrastructure only.  Rounding rule: c and x* arrive as float32 draws;
y = A x* is evaluated in FP64 (dense A for n <= DENSE_MAX, else the FFT
reference) and rounded to float32; the step size tau = 1 / max_k |c_hat_k|^2
and lam = frac * ||A^T y||_inf are evaluated in FP64 on the rounded data and
rounded to float32.  The oracle then consumes float64(float32(.)) of every
value, so both sides solve the identical problem and a parity gap measures
only the GPU's arithmetic.

Step size: Alg. 1 asks for tau in (0, ||A||_2^-2).  max_k |c_hat_k|^2 bounds
||A||_2^2 from above (A A^T's eigenvalues are averages of |c_hat|^2 over alias
classes), so tau = 1/max|c_hat|^2 is admissible.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import dense, fftref

DENSE_MAX = 8192


@dataclasses.dataclass
class Problem:
    n: int
    d: int
    c: np.ndarray       # float32
    y: np.ndarray       # float32, length m
    x_true: np.ndarray  # float32
    lam: np.float32
    tau: np.float32

    @property
    def m(self):
        return self.n // self.d

    def op(self):
        return fftref.Operator(self.c.astype(np.float64), self.d)

    def A(self):
        return dense.dense_A(self.c.astype(np.float64), self.d)


def measure(c32, d, x32):
    """y = A x* in FP64, rounded to float32."""
    n = c32.shape[0]
    if n <= DENSE_MAX:
        y = dense.dense_A(c32.astype(np.float64), d) @ x32.astype(np.float64)
    else:
        y = fftref.Operator(c32.astype(np.float64), d).A(x32.astype(np.float64))
    return y.astype(np.float32)


def step_size(c32):
    """tau = 1 / max_k |c_hat_k|^2 (FP64), rounded to float32."""
    op = fftref.Operator(c32.astype(np.float64), 1)
    return np.float32(1.0 / op.max_chat_sq())


def lam_max(c32, d, y32):
    """||A^T y||_inf in FP64: the smallest lam for which x = 0 solves the LASSO."""
    n = c32.shape[0]
    if n <= DENSE_MAX:
        g = dense.dense_A(c32.astype(np.float64), d).T @ y32.astype(np.float64)
    else:
        g = fftref.Operator(c32.astype(np.float64), d).AT(y32.astype(np.float64))
    return float(np.max(np.abs(g)))


def build(sig, lam_frac=0.01):
    """Problem instance from a workloads.Signal1D draw."""
    y = measure(sig.c, sig.d, sig.x_true)
    tau = step_size(sig.c)
    lam = np.float32(lam_frac * lam_max(sig.c, sig.d, y))
    return Problem(n=sig.n, d=sig.d, c=sig.c, y=y, x_true=sig.x_true,
                   lam=lam, tau=tau)
