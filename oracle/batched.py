"""Batched ISTA and ADMM in the FP64 oracle (test infrastructure).

Batching changes nothing about each signal's problem: the batched solve is
the plain ISTA of Alg. 1 (or ADMM of Alg. 2 with its own rho) run
independently on every signal (dense A for n <= 8192, the FFT reference
above that), which the single-signal pins already fix.
"""
from __future__ import annotations

import numpy as np

from . import dense, fftref, problem


def build_batch(signals, lam_frac=0.01):
    """Problem instances (float32 data, per-signal lam and tau) for a list of
    workloads.Signal1D draws."""
    return [problem.build(s, lam_frac) for s in signals]


def ista_one(pr, iters):
    y = pr.y.astype(np.float64)
    if pr.n <= problem.DENSE_MAX:
        return dense.ista(pr.A(), y, float(pr.lam), float(pr.tau), iters)
    return fftref.ista(pr.op(), y, float(pr.lam), float(pr.tau), iters)


def ista_batched(problems, iters):
    """x(iters) of every signal, in order."""
    return [ista_one(pr, iters) for pr in problems]


def admm_one(pr, rho, iters):
    """(x, z, u) after `iters` ADMM steps from zero."""
    y = pr.y.astype(np.float64)
    if pr.n <= problem.DENSE_MAX:
        return dense.admm(pr.A(), y, float(pr.lam), float(rho), iters)
    return fftref.admm(pr.op(), y, float(pr.lam), float(rho), iters)


def admm_batched(problems, rhos, iters):
    """(x, z, u) of every signal, in order; rhos[i] is signal i's rho."""
    return [admm_one(pr, r, iters) for pr, r in zip(problems, rhos)]


def concat(problems):
    """Concatenated float32 inputs in list order: c, y, lam, tau and sizes."""
    ns = np.array([p.n for p in problems], dtype=np.int64)
    c = np.concatenate([p.c for p in problems]).astype(np.float32)
    y = np.concatenate([p.y for p in problems]).astype(np.float32)
    lam = np.array([p.lam for p in problems], dtype=np.float32)
    tau = np.array([p.tau for p in problems], dtype=np.float32)
    return ns, c, y, lam, tau
