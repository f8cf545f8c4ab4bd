"""Unrolled ISTA with per-iteration parameters and its hand adjoint (FP64).

Test infrastructure only.  K iterations of Alg. 1 with a step tau_t and a
threshold lam_t per iteration, shared by a batch of signals that share one
sensing operator A = P C:

    x_0 = 0,
    g_t = A^T (y - A x_{t-1}),   v_t = x_{t-1} + tau_t g_t,
    x_t = eta_{theta_t}(v_t),    theta_t = tau_t lam_t        (Eq. 4)

With lam_t = lam and tau_t = tau for every t this is exactly ISTA (a pin).
Loss: L = sum over the batch of ||x_K - x*||^2.

Adjoint (reverse mode, derived by hand from the recursion above):
    xbar_K = 2 (x_K - x*)
    for t = K .. 1, with the mask M_t = 1[|v_t| > theta_t]:
      vbar_t     = M_t * xbar_t
      thetabar_t = -< sgn(v_t) M_t , xbar_t >
      lambar_t   = tau_t thetabar_t
      taubar_t   = lam_t thetabar_t + < vbar_t , g_t >
      ybar      += tau_t A vbar_t
      xbar_{t-1} = vbar_t - tau_t A^T A vbar_t
Sums run over the batch and all entries.  The threshold's derivative is
undefined where |v_t| = theta_t exactly; that set has measure zero for
continuous data.
"""
from __future__ import annotations

import numpy as np

from . import fftref


def _A(op, X):
    return np.stack([op.A(x) for x in X])


def _AT(op, R):
    return np.stack([op.AT(r) for r in R])


def forward(op, Y, lam, tau, K):
    """Returns x_K and the per-step records (x_{t-1}, g_t, v_t)."""
    Y = np.asarray(Y, np.float64)
    X = np.zeros((Y.shape[0], op.n))
    rec = []
    for t in range(K):
        G = _AT(op, Y - _A(op, X))
        V = X + tau[t] * G
        th = tau[t] * lam[t]
        Xn = fftref.soft(V, th)
        rec.append((X, G, V))
        X = Xn
    return X, rec


def loss(XK, Xstar):
    return float(np.sum((XK - Xstar) ** 2))


def backward(op, Y, lam, tau, K, Xstar, flip=()):
    """Gradients of L with respect to lam (K), tau (K) and Y (B x m).

    `flip` names entries (t, b, i) whose mask M_t is inverted.  At an entry
    with |v_t| within rounding of theta_t the threshold decision of a lower
    precision implementation may go either way; both choices give a valid
    (one-sided) derivative, and a comparison accepts any of them."""
    XK, rec = forward(op, Y, lam, tau, K)
    xbar = 2.0 * (XK - np.asarray(Xstar, np.float64))
    g_lam = np.zeros(K)
    g_tau = np.zeros(K)
    g_Y = np.zeros_like(np.asarray(Y, np.float64))
    for t in range(K - 1, -1, -1):
        Xp, G, V = rec[t]
        th = tau[t] * lam[t]
        Mk = (np.abs(V) > th).astype(np.float64)
        for (tf, b, i) in flip:
            if tf == t:
                Mk[b, i] = 1.0 - Mk[b, i]
        vbar = Mk * xbar
        thbar = -float(np.sum(np.sign(V) * Mk * xbar))
        g_lam[t] = tau[t] * thbar
        g_tau[t] = lam[t] * thbar + float(np.sum(vbar * G))
        Av = _A(op, vbar)
        g_Y += tau[t] * Av
        xbar = vbar - tau[t] * _AT(op, Av)
    return g_lam, g_tau, g_Y


def min_margin(op, Y, lam, tau, K):
    """Smallest | |v_t| - theta_t | over all steps (distance to a kink)."""
    _, rec = forward(op, Y, lam, tau, K)
    return min(float(np.min(np.abs(np.abs(V) - tau[t] * lam[t]))) for t, (_, _, V) in enumerate(rec))


def ambiguous(op, Y, lam, tau, K, delta):
    """Entries (t, b, i) with | |v_t| - theta_t | < delta."""
    _, rec = forward(op, Y, lam, tau, K)
    out = []
    for t, (_, _, V) in enumerate(rec):
        bb, ii = np.nonzero(np.abs(np.abs(V) - tau[t] * lam[t]) < delta)
        out += [(t, int(b), int(i)) for b, i in zip(bb, ii)]
    return out
