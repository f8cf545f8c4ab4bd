"""Pins for the unrolled-ISTA oracle and its hand adjoint."""
import numpy as np
import pytest
import torch

import workloads
from oracle import dense, fftref, problem, unrolled


def setup(n, d, B, k, seed, K):
    rng = np.random.default_rng(seed)
    m = n // d
    c = (rng.standard_normal(n) / np.sqrt(m)).astype(np.float32).astype(np.float64)
    op = fftref.Operator(c, d)
    Xs = np.zeros((B, n))
    for b in range(B):
        Xs[b, rng.choice(n, k, replace=False)] = rng.standard_normal(k)
    Y = np.stack([op.A(x) for x in Xs])
    lam0 = 0.05 * np.mean([np.max(np.abs(op.AT(y))) for y in Y])
    tau0 = 1.0 / op.max_chat_sq()
    lam = lam0 * (1 + 0.2 * rng.uniform(-1, 1, K))
    tau = tau0 * (1 + 0.2 * rng.uniform(-1, 0.5, K))
    return op, Y, Xs, lam, tau


def test_constant_parameters_reduce_to_ista():
    pr = problem.build(workloads.signal(512, 4, 6, 21))
    A = pr.A()
    y = pr.y.astype(np.float64)
    K = 40
    xi = dense.ista(A, y, float(pr.lam), float(pr.tau), K)
    XK, _ = unrolled.forward(pr.op(), y[None, :], np.full(K, float(pr.lam)), np.full(K, float(pr.tau)), K)
    assert np.max(np.abs(XK[0] - xi)) <= 1e-12 * np.max(np.abs(xi))


def torch_dense_grads(op, Y, Xs, lam, tau, K):
    """Reverse mode by torch autograd through the loop with a dense A."""
    A = torch.tensor(dense.dense_A(op.c, op.d), dtype=torch.float64)
    Yt = torch.tensor(Y, dtype=torch.float64, requires_grad=True)
    lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
    tt = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    X = torch.zeros(Y.shape[0], op.n, dtype=torch.float64)
    for t in range(K):
        G = (Yt - X @ A.T) @ A
        V = X + tt[t] * G
        th = tt[t] * lt[t]
        X = torch.sign(V) * torch.relu(V.abs() - th)
    L = ((X - torch.tensor(Xs)) ** 2).sum()
    L.backward()
    return lt.grad.numpy(), tt.grad.numpy(), Yt.grad.numpy()


def test_adjoint_matches_dense_autograd():
    K = 12
    op, Y, Xs, lam, tau = setup(64, 4, 2, 3, 5, K)
    gl, gt, gy = unrolled.backward(op, Y, lam, tau, K, Xs)
    rl, rt, ry = torch_dense_grads(op, Y, Xs, lam, tau, K)
    for a, b in ((gl, rl), (gt, rt), (gy, ry)):
        assert np.max(np.abs(a - b)) <= 1e-10 * max(np.max(np.abs(b)), 1e-30)


def test_adjoint_matches_finite_differences():
    """Central differences, relative step h = 1e-6, at n = 256, d = 4,
    k = 4, batch 2, K = 50.  The derivative is not defined at a kink, so the
    instance is the first seed whose every |v_t| lies at least 1e-6 from its
    threshold (the perturbations move v_t by well under that)."""
    K = 50
    for seed in range(11, 60):
        op, Y, Xs, lam, tau = setup(256, 4, 2, 4, seed, K)
        if unrolled.min_margin(op, Y, lam, tau, K) > 1e-6:
            break
    else:
        pytest.fail("no instance away from the kinks")
    gl, gt, gy = unrolled.backward(op, Y, lam, tau, K, Xs)
    f = lambda Y_, l_, t_: unrolled.loss(unrolled.forward(op, Y_, l_, t_, K)[0], Xs)
    h = 1e-6
    for t in (0, 7, 23, 49):
        e = np.zeros(K)
        e[t] = h * lam[t]
        fd = (f(Y, lam + e, tau) - f(Y, lam - e, tau)) / (2 * e[t])
        assert abs(fd - gl[t]) <= 1e-6 * max(abs(gl).max(), 1e-30), (t, fd, gl[t])
        e = np.zeros(K)
        e[t] = h * tau[t]
        fd = (f(Y, lam, tau + e) - f(Y, lam, tau - e)) / (2 * e[t])
        assert abs(fd - gt[t]) <= 1e-6 * max(abs(gt).max(), 1e-30), (t, fd, gt[t])
    for (b, i) in ((0, 3), (1, 40), (0, 63)):
        E = np.zeros_like(Y)
        E[b, i] = h
        fd = (f(Y + E, lam, tau) - f(Y - E, lam, tau)) / (2 * h)
        assert abs(fd - gy[b, i]) <= 1e-6 * max(np.abs(gy).max(), 1e-30), (b, i, fd, gy[b, i])


def _mut_backward_no_tau_in_ybar(op, Y, lam, tau, K, Xs):
    XK, rec = unrolled.forward(op, Y, lam, tau, K)
    xbar = 2.0 * (XK - Xs)
    g_l, g_t, g_y = np.zeros(K), np.zeros(K), np.zeros_like(Y)
    for t in range(K - 1, -1, -1):
        Xp, G, V = rec[t]
        Mk = (np.abs(V) > tau[t] * lam[t]).astype(float)
        vbar = Mk * xbar
        thbar = -float(np.sum(np.sign(V) * Mk * xbar))
        g_l[t] = tau[t] * thbar
        g_t[t] = lam[t] * thbar + float(np.sum(vbar * G))
        Av = np.stack([op.A(v) for v in vbar])
        g_y += Av                       # planted: tau_t missing
        xbar = vbar - tau[t] * np.stack([op.AT(a) for a in Av])
    return g_l, g_t, g_y


def _mut_backward_threshold_sign(op, Y, lam, tau, K, Xs):
    g_l, g_t, g_y = unrolled.backward(op, Y, lam, tau, K, Xs)
    return -g_l, g_t, g_y              # planted: sign of the threshold derivative


@pytest.mark.parametrize("mut", [_mut_backward_no_tau_in_ybar, _mut_backward_threshold_sign])
def test_planted_adjoint_mistakes_are_caught(mut):
    K = 12
    op, Y, Xs, lam, tau = setup(64, 4, 2, 3, 5, K)
    gl, gt, gy = mut(op, Y, lam, tau, K, Xs)
    rl, rt, ry = torch_dense_grads(op, Y, Xs, lam, tau, K)
    ok = all(np.max(np.abs(a - b)) <= 1e-10 * max(np.max(np.abs(b)), 1e-30)
             for a, b in ((gl, rl), (gt, rt), (gy, ry)))
    assert not ok


def test_flipping_a_decided_mask_changes_the_gradients():
    """The mask override is live: flipping an entry far from its kink changes
    the gradients, and flipping nothing changes nothing."""
    K = 12
    op, Y, Xs, lam, tau = setup(64, 4, 2, 3, 5, K)
    base = unrolled.backward(op, Y, lam, tau, K, Xs)
    same = unrolled.backward(op, Y, lam, tau, K, Xs, flip=[])
    assert all(np.array_equal(a, b) for a, b in zip(base, same))
    _, rec = unrolled.forward(op, Y, lam, tau, K)
    V = rec[K - 1][2]
    b, i = np.unravel_index(np.argmax(np.abs(V)), V.shape)
    moved = unrolled.backward(op, Y, lam, tau, K, Xs, flip=[(K - 1, int(b), int(i))])
    assert not np.allclose(moved[0], base[0])
    amb = unrolled.ambiguous(op, Y, lam, tau, K, 1e300)
    assert len(amb) == K * Y.shape[0] * op.n
