"""GPU parity of the differentiable unrolled ISTA against the FP64 oracle
(forward iterate and the hand adjoint's gradients)."""
import numpy as np
import pytest

import workloads
from oracle import fftref, unrolled

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# |v_t| closer than this to its threshold counts as undecided in FP32: the
# observed FP32 error of v_t on these sizes is below 3e-7 (|v| <= 2)
KINK = 1e-6
MAX_AMBIG = 6


def instance(n, d, B, k, K, seed):
    """float32 problem (shared c, B truths, per-step lam / tau) with at most
    MAX_AMBIG entries of any v_t within KINK of its threshold."""
    for s in range(seed, seed + 100):
        rng = np.random.default_rng(s)
        m = n // d
        c = (rng.standard_normal(n) / np.sqrt(m)).astype(np.float32)
        op = fftref.Operator(c.astype(np.float64), d)
        Xs = np.zeros((B, n))
        for b in range(B):
            Xs[b, rng.choice(n, k, replace=False)] = rng.standard_normal(k)
        Y = np.stack([op.A(x) for x in Xs]).astype(np.float32)
        lam0 = 0.05 * np.mean([np.max(np.abs(op.AT(y))) for y in Y.astype(np.float64)])
        tau0 = 1.0 / op.max_chat_sq()
        lam = (lam0 * (1 + 0.2 * rng.uniform(-1, 1, K))).astype(np.float32)
        tau = (tau0 * (1 + 0.2 * rng.uniform(-1, 0.5, K))).astype(np.float32)
        amb = unrolled.ambiguous(op, Y.astype(np.float64), lam.astype(np.float64), tau.astype(np.float64), K, KINK)
        if len(amb) <= MAX_AMBIG:
            return c, op, Y, Xs.astype(np.float32), lam, tau, amb
    pytest.fail("no instance with few undecided threshold entries")


def check_grads(got, op, Y, lam, tau, K, Xs, amb, tol):
    """The GPU gradients match the oracle's for some choice of the undecided
    threshold decisions (every subset of `amb` flipped)."""
    args = (op, Y.astype(np.float64), lam.astype(np.float64), tau.astype(np.float64), K, Xs)
    got = [h(v) for v in got]
    best = None
    for mask in range(1 << len(amb)):
        flip = [amb[j] for j in range(len(amb)) if mask >> j & 1]
        ref = unrolled.backward(*args, flip=flip)
        errs = [rel(a, b) for a, b in zip(got, ref)]
        if best is None or max(errs) < max(best):
            best = errs
        if max(errs) <= tol:
            break
    print("unrolled grads rel err lam %.2e tau %.2e y %.2e (%d undecided entries)" % (*best, len(amb)))
    assert max(best) <= tol


def test_constant_parameters_equal_plain_ista():
    pr_sig = workloads.signal(4096, 4, 20, 31)
    from oracle import problem
    pr = problem.build(pr_sig)
    K = 30
    y = g(pr.y[None, :])
    xK, _ = cs.unrolled_ista_fwd(g(pr.c), 4, y, g(np.full(K, pr.lam)), g(np.full(K, pr.tau)), K, 10)
    cs.set_solver_path(cs.PATH_TWO_PASS)
    x = cs.ista_solve(g(pr.c), 4, g(pr.y), pr.lam, pr.tau, K)
    cs.set_solver_path(cs.PATH_AUTO)
    assert rel(h(xK)[0], h(x)) <= 1e-6


@pytest.mark.parametrize("n,d,B,K,every", [(1024, 4, 3, 20, 6), (4096, 2, 2, 15, 15), (2048, 8, 2, 12, 5)])
def test_forward_and_gradients_vs_oracle(n, d, B, K, every):
    c, op, Y, Xs, lam, tau, amb = instance(n, d, B, max(2, n // 256), K, 100 + n)
    xK, ckpt = cs.unrolled_ista_fwd(g(c), d, g(Y), g(lam), g(tau), K, every)
    XK, _ = unrolled.forward(op, Y.astype(np.float64), lam.astype(np.float64), tau.astype(np.float64), K)
    assert rel(h(xK), XK) <= 1e-4
    # the loss gradient at x_K is the oracle's (2 (x_K - x*)), not the GPU's
    got = cs.unrolled_ista_bwd(g(c), d, g(Y), g(lam), g(tau), K, every, ckpt, g(2.0 * (XK - Xs)))
    check_grads(got, op, Y, lam, tau, K, Xs, amb, 1e-4)


def test_checkpointing_does_not_change_gradients():
    """every = 5 (recompute from checkpoints) and every = K (recompute from
    x_0) give identical gradients."""
    n, d, B, K = 2048, 4, 2, 20
    c, op, Y, Xs, lam, tau, _ = instance(n, d, B, 8, K, 7)
    out = []
    for every in (5, K):
        xK, ckpt = cs.unrolled_ista_fwd(g(c), d, g(Y), g(lam), g(tau), K, every)
        gx = g(2.0 * (h(xK) - Xs))
        out.append([h(v) for v in cs.unrolled_ista_bwd(g(c), d, g(Y), g(lam), g(tau), K, every, ckpt, gx)])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_autograd_function():
    n, d, B, K = 1024, 4, 2, 10
    c, op, Y, Xs, lam, tau, amb = instance(n, d, B, 4, K, 3)
    yt = g(Y).requires_grad_(True)
    lt = g(lam).requires_grad_(True)
    tt = g(tau).requires_grad_(True)
    xK = cs.UnrolledISTA.apply(yt, lt, tt, g(c), d, K, 4)
    loss = ((xK - g(Xs)) ** 2).sum()
    loss.backward()
    check_grads((lt.grad, tt.grad, yt.grad), op, Y, lam, tau, K, Xs, amb, 1e-4)


def test_shared_c_batch_shape_forward_and_aggregate_gradients():
    """The differentiable workload's shape (n = 2^16, d = 4, k = 256, K = 50,
    checkpoints every 10) on 4 signals: the forward iterate per signal, and
    the lam / tau gradients, which aggregate over the batch."""
    d, K, every = 4, 50, 10
    c, Xs = workloads.shared_c_batch(batch=4)
    assert c.shape[0] == 1 << 16
    op = fftref.Operator(c.astype(np.float64), d)
    Y = np.stack([op.A(x.astype(np.float64)) for x in Xs]).astype(np.float32)
    lam = np.full(K, unrolled_lam0(op, Y, 0.01), np.float32)
    tau = np.full(K, 1.0 / op.max_chat_sq(), np.float32)
    xK, ckpt = cs.unrolled_ista_fwd(g(c), d, g(Y), g(lam), g(tau), K, every)
    XK, _ = unrolled.forward(op, Y.astype(np.float64), lam.astype(np.float64), tau.astype(np.float64), K)
    assert rel(h(xK), XK) <= 1e-4
    # about one FP32-undecided threshold entry is expected at this size; its
    # effect on the gradients is of order 1e-6 (relative), far below the bar
    gl, gt, gy = cs.unrolled_ista_bwd(g(c), d, g(Y), g(lam), g(tau), K, every, ckpt, g(2.0 * (XK - Xs)))
    rl, rt, ry = unrolled.backward(op, Y.astype(np.float64), lam.astype(np.float64), tau.astype(np.float64), K, Xs)
    print("shared_c_batch-shaped: rel err lam %.2e tau %.2e y %.2e" % (rel(h(gl), rl), rel(h(gt), rt), rel(h(gy), ry)))
    assert rel(h(gl), rl) <= 1e-4 and rel(h(gt), rt) <= 1e-4 and rel(h(gy), ry) <= 1e-4


def test_unrolled_bad_arguments():
    c = g(np.ones(1024))
    y = g(np.ones((2, 256)))
    lam = g(np.ones(5))
    with pytest.raises(cs.CsError):
        cs.unrolled_ista_fwd(c, 4, y, lam, lam, 5, 0)
    with pytest.raises(cs.CsError):
        cs.unrolled_ista_fwd(c, 3, g(np.ones((2, 1024 // 3))), lam, lam, 5, 2)
    with pytest.raises(cs.CsError):
        cs.unrolled_ista_fwd(c, 4, y, g(np.zeros(0)), g(np.zeros(0)), 0, 2)


def unrolled_lam0(op, Y, frac):
    """lam_t initial value: frac * mean over the batch of ||A^T y_b||_inf."""
    return frac * float(np.mean([np.max(np.abs(op.AT(y.astype(np.float64)))) for y in Y]))


@pytest.mark.timeout(900)
def test_shared_c_batch_full_size():
    """The timed configuration itself: all 64 signals (n = 2^16, d = 4,
    K = 50, checkpoints every 10) in one forward and one backward call,
    every signal against the FP64 oracle: x_K and dL/dy per signal, and the
    batch's lam / tau gradients, at 1e-4.  Extra: the lam / tau gradients
    equal the sums over the two halves of the batch."""
    prm = workloads.SHARED_C_PARAMS
    K, every, d = prm["K"], prm["every"], 4
    c, Xs = workloads.shared_c_batch()
    B = Xs.shape[0]
    op = fftref.Operator(c.astype(np.float64), d)
    Y = np.stack([op.A(x.astype(np.float64)) for x in Xs]).astype(np.float32)
    lam = np.full(K, unrolled_lam0(op, Y, prm["lam_frac"]), np.float32)
    tau = np.full(K, 1.0 / op.max_chat_sq(), np.float32)
    xK, ckpt = cs.unrolled_ista_fwd(g(c), d, g(Y), g(lam), g(tau), K, every)
    xK = h(xK)
    args = (op, Y.astype(np.float64), lam.astype(np.float64), tau.astype(np.float64), K)
    XK, _ = unrolled.forward(*args)
    ex = max(rel(xK[b], XK[b]) for b in range(B))
    assert ex <= 1e-4, ex
    # the loss gradient at x_K is the oracle's, so the backward passes differ
    # only by their own arithmetic
    gx = 2.0 * (XK - Xs)
    gl, gt, gy = (h(v) for v in cs.unrolled_ista_bwd(g(c), d, g(Y), g(lam), g(tau), K, every, ckpt, g(gx)))
    rl, rt, ry = unrolled.backward(*args, Xs)
    el, et = rel(gl, rl), rel(gt, rt)
    ey = max(rel(gy[b], ry[b]) for b in range(B))
    print("64 x 2^16 unrolled: worst x_K rel err %.2e; gradients rel err lam %.2e tau %.2e, worst dL/dy row %.2e"
          % (ex, el, et, ey))
    assert el <= 1e-4 and et <= 1e-4 and ey <= 1e-4
    halves = []
    for sl in (slice(0, B // 2), slice(B // 2, B)):
        xh, ch = cs.unrolled_ista_fwd(g(c), d, g(Y[sl]), g(lam), g(tau), K, every)
        assert np.array_equal(h(xh), xK[sl])
        halves.append([h(v) for v in cs.unrolled_ista_bwd(g(c), d, g(Y[sl]), g(lam), g(tau), K, every, ch, g(gx[sl]))])
    assert rel(halves[0][0] + halves[1][0], gl) <= 1e-5
    assert rel(halves[0][1] + halves[1][1], gt) <= 1e-5
    assert np.array_equal(np.concatenate([halves[0][2], halves[1][2]]), gy)
