"""GPU parity of the batched ISTA entry point against the FP64 oracle (each
signal solved on its own) and against the plain single-signal solver."""
import numpy as np
import pytest

import workloads
from oracle import batched, problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")
IT_TOL = 1e-4


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_batch(probs, d, iters):
    ns, c, y, lam, tau = batched.concat(probs)
    x = cs.ista_solve_batched(ns, d, g(c), g(y), g(lam), g(tau), iters)
    xs = h(x)
    off_n, _ = cs.batch_offsets(ns, d)
    return [xs[o:o + n] for o, n in zip(off_n, ns)]


def mixed(d, sizes, seed):
    rng = np.random.default_rng(seed)
    sigs = [workloads.signal(int(n), d, max(2, int(n) // 256), int(rng.integers(1 << 30))) for n in sizes]
    return batched.build_batch(sigs)


@pytest.mark.parametrize("d", [2, 4, 8])
def test_batched_mixed_sizes_vs_oracle(d):
    sizes = [1 << 12, 1 << 10, 1 << 14, 1 << 11, 1 << 13, 1 << 10, 1 << 16, 1 << 12]
    probs = mixed(d, sizes, 40 + d)
    T = 30
    got = run_batch(probs, d, T)
    ref = batched.ista_batched(probs, T)
    for i, (a, b) in enumerate(zip(got, ref)):
        assert rel(a, b) <= IT_TOL, (i, sizes[i], rel(a, b))


def test_batched_equals_plain_solver():
    """Each signal of a batch is solved with the same arithmetic as a plain
    solve of that signal alone."""
    d = 4
    sizes = [1 << 13, 1 << 10, 1 << 15, 1 << 18]
    probs = mixed(d, sizes, 7)
    T = 25
    got = run_batch(probs, d, T)
    for a, pr in zip(got, probs):
        x = h(cs.ista_solve(g(pr.c), d, g(pr.y), pr.lam, pr.tau, T))
        assert rel(a, x) <= 1e-6


def test_batched_uneven_batch_shape():
    """Sizes drawn like the batched workload (n = 2^12 .. 2^18, k = n/256),
    a smaller count; every signal checked at t = 100."""
    sigs = workloads.uneven_batch(count=16)
    probs = batched.build_batch(sigs)
    T = 100
    got = run_batch(probs, 4, T)
    ref = batched.ista_batched(probs, T)
    worst = max(rel(a, b) for a, b in zip(got, ref))
    print("uneven_batch-shaped batch worst rel err at t=100: %.3e" % worst)
    assert worst <= IT_TOL


def test_batched_zero_iterations_and_empty():
    probs = mixed(4, [1 << 10, 1 << 12], 3)
    got = run_batch(probs, 4, 0)
    assert all(np.all(a == 0.0) for a in got)
    # count = 0 with null pointers is a no-op
    cs.load().cs_ista_solve_batched(0, None, 4, None, None, None, None, None, None, 5, None, None)


def test_batched_repeat_and_change():
    """Same batch twice (cached descriptors) gives identical results; a
    different batch afterwards is solved correctly."""
    probs = mixed(4, [1 << 11, 1 << 13, 1 << 10], 9)
    a = run_batch(probs, 4, 20)
    b = run_batch(probs, 4, 20)
    assert all(np.array_equal(p, q) for p, q in zip(a, b))
    probs2 = mixed(4, [1 << 12, 1 << 14], 10)
    got = run_batch(probs2, 4, 20)
    ref = batched.ista_batched(probs2, 20)
    assert all(rel(p, q) <= IT_TOL for p, q in zip(got, ref))


def test_batched_rejects_bad_sizes():
    probs = mixed(4, [1 << 10], 1)
    ns, c, y, lam, tau = batched.concat(probs)
    with pytest.raises(cs.CsError):
        cs.ista_solve_batched(np.array([1 << 9]), 4, g(np.ones(1 << 9)), g(np.ones(1 << 7)), g(lam), g(tau), 3)
    with pytest.raises(cs.CsError):
        cs.ista_solve_batched(ns, 16, g(c), g(np.ones(len(c) // 16)), g(lam), g(tau), 3)


@pytest.mark.parametrize("d", [2, 8])
def test_batched_length_groups_vs_oracle(d):
    """Several signals of one long length (solved together as a group) mixed
    with short ones, in interleaved order."""
    sizes = [1 << 15, 1 << 11, 1 << 16, 1 << 15, 1 << 13, 1 << 16, 1 << 15, 1 << 10]
    probs = mixed(d, sizes, 60 + d)
    T = 20
    got = run_batch(probs, d, T)
    ref = batched.ista_batched(probs, T)
    for i, (a, b) in enumerate(zip(got, ref)):
        assert rel(a, b) <= IT_TOL, (i, sizes[i], rel(a, b))


def test_batched_groups_repeat_and_reorder():
    """A grouped batch twice gives identical results; the same signals in
    another order (other group descriptors) give the same per-signal x."""
    d = 4
    sizes = [1 << 15, 1 << 12, 1 << 15, 1 << 17]
    probs = mixed(d, sizes, 21)
    a = run_batch(probs, d, 15)
    b = run_batch(probs, d, 15)
    assert all(np.array_equal(p, q) for p, q in zip(a, b))
    perm = [3, 2, 1, 0]
    c = run_batch([probs[i] for i in perm], d, 15)
    for k, i in enumerate(perm):
        assert np.array_equal(c[k], a[i])


def test_batched_full_workload_sampled():
    """The timed configuration itself: all 512 signals of the uneven batch
    (n_i = 2^12 .. 2^18, d = 4) in one call, 200 iterations, so the work
    queue and every length group run as in the benchmark; the first signal
    of each length and the last signal of the batch against the oracle."""
    sigs = workloads.uneven_batch()
    probs = batched.build_batch(sigs, workloads.UNEVEN_PARAMS["lam_frac"])
    T = workloads.UNEVEN_PARAMS["ista_iters"]
    got = run_batch(probs, 4, T)
    ns = [p.n for p in probs]
    pick = sorted({ns.index(n) for n in set(ns)} | {len(ns) - 1})
    assert len(set(ns[i] for i in pick)) == 7
    worst = 0.0
    for i in pick:
        e = rel(got[i], batched.ista_one(probs[i], T))
        worst = max(worst, e)
        assert e <= IT_TOL, (i, ns[i], e)
    print("full uneven batch, %d sampled signals, worst rel err at t=%d: %.3e" % (len(pick), T, worst))
