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
    cs.load().cs_ista_solve_batched(0, None, None, None, None, None, None, None, None, 5, None, None)


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


# ----------------------------------------------------------------------------
# per-signal decimation, batched ADMM, the schedule report
# ----------------------------------------------------------------------------
def mixed_d(specs, seed):
    """specs: list of (n, d); one draw per signal."""
    rng = np.random.default_rng(seed)
    sigs = [workloads.signal(int(n), int(d), max(2, int(n) // 256), int(rng.integers(1 << 30))) for n, d in specs]
    return batched.build_batch(sigs)


def split(xs, ns):
    off_n, _ = cs.batch_offsets(ns, 4)
    return [xs[o:o + n] for o, n in zip(off_n, ns)]


SPECS = [(1 << 12, 2), (1 << 15, 8), (1 << 10, 4), (1 << 17, 4), (1 << 13, 8), (1 << 16, 2), (1 << 11, 2),
         (1 << 18, 8), (1 << 14, 4), (1 << 12, 8)]


def test_batched_per_signal_decimation_vs_oracle():
    """Signals with different decimations in one call, each against its own
    oracle solve."""
    probs = mixed_d(SPECS, 91)
    ns, c, y, lam, tau = batched.concat(probs)
    ds = np.array([p.d for p in probs], np.int32)
    T = 40
    xs = h(cs.ista_solve_batched(ns, ds, g(c), g(y), g(lam), g(tau), T))
    ref = batched.ista_batched(probs, T)
    worst = 0.0
    for i, (a, b) in enumerate(zip(split(xs, ns), ref)):
        e = rel(a, b)
        worst = max(worst, e)
        assert e <= IT_TOL, (i, SPECS[i], e)
    print("per-signal d batch: worst rel err at t=%d: %.3e" % (T, worst))


def admm_batch(probs, rhos, T, warm_from=None):
    ns, c, y, lam, _ = batched.concat(probs)
    ds = np.array([p.d for p in probs], np.int32)
    kw = {}
    if warm_from is not None:
        kw = dict(z_cat=g(warm_from[0]), u_cat=g(warm_from[1]), warm=True)
    x, z, u = cs.admm_solve_batched(ns, ds, g(c), g(y), g(lam), g(np.asarray(rhos, np.float32)), T, **kw)
    return ns, h(x), h(z), h(u)


def test_batched_admm_vs_oracle():
    """Batched ADMM with per-signal rho and d: x, z, u of every signal
    against the oracle's ADMM (Alg. 2) at t = 60."""
    probs = mixed_d(SPECS, 92)
    rhos = [1.0, 0.5, 2.0, 1.0, 1.0, 0.25, 1.0, 1.0, 4.0, 1.0]
    T = 60
    ns, x, z, u = admm_batch(probs, rhos, T)
    ref = batched.admm_batched(probs, rhos, T)
    worst = 0.0
    for i, (a, b, cc, r) in enumerate(zip(split(x, ns), split(z, ns), split(u, ns), ref)):
        ex, ez = rel(a, r[0]), rel(b, r[1])
        eu = rel(cc, r[2]) if np.linalg.norm(r[2]) > 0 else float(np.abs(cc).max())
        worst = max(worst, ex, ez, eu)
        assert ex <= IT_TOL and ez <= IT_TOL and eu <= IT_TOL, (i, SPECS[i], ex, ez, eu)
    print("batched ADMM: worst x/z/u rel err at t=%d: %.3e" % (T, worst))


def test_batched_admm_warm_start_continues():
    """T1 cold iterations, then T2 warm iterations from the returned (z, u),
    equal T1 + T2 cold iterations."""
    probs = mixed_d(SPECS[:6], 93)
    rhos = [1.0] * 6
    ns, x1, z1, u1 = admm_batch(probs, rhos, 15)
    _, x2, z2, u2 = admm_batch(probs, rhos, 10, warm_from=(z1, u1))
    _, x3, z3, u3 = admm_batch(probs, rhos, 25)
    for a, b in ((x2, x3), (z2, z3), (u2, u3)):
        assert rel(a, b) <= 1e-6


def test_batched_admm_zero_iterations():
    probs = mixed_d(SPECS[:3], 94)
    ns, x, z, u = admm_batch(probs, [1.0] * 3, 0)
    assert not x.any() and not z.any() and not u.any()
    zw = np.full(len(x), 0.5)
    uw = np.full(len(x), -0.25)
    _, x, z, u = admm_batch(probs, [1.0] * 3, 0, warm_from=(zw, uw))
    assert np.all(z == 0.5) and np.all(u == -0.25)


def test_batched_schedule_report():
    """After a batched call the library reports its schedule: one grid that
    fits on the device, the tuner's trials, and whether a graph replay ran."""
    probs = mixed_d(SPECS, 95)
    ns, c, y, lam, tau = batched.concat(probs)
    ds = np.array([p.d for p in probs], np.int32)
    cs.ista_solve_batched(ns, ds, g(c), g(y), g(lam), g(tau), 5)
    torch.cuda.synchronize()
    info = cs.batched_schedule()
    print("batched schedule:", info)
    assert info["grid"] >= 1 and info["wg_per_cu"] >= 1
    assert isinstance(info["trials"], list) and len(info["trials"]) >= 1
    assert isinstance(info["graph"], bool)


def test_batched_admm_full_workload_sampled():
    """The 512-signal uneven batch through batched ADMM (rho = 1, 100
    iterations): the first signal of each length and the last signal against
    the oracle's ADMM."""
    sigs = workloads.uneven_batch()
    probs = batched.build_batch(sigs, workloads.UNEVEN_PARAMS["lam_frac"])
    T = 100
    rhos = [1.0] * len(probs)
    ns, x, z, u = admm_batch(probs, rhos, T)
    xs, zs = split(x, ns), split(z, ns)
    nl = [p.n for p in probs]
    pick = sorted({nl.index(n) for n in set(nl)} | {len(nl) - 1})
    worst = 0.0
    for i in pick:
        r = batched.admm_one(probs[i], 1.0, T)
        ex, ez = rel(xs[i], r[0]), rel(zs[i], r[1])
        worst = max(worst, ex, ez)
        assert ex <= IT_TOL and ez <= IT_TOL, (i, nl[i], ex, ez)
    print("full uneven batch ADMM, %d sampled signals, worst rel err at t=%d: %.3e" % (len(pick), T, worst))
