"""Parity at the configurations the benchmark times, in the launch the
benchmark times, against the FP64 oracle.

  * large single signal (n = 2^22, m = 2^20, d = 4): ISTA per iterate at
    t = 1..12, 25, 50, 75, 100 and the final objective at T = 300; ADMM (rho = 1)
    x and z per iterate at the same t and the final objective on z(100);
  * 4096 x 4096 deblurring scene: x and z at t = 100 and F(z(200));
  * deblurring shape (n = 2^20, d = 2, order-5 box blur): F(z(300)).

Gates: relative l2 error <= 1e-4 for every compared iterate; relative
difference <= 1e-5 of the final objective, both objectives evaluated by the
oracle in FP64 (1/2 ||y - A x||^2 + lam ||x||_1).  Each test prints its worst
error.  The oracle runs once per workload (module fixtures, about 1-2
minutes each on one host core for the FFT references).
"""
import sys
import time

import numpy as np
import pytest

import workloads
from oracle import deblur, fftref, problem, twod

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")
IT_TOL = 1e-4
OBJ_TOL = 1e-5
T_CHECK = list(range(1, 13)) + [25, 50, 75, 100]


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def progress(tag, every=25):
    """Callback for the oracle loops: one line on stderr every `every`
    iterations, so a long FP64 reference shows that it is moving."""
    t0 = time.perf_counter()

    def cb(t, *_):
        if t % every == 0:
            print("[oracle %s] t=%d (%.0fs)" % (tag, t, time.perf_counter() - t0), file=sys.stderr, flush=True)
    return cb


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ----------------------------------------------------------------------------
# large single signal, n = 2^22
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def large():
    pr = problem.build(workloads.large_signal())
    return pr, pr.op()


@pytest.fixture(scope="module")
def large_ista_oracle(large):
    pr, op = large
    T = workloads.LARGE_PARAMS["ista_iters"]
    keep = set(T_CHECK) | {T}
    hist = {}
    tick = progress("n=2^22 ISTA")

    def cb(t, x):
        tick(t)
        if t in keep:
            hist[t] = x.copy()
    fftref.ista(op, pr.y.astype(np.float64), float(pr.lam), float(pr.tau), T, callback=cb)
    return hist


@pytest.fixture(scope="module")
def large_admm_oracle(large):
    pr, op = large
    T = workloads.LARGE_PARAMS["admm_iters"]
    keep = set(T_CHECK) | {T}
    hist = {}
    tick = progress("n=2^22 ADMM")

    def cb(t, x, z, u):
        tick(t)
        if t in keep:
            hist[t] = (x.copy(), z.copy())
    fftref.admm(op, pr.y.astype(np.float64), float(pr.lam), workloads.LARGE_PARAMS["rho"], T, callback=cb)
    return hist


@pytest.mark.timeout(900)
def test_large_ista_iterates_and_final_objective(large, large_ista_oracle):
    pr, op = large
    cs.set_solver_path(cs.PATH_AUTO)
    c, yg = g(pr.c), g(pr.y)
    worst = 0.0
    for t in T_CHECK:
        e = rel(h(cs.ista_solve(c, pr.d, yg, pr.lam, pr.tau, t)), large_ista_oracle[t])
        worst = max(worst, e)
        assert e <= IT_TOL, (t, e)
    T = workloads.LARGE_PARAMS["ista_iters"]
    xT = h(cs.ista_solve(c, pr.d, yg, pr.lam, pr.tau, T))
    cs.check_device()
    y, lam = pr.y.astype(np.float64), float(pr.lam)
    fg = fftref.objective(op, y, lam, xT)
    fo = fftref.objective(op, y, lam, large_ista_oracle[T])
    ef = abs(fg - fo) / fo
    print("n=2^22 ISTA: worst iterate rel err %.2e (t <= 100), final objective rel err %.2e at T=%d "
          "(x(T) rel err %.2e)" % (worst, ef, T, rel(xT, large_ista_oracle[T])))
    assert ef <= OBJ_TOL


@pytest.mark.timeout(900)
def test_large_admm_iterates_and_final_objective(large, large_admm_oracle):
    pr, op = large
    rho = workloads.LARGE_PARAMS["rho"]
    cs.set_solver_path(cs.PATH_AUTO)
    c, yg = g(pr.c), g(pr.y)
    worst = 0.0
    T = workloads.LARGE_PARAMS["admm_iters"]
    for t in T_CHECK:
        x, z, u = (h(v) for v in cs.admm_solve(c, pr.d, yg, pr.lam, rho, t))
        xo, zo = large_admm_oracle[t]
        ex, ez = rel(x, xo), rel(z, zo)
        worst = max(worst, ex, ez)
        assert ex <= IT_TOL and ez <= IT_TOL, (t, ex, ez)
    cs.check_device()
    y, lam = pr.y.astype(np.float64), float(pr.lam)
    fg = fftref.objective(op, y, lam, z)          # z(T): t = T is among T_CHECK
    fo = fftref.objective(op, y, lam, large_admm_oracle[T][1])
    ef = abs(fg - fo) / fo
    print("n=2^22 ADMM: worst x/z iterate rel err %.2e (t <= 100), final objective on z rel err %.2e at T=%d"
          % (worst, ef, T))
    assert ef <= OBJ_TOL


# ----------------------------------------------------------------------------
# 4096 x 4096 deblurring scene
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def scene():
    pr = twod.build(workloads.scene_2d(), workloads.SCENE2D_PARAMS["lam_frac"])
    op = pr.op()
    T = workloads.SCENE2D_PARAMS["admm_iters"]
    _, hist = twod.admm(op, pr.y.astype(np.float64).ravel(), float(pr.lam), workloads.SCENE2D_PARAMS["rho"], T,
                        record=True, record_every=100, callback=progress("4096^2 ADMM"))
    return pr, op, {t: (x, z) for (t, x, z, u) in hist}


@pytest.mark.timeout(900)
def test_scene_2d_iterate_100_and_final_objective(scene):
    pr, op, ref = scene
    rho, T = workloads.SCENE2D_PARAMS["rho"], workloads.SCENE2D_PARAMS["admm_iters"]
    sg, hg, yg = g(pr.s), g(pr.h), g(pr.y)
    x, z, u = (h(v).ravel() for v in cs.admm_solve2(sg, hg, yg, pr.lam, rho, 100))
    ex, ez = rel(x, ref[100][0]), rel(z, ref[100][1])
    assert ex <= IT_TOL and ez <= IT_TOL, (ex, ez)
    x, z, u = (h(v).ravel() for v in cs.admm_solve2(sg, hg, yg, pr.lam, rho, T))
    y, lam = pr.y.astype(np.float64).ravel(), float(pr.lam)
    fg = twod.objective(op, y, lam, z)
    fo = twod.objective(op, y, lam, ref[T][1])
    ef = abs(fg - fo) / fo
    print("4096^2 ADMM: x(100) rel err %.2e, z(100) rel err %.2e, F(z(%d)) rel err %.2e (z(T) rel err %.2e)"
          % (ex, ez, T, ef, rel(z, ref[T][1])))
    assert ef <= OBJ_TOL


# ----------------------------------------------------------------------------
# deblurring shape of Section 7 (n = 2^20, d = 2, order-5 box blur)
# ----------------------------------------------------------------------------
@pytest.mark.timeout(900)
def test_deblur_1d_final_objective():
    prm = workloads.DEBLUR1D_PARAMS
    sig = workloads.deblur_field()
    op = fftref.Operator(deblur.composite_generator(sig.c, prm["L"]), sig.d)
    y = op.A(sig.x_true.astype(np.float64)).astype(np.float32)
    c64 = sig.c.astype(np.float64)
    c_in = np.mean([np.roll(c64, -t) for t in range(prm["L"])], axis=0).astype(np.float32)
    lam, rho, T = prm["lam"], prm["rho"], prm["admm_iters"]
    (xo, zo, uo), hist = fftref.admm(op, y.astype(np.float64), lam, rho, T, record=True, record_every=100,
                                     callback=progress("deblur 1-D ADMM", every=100))
    x, z, u = (h(v) for v in cs.admm_solve(g(c_in), sig.d, g(y), lam, rho, T))
    y64 = y.astype(np.float64)
    fg = fftref.objective(op, y64, lam, z)
    fo = fftref.objective(op, y64, lam, zo)
    ef = abs(fg - fo) / fo
    ez100 = None
    x100, z100, _ = (h(v) for v in cs.admm_solve(g(c_in), sig.d, g(y), lam, rho, 100))
    ez100 = rel(z100, hist[0][2])
    print("deblur 1-D: z(100) rel err %.2e, F(z(%d)) rel err %.2e, z(T) rel err %.2e" % (ez100, T, ef, rel(z, zo)))
    assert ez100 <= IT_TOL and rel(x100, hist[0][1]) <= IT_TOL
    assert ef <= OBJ_TOL
