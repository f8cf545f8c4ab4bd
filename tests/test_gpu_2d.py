"""GPU parity of the 2-D path (A = P C H, 2x2 decimation) against the FP64
2-D oracle, through the C ABI.

Tolerances as in 1-D: operators relative l2 <= 1e-5 (one forward and one
inverse FP32 2-D transform); solver iterates relative l2 <= 1e-4 for every
compared iterate; final objective (oracle FP64 on both iterates) <= 1e-5.
"""
import numpy as np
import pytest

import workloads
from oracle import twod

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")
OP_TOL = 1e-5
IT_TOL = 1e-4
OBJ_TOL = 1e-5


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h_(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(R, C, n_src, seed, lam_frac=0.005):
    """A scene drawn like the 4096 x 4096 workload, at R x C."""
    return twod.build(workloads.draw_2d(np.random.default_rng(seed), R, C, n_src), lam_frac)


SHAPES = [(16, 16), (16, 64), (64, 16), (64, 64), (256, 128), (128, 512), (1024, 1024)]


@pytest.mark.parametrize("R,C", SHAPES)
@pytest.mark.parametrize("psf", [True, False])
def test_apply_and_transpose(R, C, psf):
    rng = np.random.default_rng(R * 7 + C)
    s = rng.choice([-1.0, 1.0], (R, C))
    hh = workloads.gaussian_psf(R, C) if psf else None
    op = twod.Operator2D(s, hh, 2, 2)
    x = rng.standard_normal((R, C))
    r = rng.standard_normal((R // 2, C // 2))
    sg, hg = g(s), (g(hh) if psf else None)
    y = h_(cs.apply2(sg, hg, g(x)))
    xt = h_(cs.apply2_T(sg, hg, g(r)))
    yr = op.A(x.astype(np.float32).astype(np.float64))
    xr = op.AT(r.astype(np.float32).astype(np.float64))
    assert rel(y, yr) <= OP_TOL, rel(y, yr)
    assert rel(xt, xr) <= OP_TOL, rel(xt, xr)


def test_structured_inputs():
    """An impulse image gives the kernel itself (decimated); a constant image
    gives sum(s) * sum(h) everywhere."""
    R, C = 64, 32
    rng = np.random.default_rng(2)
    s = rng.choice([-1.0, 1.0], (R, C))
    hh = workloads.gaussian_psf(R, C)
    op = twod.Operator2D(s, hh, 2, 2)
    e = np.zeros((R, C))
    e[0, 0] = 1.0
    y = h_(cs.apply2(g(s), g(hh), g(e)))
    assert rel(y, op.A(e.ravel())) <= OP_TOL
    y1 = h_(cs.apply2(g(s), g(hh), g(np.ones((R, C)))))
    ref = np.full((R // 2, C // 2), s.astype(np.float32).astype(np.float64).sum() * hh.astype(np.float32).astype(np.float64).sum())
    assert np.max(np.abs(y1 - ref)) <= 1e-5 * np.abs(s).sum()


@pytest.mark.parametrize("R,C", [(64, 64), (4096, 4096)])
def test_norm_bound(R, C):
    rng = np.random.default_rng(5)
    s = rng.choice([-1.0, 1.0], (R, C))
    hh = workloads.gaussian_psf(R, C)
    op = twod.Operator2D(s.astype(np.float32), hh.astype(np.float32), 2, 2)
    got = float(h_(cs.norm_bound2(g(s), g(hh)))[0])
    assert abs(got - op.max_chat_sq()) <= 1e-5 * op.max_chat_sq()


@pytest.mark.parametrize("R,C,rho", [(64, 64, 1.0), (64, 128, 300.0), (128, 64, 30.0)])
def test_admm_per_iterate(R, C, rho):
    pr = problem(R, C, 12, 40 + R + C)
    op = pr.op()
    y = pr.y.astype(np.float64).ravel()
    lam = float(pr.lam)
    T = 60
    _, hist = twod.admm(op, y, lam, rho, T, record=True)
    sg, hg, yg = g(pr.s), g(pr.h), g(pr.y)
    worst = 0.0
    nnz = 0
    for t in list(range(1, 21)) + [30, 45, 60]:
        x, z, u = (h_(v) for v in cs.admm_solve2(sg, hg, yg, pr.lam, rho, t))
        _, xo, zo, uo = hist[t - 1]
        ex = rel(x, xo)
        ez = rel(z, zo) if np.any(zo) else float(np.abs(z).max())
        worst = max(worst, ex, ez)
        nnz = max(nnz, int(np.count_nonzero(zo)))
        assert ex <= IT_TOL and ez <= IT_TOL, (t, ex, ez)
    print("2-D admm %dx%d rho=%g: worst rel err %.2e, max nnz(z) %d" % (R, C, rho, worst, nnz))


@pytest.mark.parametrize("R,C", [(64, 64), (128, 256)])
def test_ista_per_iterate(R, C):
    pr = problem(R, C, 10, 77 + R)
    op = pr.op()
    y = pr.y.astype(np.float64).ravel()
    lam, tau = float(pr.lam), float(pr.tau)
    T = 40
    _, hist = twod.ista(op, y, lam, tau, T, record=True)
    sg, hg, yg = g(pr.s), g(pr.h), g(pr.y)
    for t in list(range(1, 11)) + [20, 40]:
        x = h_(cs.ista_solve2(sg, hg, yg, pr.lam, pr.tau, t))
        e = rel(x, hist[t - 1][1])
        assert e <= IT_TOL, (t, e)


def test_admm_final_objective_and_trace():
    R, C, rho = 128, 128, 50.0
    pr = problem(R, C, 30, 9)
    op = pr.op()
    y = pr.y.astype(np.float64).ravel()
    lam = float(pr.lam)
    T = 200
    (xo, zo, uo), hist = twod.admm(op, y, lam, rho, T, record=True)
    obj = torch.empty(T, device=DEV, dtype=torch.float32)
    x, z, u = (h_(v) for v in cs.admm_solve2(g(pr.s), g(pr.h), g(pr.y), pr.lam, rho, T, obj=obj))
    fo, fg = twod.objective(op, y, lam, zo), twod.objective(op, y, lam, z.ravel())
    assert abs(fg - fo) <= OBJ_TOL * fo, (fg, fo)
    ref = np.array([twod.objective(op, y, lam, r[1]) for r in hist])
    err = np.abs(h_(obj) - ref) / ref
    print("2-D admm trace: worst rel err %.2e" % err.max())
    assert err.max() <= OBJ_TOL


def test_ista_trace():
    R, C = 64, 128
    pr = problem(R, C, 10, 19)
    op = pr.op()
    y = pr.y.astype(np.float64).ravel()
    lam, tau = float(pr.lam), float(pr.tau)
    T = 50
    _, hist = twod.ista(op, y, lam, tau, T, record=True)
    obj = torch.empty(T, device=DEV, dtype=torch.float32)
    cs.ista_solve2(g(pr.s), g(pr.h), g(pr.y), pr.lam, pr.tau, T, obj=obj)
    ref = np.array([twod.objective(op, y, lam, r[1]) for r in hist])
    assert np.max(np.abs(h_(obj) - ref) / ref) <= OBJ_TOL


def test_admm_warm_start_continues():
    R, C, rho = 64, 64, 20.0
    pr = problem(R, C, 12, 3)
    sg, hg, yg = g(pr.s), g(pr.h), g(pr.y)
    x, z, u = cs.admm_solve2(sg, hg, yg, pr.lam, rho, 25)
    x2, z2, u2 = cs.admm_solve2(sg, hg, yg, pr.lam, rho, 15, x=x.clone(), z=z.clone(), u=u.clone(), warm=True)
    xr, zr, ur = cs.admm_solve2(sg, hg, yg, pr.lam, rho, 40)
    assert rel(h_(x2), h_(xr)) <= 1e-6 and rel(h_(z2), h_(zr)) <= 1e-6


def test_zero_iterations_and_bad_arguments():
    R, C = 64, 64
    s = g(np.ones((R, C)))
    y = g(np.ones((R // 2, C // 2)))
    x = torch.full((R, C), 5.0, device=DEV)
    cs.ista_solve2(s, None, y, 0.1, 0.1, 0, x=x)
    assert float(h_(x).max()) == 0.0
    with pytest.raises(cs.CsError):
        cs.admm_solve2(s, None, y, 0.1, 0.0, 5)
    with pytest.raises(cs.CsError):
        cs.apply2(g(np.ones((48, 64))), None, g(np.ones((48, 64))))


# ----------------------------------------------------------------------------
# The 4096 x 4096 deblurring workload (20000 point sources, Gaussian PSF
# sigma = 2, +-1 sensing kernel, rho = 1)
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def scene_2d():
    pr = twod.build(workloads.scene_2d(), workloads.SCENE2D_PARAMS["lam_frac"])
    return pr, pr.op()


def test_scene_2d_operator_full_size(scene_2d):
    pr, op = scene_2d
    y = h_(cs.apply2(g(pr.s), g(pr.h), g(pr.x_true)))
    assert rel(y, pr.y.astype(np.float64)) <= OP_TOL


def test_scene_2d_first_iterates(scene_2d):
    pr, op = scene_2d
    y = pr.y.astype(np.float64).ravel()
    lam, rho = float(pr.lam), workloads.SCENE2D_PARAMS["rho"]
    _, hist = twod.admm(op, y, lam, rho, 3, record=True)
    sg, hg, yg = g(pr.s), g(pr.h), g(pr.y)
    for t in (1, 2, 3):
        x, z, u = (h_(v) for v in cs.admm_solve2(sg, hg, yg, pr.lam, rho, t))
        assert rel(x, hist[t - 1][1]) <= IT_TOL, t
        zo = hist[t - 1][2]
        assert (rel(z, zo) if np.any(zo) else np.abs(z).max()) <= IT_TOL, t


def test_scene_2d_full_run_trace(scene_2d):
    """200 iterations: the GPU's trace ends at the oracle's FP64 objective of
    the returned x, and the trace decreases from F(x_1)."""
    pr, op = scene_2d
    y = pr.y.astype(np.float64).ravel()
    lam, rho = float(pr.lam), workloads.SCENE2D_PARAMS["rho"]
    T = workloads.SCENE2D_PARAMS["admm_iters"]
    obj = torch.empty(T, device=DEV, dtype=torch.float32)
    x, z, u = cs.admm_solve2(g(pr.s), g(pr.h), g(pr.y), pr.lam, rho, T, obj=obj)
    f = h_(obj)
    ref = twod.objective(op, y, lam, h_(x).ravel())
    assert abs(f[-1] - ref) <= OBJ_TOL * ref, (f[-1], ref)
    assert f[-1] < f[0]
