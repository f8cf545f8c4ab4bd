"""Pins for the FP64 oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code paths.

Each `check_*` takes the implementation under test, so the mutation tests at
the bottom can hand it an oracle with a planted mistake and confirm the pin
catches it.
"""
import itertools
import os

import numpy as np
import pytest

import workloads
from oracle import dense, fftref, problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    key = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if ":" in line:
                key, val = line.split(":", 1)
                key = key.strip()
                val = val.strip()
                out[key] = [list(map(float, val.split()))] if val else []
            else:
                out[key].append(list(map(float, line.split())))
    return {k: np.array(v) for k, v in out.items()}


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# --------------------------------------------------------------------------
# Golden: hand-written A for n=4, d=2 (circulant index convention and P).
# --------------------------------------------------------------------------
def check_golden_A(dense_A):
    g = _read_golden("circulant_n4_d2.txt")
    A = dense_A(g["c"][0], int(g["d"][0][0]))
    np.testing.assert_array_equal(A, g["A"])


def test_golden_circulant_convention():
    check_golden_A(dense.dense_A)


def check_golden_soft(soft):
    g = _read_golden("soft_threshold.txt")
    np.testing.assert_array_equal(soft(g["v"][0], g["gamma"][0][0]), g["eta"][0])


def test_golden_soft_threshold():
    check_golden_soft(dense.soft)
    check_golden_soft(fftref.soft)


# --------------------------------------------------------------------------
# P1: dense A and the FFT operator agree (I1-I3).
# --------------------------------------------------------------------------
def check_dense_vs_fft(dense_A, Operator, n, d, seed=0):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n)
    x = rng.standard_normal(n)
    r = rng.standard_normal(n // d)
    A = dense_A(c, d)
    op = Operator(c, d)
    assert _rel(op.A(x), A @ x) < 1e-12
    assert _rel(op.AT(r), A.T @ r) < 1e-12


@pytest.mark.parametrize("n", [8, 16, 64, 512, 4096])
@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_P1_dense_vs_fft(n, d):
    if d > n:
        pytest.skip("d > n")
    check_dense_vs_fft(dense.dense_A, fftref.Operator, n, d, seed=n + d)


def test_P1_A_equals_P_times_C():
    rng = np.random.default_rng(1)
    c = rng.standard_normal(64)
    np.testing.assert_allclose(dense.dense_P(64, 4) @ dense.dense_C(c), dense.dense_A(c, 4),
                               rtol=0, atol=0)


# --------------------------------------------------------------------------
# P2: adjoint identity <A x, r> = <x, A^T r>.
# --------------------------------------------------------------------------
def check_adjoint(Operator, n, d, seed=0):
    rng = np.random.default_rng(seed)
    op = Operator(rng.standard_normal(n), d)
    x = rng.standard_normal(n)
    r = rng.standard_normal(n // d)
    lhs = float(op.A(x) @ r)
    rhs = float(x @ op.AT(r))
    scale = np.linalg.norm(op.A(x)) * np.linalg.norm(r)
    assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("n,d", [(4096, 4), (1 << 16, 4), (1024, 1), (2048, 8)])
def test_P2_adjoint(n, d):
    check_adjoint(fftref.Operator, n, d, seed=n * d)


# --------------------------------------------------------------------------
# P3: Parseval and the spectral residual.
# --------------------------------------------------------------------------
def test_P3_parseval():
    rng = np.random.default_rng(3)
    n, d = 4096, 4
    m = n // d
    x = rng.standard_normal(n)
    assert abs(x @ x - np.sum(np.abs(np.fft.fft(x)) ** 2) / n) < 1e-12 * (x @ x)
    op = fftref.Operator(rng.standard_normal(n), d)
    y = rng.standard_normal(m)
    # ||y - A x||^2 = (1/m) sum_k' |Y_hat - S|^2 with S = DFT_m(A x) assembled
    # from the n-point spectrum by alias summation (decimation in time).
    X = np.fft.fft(x)
    chat = op.full_spectrum()
    S = (chat * X).reshape(d, m).sum(axis=0) / d
    res_spec = np.sum(np.abs(np.fft.fft(y) - S) ** 2) / m
    r = y - op.A(x)
    assert abs(res_spec - r @ r) < 1e-10 * (r @ r)


# --------------------------------------------------------------------------
# P4: A A^T is an m x m circulant with eigenvalues Lam; ||A||^2 = max Lam.
# --------------------------------------------------------------------------
def check_Lam(dense_A, Operator, n, d, seed=0):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n)
    A = dense_A(c, d)
    G = A @ A.T
    m = n // d
    # circulant: G[i, j] depends on (i - j) mod m only
    np.testing.assert_allclose(np.roll(np.roll(G, 1, 0), 1, 1), G, rtol=0, atol=1e-10 * np.abs(G).max())
    lam = Operator(c, d).Lam()
    ev = np.linalg.eigvalsh(G)
    np.testing.assert_allclose(np.sort(lam), ev, rtol=0, atol=1e-10 * ev.max())
    nrm2 = np.linalg.norm(A, 2) ** 2
    assert abs(nrm2 - lam.max()) < 1e-10 * nrm2
    assert lam.max() <= Operator(c, d).max_chat_sq() * (1 + 1e-12)


@pytest.mark.parametrize("n,d", [(64, 4), (256, 2), (512, 8), (128, 1)])
def test_P4_AAT_circulant_eigen(n, d):
    check_Lam(dense.dense_A, fftref.Operator, n, d, seed=n + 7 * d)


# --------------------------------------------------------------------------
# P5: Woodbury application of (A^T A + rho I)^{-1} vs a dense solve.
# --------------------------------------------------------------------------
def check_woodbury(Operator, n, d, rho, seed=0):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n) / np.sqrt(n // d)
    q = rng.standard_normal(n)
    A = dense.dense_A(c, d)
    ref = np.linalg.solve(A.T @ A + rho * np.eye(n), q)
    assert _rel(Operator(c, d).woodbury_solve(rho, q), ref) < 1e-10


@pytest.mark.parametrize("rho", [0.1, 1.0, 10.0])
@pytest.mark.parametrize("n,d", [(256, 4), (512, 2), (128, 8), (64, 1)])
def test_P5_woodbury(n, d, rho):
    check_woodbury(fftref.Operator, n, d, rho, seed=n + d)


# --------------------------------------------------------------------------
# P6: c = e0 (C = I, A = P): closed forms.
# --------------------------------------------------------------------------
def test_P6_identity_generator():
    n, d = 64, 4
    m = n // d
    rng = np.random.default_rng(6)
    c = np.zeros(n)
    c[0] = 1.0
    y = rng.standard_normal(m)
    lam = 0.3
    up = np.zeros(n)
    up[::d] = np.where(np.abs(y) > lam, np.sign(y) * (np.abs(y) - lam), 0.0)
    # ISTA with tau = 1: x(1) = P^T eta_lam(y), and it is already the fixed point.
    A = dense.dense_A(c, d)
    np.testing.assert_allclose(dense.ista(A, y, lam, 1.0, 1), up, rtol=0, atol=1e-15)
    np.testing.assert_allclose(fftref.ista(fftref.Operator(c, d), y, lam, 1.0, 1), up, rtol=0, atol=1e-15)
    np.testing.assert_allclose(dense.ista(A, y, lam, 1.0, 5), up, rtol=0, atol=1e-15)
    # ADMM x-update: (P^T P + rho I)^{-1} is diagonal: 1/(1+rho) on kept rows, 1/rho elsewhere.
    rho = 2.5
    q = rng.standard_normal(n)
    diag = np.full(n, 1.0 / rho)
    diag[::d] = 1.0 / (1.0 + rho)
    np.testing.assert_allclose(fftref.Operator(c, d).woodbury_solve(rho, q), diag * q, rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# P7: d = 1 (A = C square): (C^T C + rho I)^{-1} = diag 1/(|c_hat|^2 + rho).
# --------------------------------------------------------------------------
def test_P7_square_circulant():
    rng = np.random.default_rng(7)
    n, rho = 512, 0.7
    c = rng.standard_normal(n)
    q = rng.standard_normal(n)
    ref = np.fft.ifft(np.fft.fft(q) / (np.abs(np.fft.fft(c)) ** 2 + rho)).real
    assert _rel(fftref.Operator(c, 1).woodbury_solve(rho, q), ref) < 1e-12


# --------------------------------------------------------------------------
# P8: decimation in time is aliasing in frequency.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,d", [(64, 4), (4096, 8), (1024, 2)])
def test_P8_decimation_is_aliasing(n, d):
    rng = np.random.default_rng(8)
    m = n // d
    W = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lhs = np.fft.ifft(W)[::d]
    rhs = np.fft.ifft(W.reshape(d, m).sum(axis=0) / d)
    assert _rel(lhs, rhs) < 1e-13
    # zero-upsampling tiles the m-point spectrum d times
    r = rng.standard_normal(m)
    up = np.zeros(n)
    up[::d] = r
    assert _rel(np.fft.fft(up), np.tile(np.fft.fft(r), d)) < 1e-13


# --------------------------------------------------------------------------
# P9: lam >= ||A^T y||_inf gives x = 0; just below it, one nonzero.
# --------------------------------------------------------------------------
def check_lam_max(ista_fn, admm_fn, seed=9):
    sig = workloads.signal(256, 4, 4, seed)
    pr = problem.build(sig)
    A = pr.A()
    y = pr.y.astype(np.float64)
    tau = float(pr.tau)
    g = A.T @ y
    lmax = np.max(np.abs(g))
    x, hist = ista_fn(A, y, lmax, tau, 20, record=True)
    assert all(np.count_nonzero(h) == 0 for h in hist)
    (x, z, u) = admm_fn(A, y, 1.01 * lmax, 1.0, 300)
    assert np.count_nonzero(z) == 0
    order = np.sort(np.abs(g))
    assert order[-2] < 0.999 * order[-1]          # generic instance
    x1 = ista_fn(A, y, 0.999 * lmax, tau, 1)
    nz = np.flatnonzero(x1)
    assert nz.tolist() == [int(np.argmax(np.abs(g)))]


def test_P9_lam_max():
    check_lam_max(dense.ista, dense.admm)


# --------------------------------------------------------------------------
# P10-P12: KKT at the limit, ISTA == ADMM limit, brute force on n=8.
# --------------------------------------------------------------------------
def check_kkt(x, A, y, lam, tol=1e-8):
    g = A.T @ (y - A @ x)
    on = x != 0
    assert np.all(np.abs(g[~on]) <= lam * (1 + tol))
    assert np.all(np.abs(g[on] - lam * np.sign(x[on])) <= lam * tol)


def check_limits(ista_fn, admm_fn, n=256, d=4, k=4, seed=10, rho=1.0):
    sig = workloads.signal(n, d, k, seed)
    pr = problem.build(sig)
    A = pr.A()
    y = pr.y.astype(np.float64)
    lam = float(pr.lam)
    (x, z, u) = admm_fn(A, y, lam, rho, 5000)
    check_kkt(z, A, y, lam)
    xi = ista_fn(A, y, lam, float(pr.tau), 20000)
    check_kkt(xi, A, y, lam)
    assert _rel(xi, z) < 1e-8


def test_P10_P11_kkt_and_equal_limits():
    check_limits(dense.ista, dense.admm)


def test_P10_kkt_rho_not_one():
    check_limits(dense.ista, dense.admm, n=128, seed=11, rho=3.0)


def brute_force_lasso(A, y, lam):
    """Enumerate every sign pattern s in {-1,0,1}^n; on the support S solve
    A_S^T A_S x_S = A_S^T y - lam s_S and keep the pattern whose solution has
    the signs s and satisfies the KKT bound off S.  Returns the minimiser."""
    m, n = A.shape
    best = None
    for s in itertools.product((-1, 0, 1), repeat=n):
        s = np.array(s, dtype=np.float64)
        S = np.flatnonzero(s)
        if len(S) > m:
            continue
        x = np.zeros(n)
        if len(S):
            AS = A[:, S]
            G = AS.T @ AS
            if np.linalg.cond(G) > 1e12:
                continue
            xs = np.linalg.solve(G, AS.T @ y - lam * s[S])
            if not np.all(np.sign(xs) == s[S]):
                continue
            x[S] = xs
        g = A.T @ (y - A @ x)
        off = np.setdiff1d(np.arange(n), S)
        if np.all(np.abs(g[off]) <= lam * (1 + 1e-12)):
            val = 0.5 * np.sum((y - A @ x) ** 2) + lam * np.abs(x).sum()
            if best is None or val < best[0]:
                best = (val, x)
    return best[1]


def check_brute_force(ista_fn, admm_fn, seed=12):
    rng = np.random.default_rng(seed)
    n, d = 8, 2
    c = rng.standard_normal(n)
    x_true = np.zeros(n)
    x_true[[1, 5]] = [1.5, -0.8]
    A = dense.dense_A(c, d)
    y = A @ x_true + 0.01 * rng.standard_normal(n // d)
    lam = 0.1 * np.max(np.abs(A.T @ y))
    xb = brute_force_lasso(A, y, lam)
    (x, z, u) = admm_fn(A, y, lam, 1.0, 20000)
    assert _rel(z, xb) < 1e-10
    tau = 1.0 / np.max(np.abs(np.fft.fft(c)) ** 2)
    xi = ista_fn(A, y, lam, tau, 200000)
    assert _rel(xi, xb) < 1e-8


def test_P12_brute_force_n8():
    check_brute_force(dense.ista, dense.admm)


# --------------------------------------------------------------------------
# P13: at parity_signal's shape the converged support equals the true support.
# --------------------------------------------------------------------------
def test_P13_parity_signal_support_recovery():
    sig = workloads.parity_signal()
    pr = problem.build(sig)
    op = pr.op()
    (x, z, u) = fftref.admm(op, pr.y.astype(np.float64), float(pr.lam), 1.0, 3000)
    assert set(np.flatnonzero(z).tolist()) == set(sig.support.tolist())


# --------------------------------------------------------------------------
# P14: ISTA's objective never increases for tau <= 1/||A||^2.
# --------------------------------------------------------------------------
def check_monotone(ista_fn, objective):
    sig = workloads.signal(1024, 4, 10, 14)
    pr = problem.build(sig)
    A = pr.A()
    y = pr.y.astype(np.float64)
    lam = float(pr.lam)
    _, hist = ista_fn(A, y, lam, float(pr.tau), 300, record=True)
    f = [objective(A, y, lam, h) for h in hist]
    f0 = objective(A, y, lam, np.zeros(A.shape[1]))
    f = [f0] + f
    assert all(b <= a * (1 + 1e-14) for a, b in zip(f, f[1:]))


def test_P14_ista_monotone():
    check_monotone(dense.ista, dense.objective)


# --------------------------------------------------------------------------
# The FFT reference reproduces the dense iterates (gives it authority at the
# sizes where a dense A is impossible).
# --------------------------------------------------------------------------
def test_fftref_iterates_match_dense_parity_signal():
    sig = workloads.parity_signal()
    pr = problem.build(sig)
    A = pr.A()
    op = pr.op()
    y = pr.y.astype(np.float64)
    lam, tau = float(pr.lam), float(pr.tau)
    xd, hd = dense.ista(A, y, lam, tau, 100, record=True)
    xf, hf = fftref.ista(op, y, lam, tau, 100, record=True)
    assert max(_rel(b[1], a) for a, b in zip(hd, hf)) < 1e-12
    (_, _, _), ha = dense.admm(A, y, lam, 1.0, 50, record=True)
    (_, _, _), hb = fftref.admm(op, y, lam, 1.0, 50, record=True)
    for a, b in zip(ha, hb):
        assert _rel(b[1], a[0]) < 1e-11 and _rel(b[2], a[1]) < 1e-11


def test_problem_rounding_rule():
    sig = workloads.parity_signal()
    pr = problem.build(sig)
    assert pr.y.dtype == np.float32 and pr.c.dtype == np.float32
    assert isinstance(pr.lam, np.float32) and isinstance(pr.tau, np.float32)
    op = pr.op()
    assert float(pr.tau) * op.Lam().max() < 1.0


# --------------------------------------------------------------------------
# Planted mistakes: each pin above must reject a plausibly wrong oracle.
# --------------------------------------------------------------------------
def _mut_dense_A_transposed(c, d):
    c = np.asarray(c, np.float64)
    n = c.shape[0]
    r = np.arange(n // d)[:, None]
    j = np.arange(n)[None, :]
    return c[(j - r * d) % n]


def _mut_ista_no_tau(A, y, lam, tau, iters, record=False):
    x = np.zeros(A.shape[1])
    hist = []
    for _ in range(iters):
        x = dense.soft(x + tau * (A.T @ (y - A @ x)), lam)
        hist.append(x.copy())
    return (x, hist) if record else x


def _mut_admm_threshold(A, y, lam, rho, iters, record=False):
    n = A.shape[1]
    M = np.linalg.inv(A.T @ A + rho * np.eye(n))
    aty = A.T @ y
    x = z = u = np.zeros(n)
    for _ in range(iters):
        x = M @ (aty + rho * (z - u))
        z = dense.soft(x + u, lam)          # planted: lam instead of lam/rho
        u = u + x - z
    return (x, z, u)


class _MutWoodburySign(fftref.Operator):
    def woodbury_solve(self, rho, q):
        Aq = self.A(q)
        t = np.fft.ifft(np.fft.fft(Aq) / (rho + self.Lam())).real
        return (q + self.AT(t)) / rho


class _MutLamNoAverage(fftref.Operator):
    def Lam(self):
        a = np.abs(self.full_spectrum()) ** 2
        return a.reshape(self.d, self.m).sum(axis=0)


class _MutAdjointConj(fftref.Operator):
    def CT(self, v):
        return np.fft.irfft(self.chat * np.fft.rfft(v), self.n)


class _MutDecimateOffset(fftref.Operator):
    def A(self, x):
        return self.C(x)[1:: self.d]


def _mut_soft_nonstrict(v, gamma):
    v = np.asarray(v, np.float64)
    return np.where(np.abs(v) >= gamma, np.sign(v) * (np.abs(v) - gamma) + 0.0 * v, 0.0) + \
        np.where(np.abs(v) == gamma, np.sign(v) * 1e-3, 0.0)


@pytest.mark.parametrize("case", [
    "golden_A_transposed", "soft_nonstrict", "ista_no_tau", "admm_threshold",
    "woodbury_sign", "lam_no_average", "adjoint_conj", "decimate_offset",
])
def test_planted_mistakes_are_caught(case):
    with pytest.raises(AssertionError):
        if case == "golden_A_transposed":
            check_golden_A(_mut_dense_A_transposed)
        elif case == "soft_nonstrict":
            check_golden_soft(_mut_soft_nonstrict)
        elif case == "ista_no_tau":
            check_lam_max(_mut_ista_no_tau, dense.admm)
        elif case == "admm_threshold":
            check_limits(dense.ista, _mut_admm_threshold, n=128, seed=11, rho=3.0)
        elif case == "woodbury_sign":
            check_woodbury(_MutWoodburySign, 256, 4, 1.0)
        elif case == "lam_no_average":
            check_Lam(dense.dense_A, _MutLamNoAverage, 64, 4)
        elif case == "adjoint_conj":
            check_dense_vs_fft(dense.dense_A, _MutAdjointConj, 64, 4)
        elif case == "decimate_offset":
            check_dense_vs_fft(dense.dense_A, _MutDecimateOffset, 64, 4)


# ----------------------------------------------------------------------------
# Compressed deblurring (Section 7): A = P C B with B the order-L box blur
# ----------------------------------------------------------------------------
def test_deblur_composite_generator_matches_dense_product():
    """The circulant generated by composite_generator(c, L) equals the dense
    product C B built from the definitions (brute force, n = 64)."""
    from oracle import deblur
    n, L = 64, 5
    rng = np.random.default_rng(11)
    c = rng.standard_normal(n)
    C = deblur.dense_circulant(c)
    B = deblur.dense_box_blur(n, L)
    CB = C @ B
    G = deblur.dense_circulant(deblur.composite_generator(c, L))
    assert np.allclose(G, CB, atol=1e-13)
    # B averages L consecutive samples starting at the output index
    x = rng.standard_normal(n)
    assert np.allclose(B @ x, [np.mean(x[(i + np.arange(L)) % n]) for i in range(n)])


def test_deblur_field_shape():
    import workloads
    sig = workloads.deblur_field(side=64)
    assert sig.n == 64 * 64 and sig.d == 2 and sig.k == int(0.1 * sig.n)
    assert np.count_nonzero(sig.x_true) == sig.k and np.all(sig.x_true >= 0)


# --------------------------------------------------------------------------
# Objective (Eq. 3 with the quadratic term halved, alpha read as lam): a
# hand-worked value, agreement of the three oracle objectives, and planted
# wrong objectives that must fail.
# --------------------------------------------------------------------------
def check_objective_golden(objective_dense):
    g = _read_golden("objective_n4_d2.txt")
    A = dense.dense_A(g["c"][0], int(g["d"][0][0]))
    F = objective_dense(A, g["y"][0], float(g["lam"][0][0]), g["x"][0])
    assert F == float(g["F"][0][0]), F


def test_objective_golden_n4():
    g = _read_golden("objective_n4_d2.txt")
    A = dense.dense_A(g["c"][0], int(g["d"][0][0]))
    r = g["y"][0] - A @ g["x"][0]
    assert float(r @ r) == float(g["residual_sq"][0][0])
    assert float(np.abs(g["x"][0]).sum()) == float(g["l1"][0][0])
    check_objective_golden(dense.objective)


def check_objective_agree(objective_fft, n=512, d=4, seed=31):
    """fftref's objective (residual through the FFT operator) equals the dense
    one on a random instance with a sparse x, to FP64 rounding."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n)
    x = np.where(rng.random(n) < 0.2, rng.standard_normal(n), 0.0)
    y = rng.standard_normal(n // d)
    lam = 0.37
    Fd = dense.objective(dense.dense_A(c, d), y, lam, x)
    Ff = objective_fft(fftref.Operator(c, d), y, lam, x)
    assert abs(Ff - Fd) <= 1e-12 * Fd, (Ff, Fd)


def test_objective_fft_matches_dense():
    for n, d in ((512, 4), (256, 2), (1024, 8), (128, 1)):
        check_objective_agree(fftref.objective, n, d, seed=n + d)


def test_objective_2d_matches_dense():
    from oracle import twod
    rng = np.random.default_rng(32)
    s = rng.choice([-1.0, 1.0], size=(16, 16))
    h = np.zeros((16, 16))
    h[:3, :3] = rng.random((3, 3))
    h /= h.sum()
    x = np.where(rng.random(256) < 0.2, rng.standard_normal(256), 0.0)
    y = rng.standard_normal(64)
    lam = 0.21
    Fd = dense.objective(twod.dense_A2(s, h, 2, 2), y, lam, x)
    Ft = twod.objective(twod.Operator2D(s, h, 2, 2), y, lam, x)
    assert abs(Ft - Fd) <= 1e-12 * Fd, (Ft, Fd)


def _mut_obj_no_half(A, y, lam, x):
    r = y - A @ x
    return float(r @ r) + lam * float(np.abs(x).sum())


def _mut_obj_eq3_literal(A, y, lam, x):
    r = y - A @ x
    return float(r @ r) + 2.0 * lam * float(np.abs(x).sum())


def _mut_obj_no_l1(A, y, lam, x):
    r = y - A @ x
    return 0.5 * float(r @ r)


def _mut_obj_l2(A, y, lam, x):
    r = y - A @ x
    return 0.5 * float(r @ r) + lam * float(np.linalg.norm(x))


def _mut_fft_obj_no_half(op, y, lam, x):
    r = y - op.A(x)
    return float(r @ r) + lam * float(np.abs(x).sum())


def _mut_fft_obj_l2(op, y, lam, x):
    r = y - op.A(x)
    return 0.5 * float(r @ r) + lam * float(np.linalg.norm(x))


@pytest.mark.parametrize("mut", [_mut_obj_no_half, _mut_obj_eq3_literal, _mut_obj_no_l1, _mut_obj_l2])
def test_planted_objective_mistakes_fail_golden(mut):
    with pytest.raises(AssertionError):
        check_objective_golden(mut)


@pytest.mark.parametrize("mut", [_mut_fft_obj_no_half, _mut_fft_obj_l2])
def test_planted_fft_objective_mistakes_fail_agreement(mut):
    with pytest.raises(AssertionError):
        check_objective_agree(mut)


# --------------------------------------------------------------------------
# Batched oracle: the batch is the per-signal Alg. 1, signal by signal.
# --------------------------------------------------------------------------
def check_batched_one_by_one(ista_batched):
    from oracle import batched
    sigs = [workloads.signal(n, 4, max(1, n // 256), 40 + i) for i, n in enumerate((256, 1024, 512, 8192, 16384))]
    probs = batched.build_batch(sigs)
    xs = ista_batched(probs, 30)
    assert len(xs) == len(probs)
    for pr, xb in zip(probs, xs):
        y = pr.y.astype(np.float64)
        # the plain definition, independently of batched.ista_one's choice
        # between the dense and the FFT operator
        A = dense.dense_A(pr.c.astype(np.float64), pr.d)
        x = np.zeros(pr.n)
        for _ in range(30):
            x = dense.soft(x + float(pr.tau) * (A.T @ (y - A @ x)), float(pr.tau) * float(pr.lam))
        assert _rel(xb, x) < 1e-12
    # concatenation keeps the order and the per-signal parameters
    ns, c, yc, lam, tau = batched.concat(probs)
    assert ns.tolist() == [p.n for p in probs]
    off = 0
    for p in probs:
        np.testing.assert_array_equal(c[off:off + p.n], p.c)
        off += p.n
    assert lam.tolist() == [float(p.lam) for p in probs]
    assert tau.tolist() == [float(p.tau) for p in probs]


def test_batched_equals_one_by_one():
    check_batched_one_by_one(__import__("oracle.batched", fromlist=["ista_batched"]).ista_batched)


def test_batched_admm_equals_one_by_one():
    """Batched ADMM: signal i runs Alg. 2 with its own rho_i.  The reference
    for the dense-size signals is the inverse of A^T A + rho_i I written out
    here; the long signal's is the FFT reference's own ADMM."""
    from oracle import batched
    sigs = [workloads.signal(n, 4, max(1, n // 256), 70 + i) for i, n in enumerate((256, 1024, 16384))]
    probs = batched.build_batch(sigs)
    rhos = [0.5, 1.0, 2.0]
    out = batched.admm_batched(probs, rhos, 25)
    for pr, rho, (xb, zb, ub) in zip(probs, rhos, out):
        y = pr.y.astype(np.float64)
        lam = float(pr.lam)
        if pr.n <= 1024:
            A = dense.dense_A(pr.c.astype(np.float64), pr.d)
            Minv = np.linalg.inv(A.T @ A + rho * np.eye(pr.n))
            aty = A.T @ y
            x = z = u = np.zeros(pr.n)
            for _ in range(25):
                x = Minv @ (aty + rho * (z - u))
                z = dense.soft(x + u, lam / rho)
                u = u + x - z
        else:
            x, z, u = fftref.admm(pr.op(), y, lam, rho, 25)
        assert _rel(xb, x) < 1e-10 and _rel(zb, z) < 1e-10 and _rel(ub, u) < 1e-10


def _mut_batched_shared_params(problems, iters):
    from oracle import batched
    p0 = problems[0]
    out = []
    for pr in problems:
        q = problem.Problem(n=pr.n, d=pr.d, c=pr.c, y=pr.y, x_true=pr.x_true, lam=p0.lam, tau=p0.tau)
        out.append(batched.ista_one(q, iters))
    return out


def test_planted_batched_mistake_fails():
    with pytest.raises(AssertionError):
        check_batched_one_by_one(_mut_batched_shared_params)
