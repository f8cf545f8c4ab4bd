"""Seeded synthetic inputs for partial-circulant LASSO recovery.

This module only draws random numbers and rounds them to float32.  It holds
none of the method's arithmetic: no products with the sensing matrix, no FFT,
no thresholds.  Both the FP64 oracle (tests) and the HIP path (tests, bench)
take their inputs from here, so neither needs the other to build a workload.

Workload shapes follow the paper's synthetic experiments (Section 6: Gaussian
nonzeros at random positions, a Gaussian circulant generator) at these sizes:

  parity_signal   n=4096, d=4, k=40: the parity case
  large_signal    n=2^22, d=4, k=2^14: the large single signal
  scene_2d        4096x4096 scene, 20000 lognormal point sources, +-1 2-D
                  sensing kernel, sigma=2 Gaussian PSF truncated to 15x15,
                  2x decimation per axis
  uneven_batch    512 signals, n_i = 2^e, e uniform in {12..18}, d=4,
                  k_i=n_i/256
  shared_c_batch  shared generator, n=2^16, d=4, batch 64 signals with k=256
  deblur_field    1024x1024 field vectorised, 10% lognormal pixels, d=2
  random_rows_signal  1-D draw with a random row set Omega (|Omega| = m)
                  for the circulant ADMM of Section 4.3

Every draw is made in float64 and then rounded to float32 (the arrays handed to
both sides are those float32 values).  The generator c has entries
N(0, 1/m), i.e. standard deviation m^{-1/2}.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_BASE = 17070224


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32)


@dataclasses.dataclass
class Signal1D:
    """One 1-D draw: circulant generator c (first column), sparse truth x*."""
    n: int
    d: int
    k: int
    c: np.ndarray        # float32, length n
    x_true: np.ndarray   # float32, length n, k nonzeros
    support: np.ndarray  # int64, sorted positions of the nonzeros

    @property
    def m(self) -> int:
        return self.n // self.d


def draw_1d(rng: np.random.Generator, n: int, d: int, k: int) -> Signal1D:
    """Draw c ~ N(0,1/m) (length n), then a support of k distinct positions,
    then k N(0,1) values.  This draw order is fixed."""
    m = n // d
    c = rng.standard_normal(n) / np.sqrt(m)
    supp = rng.choice(n, k, replace=False)
    vals = rng.standard_normal(k)
    x = np.zeros(n)
    x[supp] = vals
    return Signal1D(n=n, d=d, k=k, c=_f32(c), x_true=_f32(x),
                    support=np.sort(supp.astype(np.int64)))


def signal(n: int, d: int, k: int, seed: int) -> Signal1D:
    """A 1-D draw of arbitrary size (test cases)."""
    return draw_1d(np.random.default_rng(seed), n, d, k)


def parity_signal(seed_offset: int = 0) -> Signal1D:
    return draw_1d(np.random.default_rng(SEED_BASE + 1 + seed_offset), 4096, 4, 40)


def large_signal(seed_offset: int = 0) -> Signal1D:
    return draw_1d(np.random.default_rng(SEED_BASE + 2 + seed_offset), 1 << 22, 4, 1 << 14)


PARITY_PARAMS = dict(ista_iters=500, admm_iters=200, rho=1.0, lam_frac=0.01)
LARGE_PARAMS = dict(ista_iters=300, admm_iters=100, rho=1.0, lam_frac=0.01)


@dataclasses.dataclass
class Scene2D:
    """2-D draw: sensing kernel s (+-1, full grid), PSF h (wrapped, sum 1),
    sparse scene x*."""
    n1: int
    n2: int
    d1: int
    d2: int
    s: np.ndarray        # float32 (n1, n2)
    h: np.ndarray        # float32 (n1, n2), wrapped PSF
    x_true: np.ndarray   # float32 (n1, n2)


def gaussian_psf(n1: int, n2: int, sigma: float = 2.0, half: int = 7) -> np.ndarray:
    """exp(-(a^2+b^2)/(2 sigma^2)) for a,b in [-half, half], normalised to sum
    one, placed periodically at (a mod n1, b mod n2)."""
    a = np.arange(-half, half + 1)
    g = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * sigma * sigma))
    g /= g.sum()
    h = np.zeros((n1, n2))
    for i, ai in enumerate(a):
        for j, bj in enumerate(a):
            h[ai % n1, bj % n2] += g[i, j]
    return h


def draw_2d(rng: np.random.Generator, n1: int, n2: int, n_src: int,
            sigma: float = 2.0, half: int = 7) -> Scene2D:
    """Draw order: source positions, lognormal(0,1) amplitudes, +-1 kernel."""
    pos = rng.choice(n1 * n2, n_src, replace=False)
    amp = rng.lognormal(0.0, 1.0, n_src)
    s = rng.choice(np.array([-1.0, 1.0]), (n1, n2))
    x = np.zeros(n1 * n2)
    x[pos] = amp
    h = gaussian_psf(n1, n2, sigma, half)
    return Scene2D(n1=n1, n2=n2, d1=2, d2=2, s=_f32(s), h=_f32(h),
                   x_true=_f32(x.reshape(n1, n2)))


def scene_2d(seed_offset: int = 0) -> Scene2D:
    return draw_2d(np.random.default_rng(SEED_BASE + 3 + seed_offset), 4096, 4096, 20000)


SCENE2D_PARAMS = dict(admm_iters=200, rho=1.0, lam_frac=0.005)


def uneven_batch(seed_offset: int = 0, count: int = 512, e_lo: int = 12, e_hi: int = 18):
    """Batched uneven sizes: all exponents first, then each signal's draws in
    the 1-D order (c, support, values); k_i = n_i/256."""
    rng = np.random.default_rng(SEED_BASE + 4 + seed_offset)
    e = rng.integers(e_lo, e_hi + 1, size=count)
    out = []
    for ei in e:
        n = 1 << int(ei)
        out.append(draw_1d(rng, n, 4, n // 256))
    return out


UNEVEN_PARAMS = dict(ista_iters=200, lam_frac=0.01)


def shared_c_batch(seed_offset: int = 0, n: int = 1 << 16, d: int = 4, batch: int = 64, k: int = 256):
    """Shared generator c, then `batch` sparse truths (support, values)."""
    rng = np.random.default_rng(SEED_BASE + 5 + seed_offset)
    m = n // d
    c = _f32(rng.standard_normal(n) / np.sqrt(m))
    xs = np.zeros((batch, n))
    for b in range(batch):
        supp = rng.choice(n, k, replace=False)
        xs[b, supp] = rng.standard_normal(k)
    return c, _f32(xs)


SHARED_C_PARAMS = dict(K=50, every=10, lam_frac=0.01)


def deblur_field(seed_offset: int = 0, side: int = 1024, frac: float = 0.1):
    """The deblurring shape of Section 7 on a synthetic field: a side x side
    image vectorised (n = side^2), about frac * n nonzero pixels with
    lognormal(0, 1) intensities at uniform positions (a star field standing
    in for the telescope image, which is not available), a Gaussian
    generator c ~ N(0, 1/m) with m = n/2 (d = 2).  The 1-D box blur of order
    DEBLUR1D_PARAMS["L"] that the sensing operator composes with c is not
    applied here.  Draw order: c, support, values."""
    rng = np.random.default_rng(SEED_BASE + 6 + seed_offset)
    n = side * side
    d = 2
    m = n // d
    k = int(frac * n)
    c = rng.standard_normal(n) / np.sqrt(m)
    supp = rng.choice(n, k, replace=False)
    vals = rng.lognormal(0.0, 1.0, k)
    x = np.zeros(n)
    x[supp] = vals
    return Signal1D(n=n, d=d, k=k, c=_f32(c), x_true=_f32(x), support=np.sort(supp.astype(np.int64)))


DEBLUR1D_PARAMS = dict(L=5, admm_iters=300, rho=1.0, lam=1e-2)


def random_rows_signal(n: int, m: int, k: int, seed: int):
    """A 1-D draw for the random-row partial circulant of Section 4.3: c ~
    N(0, 1/m) (length n), a support of k distinct positions with N(0,1)
    values, then Omega, m distinct rows out of n (sorted).  Returns
    (Signal1D with d = 0, omega)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n) / np.sqrt(m)
    supp = rng.choice(n, k, replace=False)
    vals = rng.standard_normal(k)
    omega = np.sort(rng.choice(n, m, replace=False)).astype(np.int64)
    x = np.zeros(n)
    x[supp] = vals
    sig = Signal1D(n=n, d=0, k=k, c=_f32(c), x_true=_f32(x), support=np.sort(supp.astype(np.int64)))
    return sig, omega


def random_rows_large(seed_offset: int = 0):
    """The random-row workload at the large single-signal size: n = 2^22,
    m = n/2 rows drawn at random, k = n/10 nonzeros (the paper's Section 6
    proportions m = n/2, k about n/10)."""
    n = 1 << 22
    return random_rows_signal(n, n // 2, n // 10, SEED_BASE + 7 + seed_offset)


RANDOM_ROWS_PARAMS = dict(alpha_frac=0.01, rho=1.0, sigma=1.0, tau=1.0, iters=100)


def recovery_signal(seed_offset: int = 0):
    """The recovery-time study of Section 6 (MSE over time at n = 2^15):
    m = n/2 (every other row, d = 2), k = n/10 N(0,1) nonzeros, c ~ N(0, 1/m).
    Same draw order as draw_1d."""
    n = 1 << 15
    return draw_1d(np.random.default_rng(SEED_BASE + 8 + seed_offset), n, 2, n // 10)


def recovery_random_rows(seed_offset: int = 0):
    """The same study with m = n/2 rows drawn at random (the paper's sampling),
    for the circulant ADMM of Section 4.3."""
    n = 1 << 15
    return random_rows_signal(n, n // 2, n // 10, SEED_BASE + 9 + seed_offset)


# Section 6 sets alpha = 1e-4 and sigma = tau = 0.1 with an MSE target of
# 1e-4.  Read here as: lambda = alpha (absolute), the ISTA step tau = 0.1
# (below 2 / ||A||^2 for these draws), rho = sigma = 0.1 for ADMM (Alg. 2) and
# the circulant ADMM (Alg. 3), whose multiplier step is 1 (inside the quoted
# convergence range (0, (1 + sqrt 5)/2)).  Checkpoints: iteration counts at
# which the MSE is measured (each a solve from zero).
RECOVERY_PARAMS = dict(
    lam=1e-4, ista_tau=0.1, rho=0.1, sigma=0.1, cp_tau=1.0, target_mse=1e-4,
    ista_checkpoints=[1, 2, 5, 10, 20, 50, 100, 200, 500, 1000, 2000, 5000, 10000, 20000, 40000, 60000, 80000,
                      100000, 120000, 150000],
    admm_checkpoints=[1, 2, 5, 10, 20, 50, 100, 200, 500, 800, 1000, 1100, 1200, 1500, 2000, 3000],
    cpadmm_checkpoints=[1, 2, 5, 10, 20, 50, 100, 200, 500, 1000, 2000, 2500, 3000, 4000, 5000],
)
