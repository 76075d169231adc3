"""Seeded synthetic workloads (inputs only).

This module synthesises datasets, priors and SMC sizes. It holds none of the
method's arithmetic: no estimator, control variate, weight, or move. Both the
GPU path and the CPU oracle receive exactly the arrays produced here.

Row layout of a dataset (both precisions): row k holds x_k in columns
0..d-1, y_k in column d and zeros up to the row pitch `ld`, which is rounded
up so that every row is a whole number of 64-byte segments.

The data of configuration k come from numpy's Philox generator with key
1000+k (stream 0 for the true coefficients, stream 1+c for row chunk c of
2**18 rows), so any row range can be regenerated without the rest. The SMC
seed of configuration k is 2000+k.
"""
from dataclasses import dataclass, field
import math

import numpy as np

LOGISTIC, POISSON, GAUSSIAN, STUDENT_T = 0, 1, 2, 3
FP64, MIXED = 0, 1
CHUNK = 1 << 18


def row_pitch(d: int, itemsize: int) -> int:
    per64 = 64 // itemsize
    return ((d + 1 + per64 - 1) // per64) * per64


def _gen(key: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(key) + (int(stream) << 64)))


@dataclass
class Workload:
    name: str
    family: int
    precision: int
    n: int
    d: int
    X: np.ndarray                 # n x d float64 (already rounded to fp32 for MIXED data)
    y: np.ndarray                 # n float64
    prior_mean: np.ndarray
    prior_prec: np.ndarray
    M: int
    m: int
    G: int
    L: int
    seed: int
    theta_true: np.ndarray = None
    gauss_s2: float = 1.0
    ess_frac: float = 0.5
    extra: dict = field(default_factory=dict)
    dataset: int = 0              # dataset field of the random-number counters (batch member index)

    def Xy(self, dtype) -> np.ndarray:
        """Row-major [x | y | 0-padding] array in the given dtype."""
        dt = np.dtype(dtype)
        ld = row_pitch(self.d, dt.itemsize)
        out = np.zeros((self.n, ld), dtype=dt)
        out[:, : self.d] = self.X
        out[:, self.d] = self.y
        return out

    @property
    def data_dtype(self):
        return np.float64 if self.precision == FP64 else np.float32


def _finish(X, y, precision):
    if precision == MIXED:
        X = X.astype(np.float32).astype(np.float64)
        y = y.astype(np.float32).astype(np.float64)
    return np.ascontiguousarray(X), np.ascontiguousarray(y)


# ---------------------------------------------------------------------------
# benchmark configurations
# ---------------------------------------------------------------------------

def config1(n=10_000):
    """Logistic, n=10,000, d=5 (intercept + 4 N(0,1) covariates), FP64."""
    key, d = 1001, 5
    theta = _gen(key, 0).standard_normal(d)
    X = np.empty((n, d))
    y = np.empty(n)
    for c0 in range(0, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        g = _gen(key, 1 + c0 // CHUNK)
        X[c0:c1, 0] = 1.0
        X[c0:c1, 1:] = g.standard_normal((c1 - c0, d - 1))
        p = 1.0 / (1.0 + np.exp(-(X[c0:c1] @ theta)))
        y[c0:c1] = (g.random(c1 - c0) < p).astype(np.float64)
    X, y = _finish(X, y, FP64)
    return Workload("logistic_n1e4_d5_fp64", LOGISTIC, FP64, n, d, X, y, np.zeros(d), np.eye(d) / 10.0,
                    M=256, m=500, G=4, L=10, seed=2001, theta_true=theta)


def config2(n=1_000_000, M=2048, m=5000):
    """Poisson log link, n=1e6, d=20, covariates N(0, 1/d) iid, FP32 data."""
    key, d = 1002, 20
    theta = _gen(key, 0).normal(0.0, 0.5, d)
    X = np.empty((n, d))
    y = np.empty(n)
    for c0 in range(0, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        g = _gen(key, 1 + c0 // CHUNK)
        X[c0:c1] = g.normal(0.0, 1.0 / math.sqrt(d), (c1 - c0, d))
        y[c0:c1] = g.poisson(np.exp(X[c0:c1] @ theta)).astype(np.float64)
    X, y = _finish(X, y, MIXED)
    return Workload("poisson_n1e6_d20_fp32data", POISSON, MIXED, n, d, X, y, np.zeros(d), np.eye(d),
                    M=M, m=m, G=100, L=20, seed=2002, theta_true=theta)


def config4(n=10_000_000, M=4096, m=20_000):
    """Logistic, n=1e7, d=50, heavy-tailed covariates t5 scaled to unit variance, FP32 data."""
    key, d = 1004, 50
    theta = _gen(key, 0).normal(0.0, math.sqrt(0.1), d)
    X = np.empty((n, d))
    y = np.empty(n)
    for c0 in range(0, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        g = _gen(key, 1 + c0 // CHUNK)
        X[c0:c1, 0] = 1.0
        X[c0:c1, 1:] = g.standard_t(5, (c1 - c0, d - 1)) * math.sqrt(3.0 / 5.0)
        p = 1.0 / (1.0 + np.exp(-(X[c0:c1] @ theta)))
        y[c0:c1] = (g.random(c1 - c0) < p).astype(np.float64)
    X, y = _finish(X, y, MIXED)
    return Workload("logistic_n1e7_d50_t5_fp32data", LOGISTIC, MIXED, n, d, X, y, np.zeros(d), np.eye(d) / 10.0,
                    M=M, m=m, G=100, L=15, seed=2004, theta_true=theta)


def _spline_prior(nb: int) -> np.ndarray:
    """Gaussian random-walk (second difference) smoothing prior, precision D2'D2/tau2 + kappa I."""
    D2 = np.zeros((nb - 2, nb))
    for i in range(nb - 2):
        D2[i, i], D2[i, i + 1], D2[i, i + 2] = 1.0, -2.0, 1.0
    return D2.T @ D2 / 1.0 + 1.0 * np.eye(nb)


def config5(n=5_000_000, M=4096, m=50_000):
    """Additive logistic model: 5 AR(1) covariates, cubic B-splines (20 interior knots), d=116."""
    from scipy.interpolate import BSpline
    from scipy.stats import norm

    key, p, rho = 1005, 5, 0.5
    inner = norm.ppf(np.arange(1, 21) / 21.0)
    lo, hi = -6.5, 6.5
    knots = np.concatenate([[lo] * 4, inner, [hi] * 4])
    nb = len(knots) - 4            # 24 basis functions
    d = 1 + p * (nb - 1)           # first basis of each covariate dropped
    X = np.empty((n, d))
    y = np.empty(n)
    for c0 in range(0, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        g = _gen(key, 1 + c0 // CHUNK)
        z = np.empty((c1 - c0, p))
        z[:, 0] = g.standard_normal(c1 - c0)
        for j in range(1, p):
            z[:, j] = rho * z[:, j - 1] + math.sqrt(1 - rho * rho) * g.standard_normal(c1 - c0)
        z = np.clip(z, lo, hi - 1e-9)
        X[c0:c1, 0] = 1.0
        for j in range(p):
            Bm = BSpline.design_matrix(z[:, j], knots, 3).toarray()
            X[c0:c1, 1 + j * (nb - 1): 1 + (j + 1) * (nb - 1)] = Bm[:, 1:]
        eta = -1 + np.sin(z[:, 0]) + 0.5 * (z[:, 1] ** 2 - 1) + 0.8 * np.tanh(z[:, 2]) - 0.5 * z[:, 3]
        y[c0:c1] = (g.random(c1 - c0) < 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    X, y = _finish(X, y, MIXED)
    Q0 = np.zeros((d, d))
    Q0[0, 0] = 1.0 / 10.0
    blk = _spline_prior(nb - 1)
    for j in range(p):
        s = 1 + j * (nb - 1)
        Q0[s:s + nb - 1, s:s + nb - 1] = blk
    return Workload("gam_logistic_n5e6_d116_fp32data", LOGISTIC, MIXED, n, d, X, y, np.zeros(d), Q0,
                    M=M, m=m, G=100, L=20, seed=2005)


def student_t(n=500_000, d=50, M=2048, m=1250, L=15):
    """Student-t regression of Experiment 2: y = x'theta + e, e ~ t_5; covariates with unit variances and
    pairwise correlations 0.9; theta ~ U(-5, 5); prior N(0, 10 I); m = 0.0025 n; FP32 data."""
    key = 1006
    theta = _gen(key, 0).uniform(-5.0, 5.0, d)
    X = np.empty((n, d))
    y = np.empty(n)
    for c0 in range(0, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        g = _gen(key, 1 + c0 // CHUNK)
        z0 = g.standard_normal((c1 - c0, 1))
        X[c0:c1] = math.sqrt(0.9) * z0 + math.sqrt(0.1) * g.standard_normal((c1 - c0, d))
        y[c0:c1] = X[c0:c1] @ theta + g.standard_t(5, c1 - c0)
    X, y = _finish(X, y, MIXED)
    return Workload("student_t_n5e5_d50_rho09_fp32data", STUDENT_T, MIXED, n, d, X, y, np.zeros(d),
                    np.eye(d) / 10.0, M=M, m=m, G=100, L=L, seed=2006, theta_true=theta)


def _config3_draw(b):
    g = _gen(1300 + b, 0)
    n = int(round(math.exp(g.uniform(math.log(1e4), math.log(2e6)))))
    d = int(g.integers(5, 51))
    return n, d, g


def config3_sizes(count=64):
    """(n_b, d_b) of the batched configuration: n log-uniform in [1e4, 2e6], d uniform in {5..50}."""
    nd = [_config3_draw(b)[:2] for b in range(count)]
    return np.array([x[0] for x in nd], dtype=np.int64), np.array([x[1] for x in nd], dtype=np.int64)


def config3_member(b, count=64, precision=MIXED, M=1024):
    """Dataset b of the batched configuration: logistic regression, x = [1, N(0,1)^(d-1)],
    theta_true ~ N(0, I), prior N(0, 10 I), P = 1024, m = max(200, round(0.01 n)), G = 100, L = 10.
    Dataset b draws n, d and theta_true from stream 0 of Philox key 1300 + b and row chunk c
    from stream 1 + c; every dataset uses SMC seed 2003 with b as the dataset counter field."""
    n, d, g0 = _config3_draw(b)
    key = 1300 + b
    theta = g0.standard_normal(d)
    X = np.empty((n, d))
    y = np.empty(n)
    for c0 in range(0, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        g = _gen(key, 1 + c0 // CHUNK)
        X[c0:c1, 0] = 1.0
        X[c0:c1, 1:] = g.standard_normal((c1 - c0, d - 1))
        p = 1.0 / (1.0 + np.exp(-(X[c0:c1] @ theta)))
        y[c0:c1] = (g.random(c1 - c0) < p).astype(np.float64)
    X, y = _finish(X, y, precision)
    m = max(200, int(round(0.01 * n)))
    return Workload(f"batch{count}_b{b}_logistic_n{n}_d{d}", LOGISTIC, precision, n, d, X, y, np.zeros(d),
                    np.eye(d) / 10.0, M=M, m=m, G=100, L=10, seed=2003, theta_true=theta, dataset=b)


CONFIGS = {1: config1, 2: config2, 4: config4, 5: config5}


# ---------------------------------------------------------------------------
# small test workloads
# ---------------------------------------------------------------------------

def logistic_small(n, d, seed, precision=FP64, intercept=True, M=64, m=100, G=4, L=8, prior_var=10.0,
                   theta_scale=1.0):
    g = _gen(5000 + seed, 0)
    theta = theta_scale * g.standard_normal(d)
    X = g.standard_normal((n, d))
    if intercept:
        X[:, 0] = 1.0
    y = (g.random(n) < 1.0 / (1.0 + np.exp(-(X @ theta)))).astype(np.float64)
    X, y = _finish(X, y, precision)
    return Workload(f"logistic_n{n}_d{d}", LOGISTIC, precision, n, d, X, y, np.zeros(d), np.eye(d) / prior_var,
                    M=M, m=m, G=G, L=L, seed=7000 + seed, theta_true=theta)


def poisson_small(n, d, seed, precision=FP64, M=64, m=100, G=4, L=8):
    g = _gen(6000 + seed, 0)
    theta = g.normal(0.0, 0.5, d)
    X = g.normal(0.0, 1.0 / math.sqrt(d), (n, d))
    y = g.poisson(np.exp(X @ theta)).astype(np.float64)
    X, y = _finish(X, y, precision)
    return Workload(f"poisson_n{n}_d{d}", POISSON, precision, n, d, X, y, np.zeros(d), np.eye(d),
                    M=M, m=m, G=G, L=L, seed=8000 + seed, theta_true=theta)


def student_small(n, d, seed, precision=FP64, M=64, m=100, G=4, L=8, prior_var=10.0, theta_scale=1.0):
    """Student-t regression (t_5 errors, unit scale) with an intercept."""
    g = _gen(9700 + seed, 0)
    theta = theta_scale * g.uniform(-1.0, 1.0, d)
    X = g.standard_normal((n, d))
    X[:, 0] = 1.0
    y = X @ theta + g.standard_t(5, n)
    X, y = _finish(X, y, precision)
    return Workload(f"student_n{n}_d{d}", STUDENT_T, precision, n, d, X, y, np.zeros(d), np.eye(d) / prior_var,
                    M=M, m=m, G=G, L=L, seed=9900 + seed, theta_true=theta)


def gaussian_small(n, d, seed, s2=1.0, precision=FP64, M=64, m=50, G=4, L=8, prior_var=4.0):
    """Linear regression with known noise variance s2 (conjugate test family)."""
    g = _gen(9000 + seed, 0)
    theta = g.standard_normal(d)
    X = g.standard_normal((n, d))
    X[:, 0] = 1.0
    y = X @ theta + math.sqrt(s2) * g.standard_normal(n)
    X, y = _finish(X, y, precision)
    mu0 = 0.1 * np.arange(d, dtype=np.float64)
    Q0 = np.eye(d) / prior_var + 0.05 * np.ones((d, d)) / d
    return Workload(f"gaussian_n{n}_d{d}", GAUSSIAN, precision, n, d, X, y, mu0, Q0,
                    M=M, m=m, G=G, L=L, seed=9500 + seed, theta_true=theta, gauss_s2=s2)


def batched_small(count, seed, precision=FP64, M=48, L=6, n_range=(600, 6000), d_values=None):
    """Small members of a batch for parity: logistic data as in logistic_small with per-member n
    log-uniform in n_range and d from d_values (default: uniform in 2..40, so narrow and lane-group
    rows both occur), m = max(40, n // 40), G = 4, member k with dataset field k."""
    g = _gen(9800 + seed, 0)
    out = []
    for k in range(count):
        n = int(math.exp(g.uniform(math.log(n_range[0]), math.log(n_range[1]))))
        d = int(d_values[k % len(d_values)]) if d_values is not None else int(g.integers(2, 41))
        w = logistic_small(n, d, seed=1000 * seed + k, precision=precision, M=M, m=max(40, n // 40), G=4, L=L,
                           theta_scale=min(1.0, 2.0 / math.sqrt(d)))
        w.seed = 9850 + seed
        w.dataset = k
        w.name = f"batch_small{seed}_k{k}_{w.name}"
        out.append(w)
    return out


def random_state(w: Workload, count: int, scale: float, centre: np.ndarray, seed: int):
    """Seeded particle states (theta around `centre`, uniform subsample indices)."""
    g = _gen(31337 + seed, 0)
    theta = centre[None, :] + scale * g.standard_normal((count, w.d))
    u = g.integers(0, w.n, size=(count, w.m), dtype=np.int64).astype(np.int32)
    return np.ascontiguousarray(theta), np.ascontiguousarray(u)
