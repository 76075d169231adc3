"""ctypes wrapper of the oracle shared library plus a plain SMC driver.

Test infrastructure only. Every function here calls the C oracle
(subsmc_oracle.c) or is a direct loop over its calls, in the order of
Algorithm 2 of the paper.
"""
import ctypes as C
import math

import numpy as np

from .build import ensure_built

LOGISTIC, POISSON, GAUSSIAN = 0, 1, 2

_lib = None


class _Data(C.Structure):
    _fields_ = [
        ("family", C.c_int32), ("cv_order", C.c_int32), ("n", C.c_int64),
        ("d", C.c_int32), ("ld", C.c_int32), ("Xy", C.POINTER(C.c_double)),
        ("gauss_s2", C.c_double),
    ]


class _CV(C.Structure):
    _fields_ = [
        ("theta_bar", C.POINTER(C.c_double)), ("A", C.c_double),
        ("B", C.POINTER(C.c_double)), ("C", C.POINTER(C.c_double)),
    ]


class _MoveCfg(C.Structure):
    _fields_ = [
        ("M", C.c_int32), ("m", C.c_int32), ("G", C.c_int32), ("seed", C.c_uint64),
        ("stage", C.c_uint32), ("dataset", C.c_uint32), ("mu0", C.POINTER(C.c_double)), ("Q0", C.POINTER(C.c_double)),
        ("Sigma", C.POINTER(C.c_double)), ("Lchol", C.POINTER(C.c_double)),
    ]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(ensure_built())
        L.orc_philox4x64_10.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.orc_rng_word.restype = C.c_uint64
        L.orc_rng_word.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64]
        L.orc_normal.restype = C.c_double
        L.orc_normal.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                 C.c_uint64]
        L.orc_remainder.argtypes = [C.POINTER(_Data), C.c_double, C.c_double, C.c_double,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_cv_build.argtypes = [C.POINTER(_Data), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_cholesky.restype = C.c_int
        L.orc_cholesky.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_newton_mode.restype = C.c_int
        L.orc_newton_mode.argtypes = [C.POINTER(_Data), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int)]
        L.orc_estimate.argtypes = [C.POINTER(_Data), C.POINTER(_CV), C.c_int32, C.c_int32,
                                   C.POINTER(C.c_double), C.POINTER(C.c_int32)] + [C.POINTER(C.c_double)] * 5
        L.orc_temper.restype = C.c_int
        L.orc_temper.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_moments.restype = C.c_int
        L.orc_moments.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_resample_ancestors.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_uint32, C.POINTER(C.c_int32)]
        L.orc_resample_offset.restype = C.c_uint32
        L.orc_resample_offset.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_resample_multinomial_words.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_uint64),
                                                     C.POINTER(C.c_int32)]
        L.orc_resample_multinomial.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_uint64, C.c_uint32,
                                               C.c_uint32, C.POINTER(C.c_int32)]
        L.orc_grid_point.restype = C.c_double
        L.orc_grid_point.argtypes = [C.c_double, C.c_int32]
        L.orc_temper_grid.restype = C.c_int
        L.orc_temper_grid.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.c_double, C.c_double, C.c_int32,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.orc_init_particles.restype = C.c_int
        L.orc_init_particles.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_uint64, C.c_uint32,
                                         C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.orc_move.restype = C.c_int
        L.orc_move.argtypes = [C.POINTER(_Data), C.POINTER(_CV), C.POINTER(_MoveCfg), C.c_double, C.c_double,
                               C.c_int32, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_move_range.restype = C.c_int
        L.orc_move_range.argtypes = [C.POINTER(_Data), C.POINTER(_CV), C.POINTER(_MoveCfg), C.c_double,
                                     C.c_double, C.c_int32, C.c_uint32, C.c_int32, C.c_int32,
                                     C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------

def philox4x64_10(ctr, key):
    c = (C.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def rng_word(seed, purpose, stage, move, dataset, particle, draw):
    return int(lib().orc_rng_word(seed, purpose, stage, move, dataset, particle, draw))


def normal(seed, purpose, stage, move, particle, k, dataset=0):
    return float(lib().orc_normal(seed, purpose, stage, move, dataset, particle, k))


# ---------------------------------------------------------------------------
# problem description
# ---------------------------------------------------------------------------

class Problem:
    """A dataset (rows of Xy = [x_k, y_k, padding]) with its prior and CV centre."""

    def __init__(self, Xy, d, family, prior_mean, prior_prec, cv_order=2, gauss_s2=1.0):
        self.Xy = np.ascontiguousarray(Xy, dtype=np.float64)
        self.n, self.ld = self.Xy.shape
        self.d = int(d)
        assert self.ld >= self.d + 1
        self.family = int(family)
        self.cv_order = int(cv_order)
        self.gauss_s2 = float(gauss_s2)
        self.mu0 = np.ascontiguousarray(prior_mean, dtype=np.float64)
        self.Q0 = np.ascontiguousarray(prior_prec, dtype=np.float64)
        self._data = _Data(self.family, self.cv_order, self.n, self.d, self.ld, _dp(self.Xy), self.gauss_s2)
        self.theta_bar = None

    # control variates ----------------------------------------------------
    def cv_build(self, theta_bar):
        tb = np.ascontiguousarray(theta_bar, dtype=np.float64)
        A = C.c_double()
        B = np.zeros(self.d)
        Cm = np.zeros((self.d, self.d))
        lib().orc_cv_build(C.byref(self._data), _dp(tb), C.byref(A), _dp(B), _dp(Cm))
        return float(A.value), B, Cm

    def newton_mode(self, max_iter=100):
        th = np.zeros(self.d)
        it = C.c_int()
        st = lib().orc_newton_mode(C.byref(self._data), _dp(self.mu0), _dp(self.Q0), _dp(th), max_iter, C.byref(it))
        if st != 0:
            raise RuntimeError(f"oracle newton failed: {st}")
        return th, it.value

    def set_cv_centre(self, theta_bar):
        self.theta_bar = np.ascontiguousarray(theta_bar, dtype=np.float64)
        self.A, self.B, self.C = self.cv_build(self.theta_bar)
        self._cv = _CV(_dp(self.theta_bar), self.A, _dp(self.B), _dp(self.C))

    def set_cv(self, theta_bar, A, B, Cm):
        """Control-variate centre and summaries given directly (timing runs that build them from a
        row subset; results then are not those of the full-data control variate)."""
        self.theta_bar = np.ascontiguousarray(theta_bar, dtype=np.float64)
        self.A = float(A)
        self.B = np.ascontiguousarray(B, dtype=np.float64)
        self.C = np.ascontiguousarray(Cm, dtype=np.float64)
        self._cv = _CV(_dp(self.theta_bar), self.A, _dp(self.B), _dp(self.C))

    # per-observation remainder --------------------------------------------
    def remainder(self, y, eta_bar, Delta):
        d = C.c_double()
        dp = C.c_double()
        lib().orc_remainder(C.byref(self._data), float(y), float(eta_bar), float(Delta), C.byref(d), C.byref(dp))
        return d.value, dp.value

    # estimator ------------------------------------------------------------
    def estimate(self, theta, u, grad=False):
        theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, self.d)
        u = np.ascontiguousarray(u, dtype=np.int32).reshape(theta.shape[0], -1)
        cnt, m = u.shape
        lhat = np.zeros(cnt)
        sig2 = np.zeros(cnt)
        dhat = np.zeros(cnt)
        gl = np.zeros((cnt, self.d)) if grad else None
        gs = np.zeros((cnt, self.d)) if grad else None
        null = C.POINTER(C.c_double)()
        lib().orc_estimate(C.byref(self._data), C.byref(self._cv), cnt, m, _dp(theta), _ip(u),
                           _dp(lhat), _dp(sig2), _dp(dhat), _dp(gl) if grad else null, _dp(gs) if grad else null)
        out = {"lhat": lhat, "sig2": sig2, "dhat": dhat}
        if grad:
            out["grad_l"] = gl
            out["grad_s"] = gs
        return out


def cholesky(S):
    S = np.ascontiguousarray(S, dtype=np.float64)
    d = S.shape[0]
    L = np.zeros_like(S)
    st = lib().orc_cholesky(d, _dp(S), _dp(L))
    if st != 0:
        raise np.linalg.LinAlgError("not positive definite")
    return L


def temper(lhat, sig2, logw, a_prev, ess_frac=0.5, n_bisect=60):
    lhat = np.ascontiguousarray(lhat, dtype=np.float64)
    sig2 = np.ascontiguousarray(sig2, dtype=np.float64)
    lw = np.array(logw, dtype=np.float64)
    a = C.c_double()
    dz = C.c_double()
    ess = C.c_double()
    st = lib().orc_temper(len(lw), _dp(lhat), _dp(sig2), _dp(lw), float(a_prev), float(ess_frac), int(n_bisect),
                          C.byref(a), C.byref(dz), C.byref(ess))
    if st != 0:
        raise FloatingPointError("all incremental weights non-finite")
    return a.value, dz.value, ess.value, lw


def moments(theta, logw):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    logw = np.ascontiguousarray(logw, dtype=np.float64)
    M, d = theta.shape
    mean = np.zeros(d)
    S = np.zeros((d, d))
    L = np.zeros((d, d))
    st = lib().orc_moments(M, d, _dp(theta), _dp(logw), _dp(mean), _dp(S), _dp(L))
    if st != 0:
        raise np.linalg.LinAlgError("particle covariance not positive definite")
    return mean, S, L


def resample_ancestors(logw, U32):
    logw = np.ascontiguousarray(logw, dtype=np.float64)
    anc = np.zeros(len(logw), dtype=np.int32)
    lib().orc_resample_ancestors(len(logw), _dp(logw), int(U32), _ip(anc))
    return anc


def resample_offset(seed, stage, dataset=0):
    return int(lib().orc_resample_offset(seed, stage, dataset))


def resample_multinomial(logw, seed, stage, dataset=0):
    """Multinomial resampling (section 2.1) with the stage's Philox words."""
    logw = np.ascontiguousarray(logw, dtype=np.float64)
    anc = np.zeros(len(logw), dtype=np.int32)
    lib().orc_resample_multinomial(len(logw), _dp(logw), int(seed), int(stage), int(dataset), _ip(anc))
    return anc


def resample_multinomial_words(logw, words):
    """Multinomial resampling with given 64-bit uniform words (one per slot)."""
    logw = np.ascontiguousarray(logw, dtype=np.float64)
    words = np.ascontiguousarray(words, dtype=np.uint64)
    anc = np.zeros(len(logw), dtype=np.int32)
    lib().orc_resample_multinomial_words(len(logw), _dp(logw), words.ctypes.data_as(C.POINTER(C.c_uint64)),
                                          _ip(anc))
    return anc


def grid_point(a_prev, j):
    return float(lib().orc_grid_point(float(a_prev), int(j)))


def temper_grid(lhat, sig2, logw, a_prev, ess_frac=0.8, S=129):
    """The paper's grid rule (section 2.2); returns a, dlogz, ess, new logw, ESS on the grid."""
    lhat = np.ascontiguousarray(lhat, dtype=np.float64)
    sig2 = np.ascontiguousarray(sig2, dtype=np.float64)
    lw = np.array(logw, dtype=np.float64)
    grid = np.zeros(S)
    a = C.c_double()
    dz = C.c_double()
    ess = C.c_double()
    st = lib().orc_temper_grid(len(lw), _dp(lhat), _dp(sig2), _dp(lw), float(a_prev), float(ess_frac), int(S),
                               _dp(grid), C.byref(a), C.byref(dz), C.byref(ess))
    if st != 0:
        raise FloatingPointError(f"oracle grid temper failed: {st}")
    return a.value, dz.value, ess.value, lw, grid


def init_particles(M, d, m, n, seed, mu0, Q0, dataset=0):
    theta = np.zeros((M, d))
    u = np.zeros((M, m), dtype=np.int32)
    logw = np.zeros(M)
    mu0 = np.ascontiguousarray(mu0, dtype=np.float64)
    Q0 = np.ascontiguousarray(Q0, dtype=np.float64)
    st = lib().orc_init_particles(M, d, m, n, seed, dataset, _dp(mu0), _dp(Q0), _dp(theta), _ip(u), _dp(logw))
    if st != 0:
        raise RuntimeError(f"oracle init failed: {st}")
    return theta, u, logw


def move(prob, theta, u, a, eps, L, seed, stage, mv, G, Sigma, Lchol, i0=0, diag=False, dataset=0):
    """One Markov move (Algorithm 1) of particles i0, i0+1, ... held in theta/u (rows).

    With diag=True also returns (count, 4): log r and log U of the u-refresh
    and of the HMC accept step.
    """
    theta = np.array(theta, dtype=np.float64, order="C")
    u = np.array(u, dtype=np.int32, order="C")
    cnt, m = u.shape
    acc = np.zeros((cnt, 2), dtype=np.int32)
    lhat = np.zeros(cnt)
    sig2 = np.zeros(cnt)
    Sigma = np.ascontiguousarray(Sigma, dtype=np.float64)
    Lchol = np.ascontiguousarray(Lchol, dtype=np.float64)
    cfg = _MoveCfg(cnt, m, int(G), int(seed), int(stage), int(dataset), _dp(prob.mu0), _dp(prob.Q0), _dp(Sigma), _dp(Lchol))
    dg = np.zeros((cnt, 4)) if diag else None
    st = lib().orc_move_range(C.byref(prob._data), C.byref(prob._cv), C.byref(cfg), float(a), float(eps),
                              int(L), int(mv), int(i0), cnt, _dp(theta), _ip(u), _ip(acc), _dp(lhat), _dp(sig2),
                              _dp(dg) if diag else C.POINTER(C.c_double)())
    if st != 0:
        raise RuntimeError(f"oracle move failed: {st}")
    if diag:
        return theta, u, acc, lhat, sig2, dg
    return theta, u, acc, lhat, sig2


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Threads of the oracle's loops over particles (timing only; no effect on results)."""
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# Algorithm 2, driven step by step
# ---------------------------------------------------------------------------

def run_smc(prob, M, m, G, seed, eps_fn, L, R, ess_frac=0.5, max_stages=10000, callback=None,
            schemes="default", grid_points=129, recentre=False, dataset=0):
    """Subsampling SMC (Algorithm 2): returns dict with log Z, temperatures, particles.

    schemes="default": ESS bisection and systematic resampling; schemes="paper":
    the paper's grid rule (ess_frac is then the grid target, 0.8 in the paper)
    and multinomial resampling (sections 2.1, 2.2).
    recentre=True: Algorithm 2 step d as written, the control variates are
    rebuilt every stage at the weighted particle mean (after reweighting,
    before resampling) and the estimator is re-evaluated there; prob keeps the
    last centre. dataset: the dataset field of every random-number counter
    (datasets of one batch draw independent streams under one seed)."""
    paper = schemes == "paper"
    theta, u, logw = init_particles(M, prob.d, m, prob.n, seed, prob.mu0, prob.Q0, dataset)
    est = prob.estimate(theta, u)
    lhat, sig2 = est["lhat"], est["sig2"]
    a = 0.0
    logz = 0.0
    temps, dlogzs, esss, accs = [], [], [], []
    stage = 0
    while a < 1.0 and stage < max_stages:
        stage += 1
        if paper:
            a_new, dz, ess, logw, _ = temper_grid(lhat, sig2, logw, a, ess_frac, grid_points)
        else:
            a_new, dz, ess, logw = temper(lhat, sig2, logw, a, ess_frac)
        logz += dz
        mean, Sigma, Lc = moments(theta, logw)
        if recentre:
            prob.set_cv_centre(mean)
            est = prob.estimate(theta, u)
            lhat, sig2 = est["lhat"], est["sig2"]
        if paper:
            anc = resample_multinomial(logw, seed, stage, dataset)
        else:
            anc = resample_ancestors(logw, resample_offset(seed, stage, dataset))
        theta, u, lhat, sig2 = theta[anc], u[anc], lhat[anc], sig2[anc]
        logw = np.full(M, -math.log(M))
        a = a_new
        eps = eps_fn(stage, a, prob.d)
        for r in range(R):
            theta, u, acc, lhat, sig2 = move(prob, theta, u, a, eps, L, seed, stage, r, G, Sigma, Lc,
                                             dataset=dataset)
            accs.append(acc.mean(axis=0))
        temps.append(a)
        dlogzs.append(dz)
        esss.append(ess)
        if callback:
            callback(stage, a, theta, u)
    return {"logz": logz, "temps": np.array(temps), "dlogz": np.array(dlogzs), "ess": np.array(esss),
            "theta": theta, "u": u, "logw": logw, "acc": np.array(accs), "stages": stage}
