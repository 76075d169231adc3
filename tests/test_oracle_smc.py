"""Pins of the oracle's tempering, mass matrix, resampling, Markov move and
whole SMC runs (sections 2.1-2.3 and 3.3-3.5, Algorithms 1 and 2).

Independent routes: scipy/numpy re-evaluations of ESS and log-sum-exp, numpy
covariance and Cholesky, a hand-derived resampling example and the offspring
count property, the closed-form leapfrog map of a quadratic target, the
closed-form posterior and (tempered) evidence of conjugate linear regression,
and brute-force quadrature for a two-parameter logistic regression.
"""
import math
import os

import numpy as np
import pytest
from scipy.special import logsumexp

import oracle
from paper_1805_03317_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U64 = (1 << 64) - 1


def np_ess(logw, lhat, sig2, a, a_prev):
    nu = (a - a_prev) * (lhat - 0.5 * (a + a_prev) * sig2)
    lw = logw + nu
    return math.exp(2 * logsumexp(lw) - logsumexp(2 * lw))


# ---------------------------------------------------------------------------
# tempering (ESS bisection), reweighting and the evidence increment
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_temper_bisection_hits_target(seed):
    g = np.random.default_rng(seed)
    M = 512
    lhat = -1000 + 40 * g.standard_normal(M)
    sig2 = np.abs(2 * g.standard_normal(M))
    logw = np.full(M, -math.log(M))
    a_prev = 0.2
    a, dz, ess, lw = oracle.temper(lhat, sig2, logw, a_prev, 0.5)
    assert a_prev < a < 1
    e_np = np_ess(logw, lhat, sig2, a, a_prev)
    assert 1 <= e_np <= M
    assert abs(e_np - ess) < 1e-9 * M
    assert abs(e_np - 0.5 * M) < 1e-6 * M
    assert np_ess(logw, lhat, sig2, a + 1e-9, a_prev) < 0.5 * M + 1e-6 * M
    # brute-force scan for the first crossing
    grid = np.linspace(a_prev, 1, 4001)
    ess_grid = np.array([np_ess(logw, lhat, sig2, x, a_prev) for x in grid])
    k = int(np.argmax(ess_grid < 0.5 * M))
    assert grid[k - 1] <= a <= grid[k]
    nu = (a - a_prev) * (lhat - 0.5 * (a + a_prev) * sig2)
    assert abs(dz - (logsumexp(logw + nu) - logsumexp(logw))) < 1e-10
    np.testing.assert_allclose(lw, logw + nu - logsumexp(logw + nu), atol=1e-10)
    assert abs(logsumexp(lw)) < 1e-12


def test_temper_jump_to_one_is_importance_sampling():
    """When ESS(1) meets the target, a = 1 and dlogZ = log mean_i exp(lambda_1,i)."""
    g = np.random.default_rng(5)
    M = 256
    lhat = -50 + 0.3 * g.standard_normal(M)
    sig2 = 0.1 * np.abs(g.standard_normal(M))
    logw = np.full(M, -math.log(M))
    a, dz, ess, lw = oracle.temper(lhat, sig2, logw, 0.0, 0.5)
    assert a == 1.0
    lam = lhat - 0.5 * sig2
    assert abs(dz - (logsumexp(lam) - math.log(M))) < 1e-11
    assert abs(ess - np_ess(logw, lhat, sig2, 1.0, 0.0)) < 1e-9 * M


def test_temper_nonfinite_particle_gets_zero_weight():
    M = 64
    lhat = np.linspace(-10, -9, M)
    lhat[3] = -np.inf
    sig2 = np.zeros(M)
    logw = np.full(M, -math.log(M))
    a, dz, ess, lw = oracle.temper(lhat, sig2, logw, 0.5, 0.5)
    assert lw[3] == -np.inf
    assert np.all(np.isfinite(np.delete(lw, 3)))


# ---------------------------------------------------------------------------
# mass matrix
# ---------------------------------------------------------------------------

def test_moments_vs_numpy():
    g = np.random.default_rng(11)
    M, d = 300, 5
    theta = g.standard_normal((M, d)) @ g.standard_normal((d, d)) + 3
    logw = g.standard_normal(M)
    logw -= logsumexp(logw)
    mean, S, L = oracle.moments(theta, logw)
    Wt = np.exp(logw)
    np.testing.assert_allclose(mean, np.average(theta, axis=0, weights=Wt), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(S, np.cov(theta.T, aweights=Wt, bias=True), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(L, np.linalg.cholesky(S), rtol=1e-12, atol=1e-13)


def test_moments_singular_cloud_gets_jitter():
    M, d = 50, 3
    theta = np.zeros((M, d))
    theta[:, 0] = np.linspace(0, 1, M)
    theta[:, 1] = 2 * theta[:, 0]
    logw = np.full(M, -math.log(M))
    mean, S, L = oracle.moments(theta, logw)
    np.testing.assert_allclose(L @ L.T, S, atol=1e-12)
    assert np.all(np.diag(L) > 0)


# ---------------------------------------------------------------------------
# systematic resampling
# ---------------------------------------------------------------------------

def test_resampling_worked_example():
    with open(os.path.join(GOLD, "systematic_resampling.txt")) as f:
        kv = {ln.split()[0]: ln.split()[1:] for ln in f if ln.strip() and not ln.startswith("#")}
    Wt = np.array([float(x) for x in kv["weights"]])
    anc = oracle.resample_ancestors(np.log(Wt), int(kv["u32"][0]))
    np.testing.assert_array_equal(anc, [int(x) for x in kv["ancestors"]])


@pytest.mark.parametrize("seed", range(5))
def test_resampling_offspring_counts(seed):
    g = np.random.default_rng(seed)
    M = 1000
    logw = 3 * g.standard_normal(M)
    logw -= logsumexp(logw)
    U32 = int(g.integers(0, 2**32))
    anc = oracle.resample_ancestors(logw, U32)
    assert np.all(np.diff(anc) >= 0)
    N = np.bincount(anc, minlength=M)
    MW = M * np.exp(logw)
    assert np.all((N >= np.floor(MW) - 1e-9) & (N <= np.ceil(MW) + 1e-9))
    # float systematic resampling gives the same ancestors away from boundaries
    cw = np.cumsum(np.exp(logw))
    pts = (np.arange(M) + U32 / 2**32) / M * cw[-1]
    ref = np.searchsorted(cw, pts, side="right")
    safe = np.min(np.abs(pts[:, None] - cw[None, :]), axis=1) > 1e-9
    np.testing.assert_array_equal(anc[safe], ref[safe])


def test_resample_offset_is_top_bits_of_stream_word():
    seed, stage = 2002, 9
    c = [(2 << 56) | (stage << 32), 0, 0, 0]
    c0 = list(c)
    c0[0] -= 1
    bg = np.random.Philox(counter=np.array(c0, dtype=np.uint64), key=np.array([seed, 0], dtype=np.uint64))
    assert oracle.resample_offset(seed, stage) == int(bg.random_raw(4)[0]) >> 32


# ---------------------------------------------------------------------------
# Markov move on the conjugate Gaussian family
# ---------------------------------------------------------------------------

def conj_posterior(w, a):
    """Tempered posterior N(mu_a, P_a^{-1}) of linear regression with known noise variance."""
    P = a * (w.X.T @ w.X) / w.gauss_s2 + w.prior_prec
    b = a * (w.X.T @ w.y) / w.gauss_s2 + w.prior_prec @ w.prior_mean
    return np.linalg.solve(P, b), P


def conj_logz(w, a):
    """log Z(a) = log of the integral of p(y|theta)^a p(theta)."""
    if a == 0:
        return 0.0
    n = w.n
    S = (w.gauss_s2 / a) * np.eye(n) + w.X @ np.linalg.solve(w.prior_prec, w.X.T)
    r = w.y - w.X @ w.prior_mean
    sign, logdet = np.linalg.slogdet(S)
    lognorm = -0.5 * (n * math.log(2 * math.pi) + logdet + r @ np.linalg.solve(S, r))
    return 0.5 * n * (1 - a) * math.log(2 * math.pi * w.gauss_s2) - 0.5 * n * math.log(a) + lognorm


def numpy_normals(seed, purpose, stage, move, particle, d):
    out = []
    for k in range(d):
        base = 2 * (k // 2)
        words = []
        for j in (base, base + 1):
            c = [(purpose << 56) | (stage << 32) | (move << 16), particle, j >> 2, 0]
            c0 = list(c)
            i = 0
            while True:
                if c0[i] > 0:
                    c0[i] -= 1
                    break
                c0[i] = U64
                i += 1
            bg = np.random.Philox(counter=np.array(c0, dtype=np.uint64), key=np.array([seed, 0], dtype=np.uint64))
            words.append(int(bg.random_raw(4)[j & 3]))
        u1 = ((words[0] >> 11) + 1) * 2.0 ** -53
        u2 = (words[1] >> 11) * 2.0 ** -53
        r = math.sqrt(-2 * math.log(u1))
        out.append(r * (math.sin(2 * math.pi * u2) if k & 1 else math.cos(2 * math.pi * u2)))
    return np.array(out)


def test_hmc_matches_closed_form_leapfrog_map():
    """Quadratic target: L leapfrog steps are the linear map T^L; check every particle's outcome."""
    w = W.gaussian_small(120, 3, seed=3, s2=0.8, m=30, G=3)
    Pb = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec, gauss_s2=w.gauss_s2)
    Pb.set_cv_centre(w.theta_true)
    a, eps, L = 0.7, 1.7, 6
    mu, Pa = conj_posterior(w, a)
    Sig = np.linalg.inv(Pa) * 1.3
    Lc = np.linalg.cholesky(Sig)
    th0, u0 = W.random_state(w, 24, 0.15, mu, seed=4)
    seed, stage, mv = w.seed, 3, 2
    th1, u1, acc, lhat, sig2 = oracle.move(Pb, th0, u0, a, eps, L, seed, stage, mv, w.G, Sig, Lc)
    assert np.all(acc[:, 0] == 1)           # d_k = 0: every block refresh is accepted
    d = w.d
    Tstep = np.block([[np.eye(d), np.zeros((d, d))], [-0.5 * eps * Pa, np.eye(d)]])
    Tdrift = np.block([[np.eye(d), eps * Sig], [np.zeros((d, d)), np.eye(d)]])
    Tmap = np.linalg.matrix_power(Tstep @ Tdrift @ Tstep, L)
    checked = 0
    for i in range(len(th0)):
        z = numpy_normals(seed, 6, stage, mv, i, d)
        p0 = np.linalg.solve(Lc.T, z)
        s = Tmap @ np.concatenate([th0[i] - mu, p0])
        thL, pL = s[:d] + mu, s[d:]
        U = lambda t: 0.5 * (t - mu) @ Pa @ (t - mu)
        H0 = U(th0[i]) + 0.5 * p0 @ Sig @ p0
        H1 = U(thL) + 0.5 * pL @ Sig @ pL
        c = [(7 << 56) | (stage << 32) | (mv << 16), i, 0, 0]
        c0 = list(c)
        c0[0] -= 1
        bg = np.random.Philox(counter=np.array(c0, dtype=np.uint64), key=np.array([seed, 0], dtype=np.uint64))
        logU = math.log(((int(bg.random_raw(4)[0]) >> 11) + 1) * 2.0 ** -53)
        if abs(logU - (H0 - H1)) < 1e-8:
            continue
        want_acc = logU < H0 - H1
        assert acc[i, 1] == want_acc
        np.testing.assert_allclose(th1[i], thL if want_acc else th0[i], rtol=0, atol=1e-11)
        checked += 1
    assert checked >= 20
    assert 0 < acc[:, 1].sum() < len(th0)


def test_move_leaves_conjugate_posterior_invariant():
    w = W.gaussian_small(200, 2, seed=5, s2=1.0, m=40, G=4)
    Pb = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec, gauss_s2=w.gauss_s2)
    Pb.set_cv_centre(w.theta_true)
    mu, Pa = conj_posterior(w, 1.0)
    Sig = np.linalg.inv(Pa)
    Lc = np.linalg.cholesky(Sig)
    g = np.random.default_rng(3)
    M = 3000
    th = mu + g.standard_normal((M, w.d)) @ Lc.T
    u = g.integers(0, w.n, (M, w.m)).astype(np.int32)
    for r in range(3):
        th, u, acc, _, _ = oracle.move(Pb, th, u, 1.0, 0.3, 5, w.seed, 1, r, w.G, Sig, Lc)
        assert acc[:, 1].mean() > 0.8
    sd = np.sqrt(np.diag(Sig))
    assert np.all(np.abs(th.mean(0) - mu) < 4 * sd / math.sqrt(M))
    np.testing.assert_allclose(np.cov(th.T), Sig, rtol=0.1, atol=0.1 * sd.max() ** 2)


# ---------------------------------------------------------------------------
# whole Subsampling SMC runs (Algorithm 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("recentre", [False, True], ids=["fixed_centre", "per_stage_centre"])
def test_smc_conjugate_gaussian_evidence_and_posterior(recentre):
    w = W.gaussian_small(150, 2, seed=7, s2=1.0, m=40, G=4, L=6)
    Pb = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec, gauss_s2=w.gauss_s2)
    mode, _ = Pb.newton_mode()
    Pb.set_cv_centre(mode)
    truth = conj_logz(w, 1.0)
    runs = []
    for s in range(6):
        temps = []
        res = oracle.run_smc(Pb, M=256, m=w.m, G=w.G, seed=100 + s, eps_fn=lambda st, a, d: 1.0 / 6, L=6, R=2,
                             recentre=recentre)
        runs.append(res)
    lz = np.array([r["logz"] for r in runs])
    se = lz.std(ddof=1) / math.sqrt(len(lz))
    assert abs(lz.mean() - truth) < 4 * se + 0.05, (lz, truth)
    # per-stage increments match the closed-form tempered evidence ratios on average
    r0 = runs[0]
    prev = 0.0
    incs = []
    for a, dz in zip(r0["temps"], r0["dlogz"]):
        incs.append(dz - (conj_logz(w, a) - conj_logz(w, prev)))
        prev = a
    assert abs(np.sum(incs)) < 0.5
    mu, Pa = conj_posterior(w, 1.0)
    th = np.concatenate([r["theta"] for r in runs])
    Sig = np.linalg.inv(Pa)
    sd = np.sqrt(np.diag(Sig))
    assert np.all(np.abs(th.mean(0) - mu) < 0.1 * sd)
    np.testing.assert_allclose(np.cov(th.T), Sig, rtol=0.15, atol=0.15 * sd.max() ** 2)
    assert all(np.all(np.diff(r["temps"]) > 0) and r["temps"][-1] == 1.0 for r in runs)


def quadrature_logistic(w, half_width=9.0, k=401):
    """log p(y) and posterior mean by a tensor grid around the mode (d = 2)."""
    Pb = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec)
    mode, _ = Pb.newton_mode()
    A, B, Cm = Pb.cv_build(mode)
    cov = np.linalg.inv(-Cm + w.prior_prec)
    sd = np.sqrt(np.diag(cov))
    g0 = np.linspace(mode[0] - half_width * sd[0], mode[0] + half_width * sd[0], k)
    g1 = np.linspace(mode[1] - half_width * sd[1], mode[1] + half_width * sd[1], k)
    T0, T1 = np.meshgrid(g0, g1, indexing="ij")
    th = np.stack([T0.ravel(), T1.ravel()], 1)
    eta = th @ w.X.T
    ll = np.sum(w.y[None] * eta - np.logaddexp(0, eta), axis=1)
    dlt = th - w.prior_mean
    lp = -0.5 * np.einsum("ij,jk,ik->i", dlt, w.prior_prec, dlt) - math.log(2 * math.pi) \
        + 0.5 * np.linalg.slogdet(w.prior_prec)[1]
    f = ll + lp
    logz = logsumexp(f) + math.log((g0[1] - g0[0]) * (g1[1] - g1[0]))
    wts = np.exp(f - logsumexp(f))
    return logz, wts @ th, mode


@pytest.mark.parametrize("recentre", [False, True], ids=["fixed_centre", "per_stage_centre"])
def test_smc_logistic_two_parameters_vs_quadrature(recentre):
    w = W.logistic_small(600, 2, seed=11, m=80, G=4, L=6)
    truth, post_mean, mode = quadrature_logistic(w)
    Pb = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec)
    Pb.set_cv_centre(mode)
    lz, means = [], []
    for s in range(5):
        if recentre:
            Pb.set_cv_centre(w.prior_mean)   # the centre then follows the particles (Algorithm 2 step d)
        res = oracle.run_smc(Pb, M=192, m=w.m, G=w.G, seed=300 + s, eps_fn=lambda st, a, d: 1.0 / 6, L=6, R=2,
                             recentre=recentre)
        lz.append(res["logz"])
        means.append(res["theta"].mean(0))
    lz = np.array(lz)
    se = lz.std(ddof=1) / math.sqrt(len(lz))
    assert abs(lz.mean() - truth) < 4 * se + 0.1, (lz, truth)
    np.testing.assert_allclose(np.mean(means, 0), post_mean, atol=0.05)
