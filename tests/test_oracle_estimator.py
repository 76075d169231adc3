"""Pins of the oracle's control variates, difference estimator and gradients.

Each check uses a route independent of the oracle's code: exact enumeration
over every subsample, 50-digit mpmath arithmetic, closed forms of the Gaussian
family, finite differences, float64 autograd of a torch re-expression, and an
independent optimiser.
"""
import itertools
import math

import mpmath as mp
import numpy as np
import pytest
import torch
from scipy import optimize
from scipy.special import gammaln, logsumexp

import oracle
from paper_1805_03317_amd import workloads as W


FAMILIES = [W.LOGISTIC, W.POISSON, W.STUDENT_T]


def small(family):
    return {W.LOGISTIC: W.logistic_small, W.POISSON: W.poisson_small, W.STUDENT_T: W.student_small}[family]


def t5_logpdf(r):
    nu = 5.0
    return gammaln((nu + 1) / 2) - gammaln(nu / 2) - 0.5 * np.log(nu * np.pi) - (nu + 1) / 2 * np.log1p(r * r / nu)


def make_problem(w, theta_bar=None, cv_order=2):
    P = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec, gauss_s2=w.gauss_s2,
                       cv_order=cv_order)
    P.set_cv_centre(w.theta_true if theta_bar is None else theta_bar)
    return P


def full_loglik(w, theta):
    """Full-data log-likelihood from the model definitions (Exp. 1 and Exp. 2; Gaussian test family)."""
    eta = w.X @ theta
    if w.family == W.LOGISTIC:
        return float(np.sum(w.y * eta - np.logaddexp(0.0, eta)))
    if w.family == W.POISSON:
        return float(np.sum(w.y * eta - np.exp(eta) - gammaln(w.y + 1)))
    if w.family == W.STUDENT_T:
        return float(np.sum(t5_logpdf(w.y - eta)))
    r = w.y - eta
    return float(np.sum(-0.5 * np.log(2 * np.pi * w.gauss_s2) - r * r / (2 * w.gauss_s2)))


# ---------------------------------------------------------------------------
# exact enumeration over all u in {1..n}^m (difference estimator, section 3.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cv_order", [2, 1])
@pytest.mark.parametrize("family", FAMILIES)
def test_enumeration_unbiased_and_variance_divisor(family, cv_order):
    """Both control variates: the second-order one of section 3.2 and the
    first-order one of Experiment 4 (q_k without its curvature term)."""
    n, m, d = 5, 3, 2
    w = small(family)(n, d, seed=3)
    P = make_problem(w, theta_bar=w.theta_true + 0.1, cv_order=cv_order)
    theta = w.theta_true + np.array([1.6, -1.3])
    us = np.array(list(itertools.product(range(n), repeat=m)), dtype=np.int32)
    est = P.estimate(np.repeat(theta[None], len(us), 0), us)
    exact = full_loglik(w, theta)
    # E_u[l_hat] = l(theta): pins the n/m scaling, the sum of q_k and every d_k
    assert abs(est["lhat"].mean() - exact) < 1e-12 * max(1, abs(exact))
    # E_u[sigma2_hat] = (m-1)/m Var_u(l_hat): pins the n^2/m^2 divisor
    var = np.mean((est["lhat"] - est["lhat"].mean()) ** 2)
    assert var > 1e-3
    assert abs(est["sig2"].mean() - (m - 1) / m * var) < 1e-12 * var
    # the d-part alone is unbiased for sum_k d_k
    dl = theta - P.theta_bar
    qsum = P.A + P.B @ dl + (0.5 * dl @ P.C @ dl if cv_order == 2 else 0.0)
    assert abs(est["dhat"].mean() - (exact - qsum)) < 1e-11


def test_gaussian_family_estimator_is_exact():
    """Quadratic log-likelihood: d_k = 0, so l_hat = l for every u and sigma2_hat = 0."""
    w = W.gaussian_small(300, 3, seed=1, s2=0.7)
    P = make_problem(w, theta_bar=w.theta_true + np.array([0.2, -0.1, 0.05]))
    th, u = W.random_state(w, 16, 0.5, w.theta_true, seed=2)
    est = P.estimate(th, u)
    for i in range(len(th)):
        exact = full_loglik(w, th[i])
        assert abs(est["lhat"][i] - exact) < 1e-12 * abs(exact)
        assert abs(est["sig2"][i]) < 1e-40
        assert abs(est["dhat"][i]) < 1e-25


# ---------------------------------------------------------------------------
# the per-observation remainder d_k = l_k - q_k against 50-digit arithmetic
# ---------------------------------------------------------------------------

def mp_remainder(family, y, eb, De):
    mp.mp.dps = 60
    y, eb, De = mp.mpf(y), mp.mpf(eb), mp.mpf(De)
    if family == W.LOGISTIC:
        f0 = lambda e: y * e - mp.log(1 + mp.exp(e))
        f1 = lambda e: y - 1 / (1 + mp.exp(-e))
        f2 = lambda e: -mp.exp(-e) / (1 + mp.exp(-e)) ** 2
    elif family == W.POISSON:
        f0 = lambda e: y * e - mp.exp(e) - mp.loggamma(y + 1)
        f1 = lambda e: y - mp.exp(e)
        f2 = lambda e: -mp.exp(e)
    else:
        nu = mp.mpf(5)
        f0 = lambda e: (mp.loggamma((nu + 1) / 2) - mp.loggamma(nu / 2) - mp.log(nu * mp.pi) / 2
                        - (nu + 1) / 2 * mp.log(1 + (y - e) ** 2 / nu))
        f1 = lambda e: (nu + 1) * (y - e) / (nu + (y - e) ** 2)
        f2 = lambda e: (nu + 1) * ((y - e) ** 2 - nu) / (nu + (y - e) ** 2) ** 2
    d = f0(eb + De) - (f0(eb) + f1(eb) * De + f2(eb) * De * De / 2)
    dp = f1(eb + De) - f1(eb) - f2(eb) * De
    return float(d), float(dp)


@pytest.mark.parametrize("family", FAMILIES)
def test_remainder_vs_mpmath(family):
    w = small(family)(10, 2, seed=1)
    P = make_problem(w)
    ebs = {W.LOGISTIC: [-8.0, -2.0, -0.3, 0.0, 0.7, 3.0, 9.0], W.POISSON: [-4.0, -0.5, 0.0, 1.2, 3.0],
           W.STUDENT_T: [-3.0, -0.5, 0.0, 0.4, 2.0]}[family]
    ys = {W.LOGISTIC: [0.0, 1.0], W.POISSON: [0.0, 3.0], W.STUDENT_T: [0.0, 1.9, -7.0]}[family]
    for eb in ebs:
        for y in ys:
            for De in [1e-7, 1e-5, 1e-4, 1e-3, 0.01, 0.1, 0.5, 1.0, 2.0, 5.0]:
                for s in (1.0, -1.0):
                    got_d, got_dp = P.remainder(y, eb, s * De)
                    want_d, want_dp = mp_remainder(family, y, eb, s * De)
                    scale = abs(eb) + 1.0 + (math.exp(eb) if family == W.POISSON else 0.0)
                    assert abs(got_d - want_d) <= 1e-14 * abs(want_d) + 1e-31 * scale, (eb, y, De)
                    assert abs(got_dp - want_dp) <= 1e-14 * abs(want_dp) + 1e-31 * scale, (eb, y, De)


def test_remainder_orders():
    """d_k = O(Delta^3) for the second-order and O(Delta^2) for the first-order control variate."""
    w = W.logistic_small(10, 2, seed=1)
    P2 = make_problem(w)
    P1 = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec, cv_order=1)
    P1.set_cv_centre(w.theta_true)
    eb = 0.4
    r2 = [abs(P2.remainder(1.0, eb, h)[0]) for h in (1e-2, 5e-3)]
    r1 = [abs(P1.remainder(1.0, eb, h)[0]) for h in (1e-2, 5e-3)]
    assert abs(math.log2(r2[0] / r2[1]) - 3) < 0.05
    assert abs(math.log2(r1[0] / r1[1]) - 2) < 0.05


# ---------------------------------------------------------------------------
# control-variate summaries A, B, C
# ---------------------------------------------------------------------------

def test_cv_gaussian_closed_form():
    w = W.gaussian_small(500, 4, seed=2, s2=1.7)
    P = make_problem(w)
    tb = np.array([0.3, -1.0, 0.2, 0.9])
    A, B, Cm = P.cv_build(tb)
    r = w.y - w.X @ tb
    assert abs(A - (-0.5 * r @ r / w.gauss_s2 - 0.5 * w.n * math.log(2 * math.pi * w.gauss_s2))) < 1e-11 * abs(A)
    np.testing.assert_allclose(B, w.X.T @ r / w.gauss_s2, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(Cm, -(w.X.T @ w.X) / w.gauss_s2, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("family", FAMILIES)
def test_cv_logistic_poisson_by_finite_differences(family):
    w = small(family)(800, 3, seed=4)
    P = make_problem(w)
    tb = w.theta_true + np.array([0.1, -0.2, 0.15])
    A, B, Cm = P.cv_build(tb)
    assert abs(A - full_loglik(w, tb)) < 1e-12 * abs(A)
    h = 1e-5
    for c in range(w.d):
        e = np.zeros(w.d)
        e[c] = h
        Ap, Bp, _ = P.cv_build(tb + e)
        Am, Bm, _ = P.cv_build(tb - e)
        assert abs((Ap - Am) / (2 * h) - B[c]) < 1e-6 * (1 + np.abs(B).max())
        np.testing.assert_allclose((Bp - Bm) / (2 * h), Cm[:, c], rtol=0, atol=1e-6 * (1 + np.abs(Cm).max()))
    np.testing.assert_allclose(Cm, Cm.T, rtol=0, atol=1e-12 * np.abs(Cm).max())


@pytest.mark.parametrize("family", FAMILIES)
def test_newton_mode_vs_independent_optimiser(family):
    w = small(family)(1500, 3, seed=5)
    P = make_problem(w)
    mode, iters = P.newton_mode()
    assert iters < 50
    A, B, Cm = P.cv_build(mode)
    grad = B - w.prior_prec @ (mode - w.prior_mean)
    assert np.abs(grad).max() < 1e-8 * (1 + np.abs(B).max())
    assert np.all(np.linalg.eigvalsh(Cm - w.prior_prec) < 0)

    def negpost(t):
        return -(full_loglik(w, t) - 0.5 * (t - w.prior_mean) @ w.prior_prec @ (t - w.prior_mean))

    res = optimize.minimize(negpost, np.zeros(w.d), method="Nelder-Mead",
                            options={"xatol": 1e-10, "fatol": 1e-12, "maxiter": 20000, "maxfev": 40000})
    np.testing.assert_allclose(mode, res.x, atol=1e-6)


# ---------------------------------------------------------------------------
# gradients of l_hat and sigma2_hat
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("family", FAMILIES)
def test_gradients_by_finite_differences(family):
    w = small(family)(2000, 3, seed=6, m=200)
    P = make_problem(w)
    th, u = W.random_state(w, 4, 0.3, w.theta_true, seed=7)
    est = P.estimate(th, u, grad=True)
    h = 1e-6
    for i in range(len(th)):
        fd_l = np.zeros(w.d)
        fd_s = np.zeros(w.d)
        for c in range(w.d):
            e = np.zeros(w.d)
            e[c] = h
            p = P.estimate(th[i] + e, u[i:i + 1])
            q = P.estimate(th[i] - e, u[i:i + 1])
            # difference the d-part separately from the O(n) constant A
            fd_l[c] = ((p["lhat"][0] - P.A) - (q["lhat"][0] - P.A)) / (2 * h)
            fd_s[c] = (p["sig2"][0] - q["sig2"][0]) / (2 * h)
        scale_l = 1 + np.abs(est["grad_l"][i]).max()
        scale_s = 1e-12 + np.abs(est["grad_s"][i]).max()
        np.testing.assert_allclose(est["grad_l"][i], fd_l, rtol=0, atol=1e-6 * scale_l)
        np.testing.assert_allclose(est["grad_s"][i], fd_s, rtol=0, atol=1e-6 * scale_s)


@pytest.mark.parametrize("cv_order", [2, 1])
@pytest.mark.parametrize("family", FAMILIES)
def test_gradients_vs_torch_autograd(family, cv_order):
    """Autograd of a float64 torch re-expression of the estimator's definition."""
    w = small(family)(1000, 4, seed=8, m=150)
    P = make_problem(w, cv_order=cv_order)
    th, u = W.random_state(w, 3, 0.4, w.theta_true, seed=9)
    est = P.estimate(th, u, grad=True)
    X = torch.tensor(w.X)
    y = torch.tensor(w.y)
    tb = torch.tensor(P.theta_bar)

    def f(e):
        if family == W.LOGISTIC:
            return y_s * e - torch.nn.functional.softplus(e)
        if family == W.STUDENT_T:
            r = y_s - e
            return (math.lgamma(3.0) - math.lgamma(2.5) - 0.5 * math.log(5 * math.pi)
                    - 3.0 * torch.log1p(r * r / 5.0))
        return y_s * e - torch.exp(e) - torch.lgamma(y_s + 1)

    for i in range(len(th)):
        t = torch.tensor(th[i], requires_grad=True)
        Xs = X[torch.tensor(u[i], dtype=torch.long)]
        y_s = y[torch.tensor(u[i], dtype=torch.long)]
        eb = (Xs @ tb).detach().requires_grad_(True)
        fb = f(eb)
        (g1,) = torch.autograd.grad(fb.sum(), eb, create_graph=True)
        (g2,) = torch.autograd.grad(g1.sum(), eb)
        De = Xs @ (t - tb)
        c2 = 0.5 if cv_order == 2 else 0.0
        dk = f(Xs @ t) - (fb.detach() + g1.detach() * De + c2 * g2.detach() * De * De)
        n, m = w.n, w.m
        Bq = torch.tensor(P.B)
        Cq = torch.tensor(P.C)
        dl = t - tb
        lhat = P.A + Bq @ dl + c2 * dl @ Cq @ dl + n / m * dk.sum()
        sig2 = n * n / (m * m) * ((dk - dk.mean()) ** 2).sum()
        gl, = torch.autograd.grad(lhat, t, retain_graph=True)
        gs, = torch.autograd.grad(sig2, t)
        assert abs(lhat.item() - est["lhat"][i]) < 1e-10 * abs(est["lhat"][i])
        assert abs(sig2.item() - est["sig2"][i]) < 1e-9 * est["sig2"][i]
        np.testing.assert_allclose(est["grad_l"][i], gl.numpy(), rtol=0, atol=1e-9 * (1 + gl.abs().max().item()))
        np.testing.assert_allclose(est["grad_s"][i], gs.numpy(), rtol=0, atol=1e-9 * gs.abs().max().item())
