"""Pins of the oracle's paper-faithful wrappers: multinomial resampling
(section 2.1) and grid-search tempering with ESS_target = 0.8 M (section 2.2).

Independent routes: a hand-derived inverse-CDF example, numpy's searchsorted
on the floating-point cumulative weights, numpy's own Philox stream for the
words, the offspring-count distribution over many stages, and numpy
re-evaluations of the ESS on the grid.
"""
import math

import numpy as np
import pytest
from scipy.special import logsumexp

import oracle

U64 = 1 << 64


def np_ess(logw, lhat, sig2, a, a_prev):
    nu = (a - a_prev) * (lhat - 0.5 * (a + a_prev) * sig2)
    lw = logw + nu
    return math.exp(2 * logsumexp(lw) - logsumexp(2 * lw))


def words_of(U):
    return np.array([int(u * U64) for u in U], dtype=np.uint64)


# ---------------------------------------------------------------------------
# multinomial resampling
# ---------------------------------------------------------------------------

def test_multinomial_worked_example():
    # W = (0.1, 0.2, 0.3, 0.4): cumulative (0.1, 0.3, 0.6, 1.0); slot k takes the
    # first particle whose cumulative weight exceeds its uniform
    lw = np.log([0.1, 0.2, 0.3, 0.4])
    np.testing.assert_array_equal(oracle.resample_multinomial_words(lw, words_of([0.05, 0.15, 0.35, 0.95])),
                                  [0, 1, 2, 3])
    np.testing.assert_array_equal(oracle.resample_multinomial_words(lw, words_of([0.99, 0.62, 0.29, 0.0])),
                                  [3, 3, 1, 0])
    np.testing.assert_array_equal(oracle.resample_multinomial_words(lw, words_of([0.31, 0.31, 0.59, 0.61])),
                                  [2, 2, 2, 3])


@pytest.mark.parametrize("seed", range(3))
def test_multinomial_is_inverse_cdf(seed):
    g = np.random.default_rng(seed)
    M = 1000
    logw = 2.5 * g.standard_normal(M)
    words = g.integers(0, 2**63, size=M, dtype=np.uint64) * np.uint64(2) + g.integers(0, 2, size=M, dtype=np.uint64)
    anc = oracle.resample_multinomial_words(logw, words)
    w = np.exp(logw - logw.max())
    cw = np.cumsum(w)
    U = words.astype(np.float64) / 2.0**64 * cw[-1]
    ref = np.searchsorted(cw, U, side="right")
    safe = np.min(np.abs(U[:, None] - cw[None, :]), axis=1) > 1e-9 * cw[-1]
    assert safe.mean() > 0.99
    np.testing.assert_array_equal(anc[safe], ref[safe])


def test_multinomial_words_are_stream_words():
    seed, stage, M = 2002, 7, 12
    lw = np.zeros(M)                                  # equal weights: ancestor = floor(M * word / 2^64)
    anc = oracle.resample_multinomial(lw, seed, stage)
    for k in range(M):
        c = np.array([(2 << 56) | (stage << 32), k, 0, 0], dtype=np.uint64)
        c[0] -= np.uint64(1)                          # numpy increments the counter before use
        bg = np.random.Philox(counter=c, key=np.array([seed, 0], dtype=np.uint64))
        word = int(bg.random_raw(4)[1])
        assert anc[k] == (word * M) >> 64


def test_multinomial_offspring_distribution():
    g = np.random.default_rng(11)
    M = 64
    logw = 1.5 * g.standard_normal(M)
    W = np.exp(logw - logsumexp(logw))
    R = 600
    N = np.zeros((R, M))
    for r in range(R):
        N[r] = np.bincount(oracle.resample_multinomial(logw, 99, r), minlength=M)
    # each count is Binomial(M, W_i): mean M W_i, variance M W_i (1 - W_i)
    se = np.sqrt(M * W * (1 - W) / R)
    z = (N.mean(0) - M * W) / se
    assert np.abs(z).max() < 4.5
    assert abs(np.mean(z**2) - 1) < 0.35
    v = N.var(0, ddof=1)
    np.testing.assert_allclose(v[W > 0.02], (M * W * (1 - W))[W > 0.02], rtol=0.35)


# ---------------------------------------------------------------------------
# grid-search tempering
# ---------------------------------------------------------------------------

def test_grid_points():
    for a_prev in (0.0, 0.25, 0.9375, 1 - 2**-20):
        assert oracle.grid_point(a_prev, 0) == 1.0
        prev = 1.0
        for j in range(1, 129):
            a = oracle.grid_point(a_prev, j)
            exact = a_prev + (1 - a_prev) * 2.0 ** (-j / 4)
            assert abs(a - exact) <= 2 * math.ulp(max(a, 1e-300)) + 1e-300
            assert a_prev <= a <= prev
            prev = a


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_grid_temper_picks_the_closest_ess(seed):
    g = np.random.default_rng(seed)
    M = 512
    lhat = -1000 + 40 * g.standard_normal(M)
    sig2 = np.abs(2 * g.standard_normal(M))
    logw = -math.log(M) + 0.3 * g.standard_normal(M)
    logw -= logsumexp(logw)
    a_prev, S = 0.2, 129
    a, dz, ess, lw, grid = oracle.temper_grid(lhat, sig2, logw, a_prev, 0.8, S)
    pts = [oracle.grid_point(a_prev, j) for j in range(S)]
    e_np = np.array([np_ess(logw, lhat, sig2, x, a_prev) for x in pts])
    np.testing.assert_allclose(grid, e_np, rtol=1e-10)
    j = int(np.argmin(np.abs(e_np - 0.8 * M)))
    assert a == pts[j]
    assert abs(ess - e_np[j]) < 1e-8 * M
    nu = (a - a_prev) * (lhat - 0.5 * (a + a_prev) * sig2)
    assert abs(dz - (logsumexp(logw + nu) - logsumexp(logw))) < 1e-10
    np.testing.assert_allclose(lw, logw + nu - logsumexp(logw + nu), atol=1e-10)


def test_grid_temper_always_moves():
    # ESS already below the target at every grid point: the closest is the
    # smallest step; a grid point equal to a_prev (a step below half an ulp)
    # is never taken
    g = np.random.default_rng(5)
    M = 256
    lhat = 1e6 * g.standard_normal(M)
    sig2 = np.zeros(M)
    logw = np.full(M, -math.log(M))
    a_prev = 1 - 2**-40
    a, dz, ess, lw, grid = oracle.temper_grid(lhat, sig2, logw, a_prev, 0.8, 129)
    assert a > a_prev
    pts = np.array([oracle.grid_point(a_prev, j) for j in range(129)])
    movers = np.flatnonzero(pts > a_prev)
    assert len(movers) < 129                          # some steps round to a_prev here
    e_np = np.array([np_ess(logw, lhat, sig2, x, a_prev) for x in pts[movers]])
    assert a == pts[movers[int(np.argmin(np.abs(e_np - 0.8 * M)))]]


def test_grid_temper_takes_one_when_every_point_meets_the_target():
    M = 256
    lhat = np.full(M, -10.0) + 1e-6 * np.arange(M)
    sig2 = np.zeros(M)
    logw = np.full(M, -math.log(M))
    a, dz, ess, lw, grid = oracle.temper_grid(lhat, sig2, logw, 0.5, 0.8, 129)
    assert a == 1.0
    assert np.all(grid >= 0.8 * M)
    assert abs(dz - (logsumexp(logw + 0.5 * lhat) - logsumexp(logw))) < 1e-12
