"""Pins of the oracle's counter-based generator and its conversions.

Philox words are checked bit for bit against numpy's independent Philox4x64-10
and the published known-answer vectors; conversions against exact integer
arithmetic on numpy-generated words and against distributional properties.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U64 = (1 << 64) - 1


def numpy_block(ctr, key):
    """Philox block at counter `ctr` via numpy (which pre-increments its counter)."""
    c = [int(v) for v in ctr]
    # subtract one with borrow across the 256-bit counter
    i = 0
    while True:
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = U64
        i += 1
        if i == 4:
            break
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array([int(k) for k in key], dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def stream_counter(purpose, stage, move, dataset, particle, draw):
    return [(purpose << 56) | (stage << 32) | (move << 16) | dataset, particle, draw >> 2, 0]


def test_philox_known_answers():
    with open(os.path.join(GOLD, "philox4x64_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        ctr, key, want = v[0:4], v[4:6], v[6:10]
        assert oracle.philox4x64_10(ctr, key) == want
        assert numpy_block(ctr, key) == want


def test_philox_matches_numpy_random_counters():
    g = np.random.default_rng(1)
    for _ in range(200):
        ctr = [int(x) for x in g.integers(0, 2**63, 4, dtype=np.int64)]
        ctr = [c * 2 + int(g.integers(0, 2)) for c in ctr]
        key = [int(x) * 2 + 1 for x in g.integers(0, 2**62, 2, dtype=np.int64)]
        assert oracle.philox4x64_10(ctr, key) == numpy_block(ctr, key)


def test_stream_layout_matches_numpy():
    seed = 2002
    for (purpose, stage, move, particle, draw) in [(0, 0, 0, 0, 0), (1, 0, 0, 7, 13), (4, 17, 3, 2047, 49),
                                                   (6, 255, 65535, 123456, 7), (2, 3, 0, 0, 0)]:
        w = oracle.rng_word(seed, purpose, stage, move, 0, particle, draw)
        blk = numpy_block(stream_counter(purpose, stage, move, 0, particle, draw), [seed, 0])
        assert w == blk[draw & 3]


def test_initial_subsample_indices_are_floor_w_n():
    """u_ij = floor(w * n / 2^64) for the purpose-1 stream, checked with Python integers."""
    M, d, m, n, seed = 3, 2, 37, 1_000_003, 77
    theta, u, logw = oracle.init_particles(M, d, m, n, seed, np.zeros(d), np.eye(d))
    for i in range(M):
        for j in range(m):
            w = numpy_block(stream_counter(1, 0, 0, 0, i, j), [seed, 0])[j & 3]
            assert u[i, j] == (w * n) >> 64
    np.testing.assert_array_equal(logw, -math.log(M))


def test_index_is_uniform():
    n, cnt, seed = 97, 200_000, 5
    theta, u, _ = oracle.init_particles(1, 1, cnt, n, seed, np.zeros(1), np.eye(1))
    counts = np.bincount(u.ravel(), minlength=n)
    assert counts.min() > 0 and u.max() < n
    chi2 = ((counts - cnt / n) ** 2 / (cnt / n)).sum()
    assert stats.chi2.sf(chi2, n - 1) > 1e-4


def test_normals_box_muller_from_numpy_words():
    seed = 99
    for particle in (0, 5):
        for k in range(6):
            base = 2 * (k // 2)
            wa = numpy_block(stream_counter(6, 2, 1, 0, particle, base), [seed, 0])[base & 3]
            wb = numpy_block(stream_counter(6, 2, 1, 0, particle, base + 1), [seed, 0])[(base + 1) & 3]
            u1 = ((wa >> 11) + 1) * 2.0 ** -53
            u2 = (wb >> 11) * 2.0 ** -53
            r = math.sqrt(-2 * math.log(u1))
            want = r * (math.sin(2 * math.pi * u2) if k & 1 else math.cos(2 * math.pi * u2))
            got = oracle.normal(seed, 6, 2, 1, particle, k)
            assert abs(got - want) <= 1e-15 * max(1.0, abs(want))


def test_normals_distribution():
    """Prior draws theta = mu0 + L0^{-T} z have the prior's mean and covariance."""
    d, M = 3, 20000
    mu0 = np.array([1.0, -2.0, 0.5])
    A = np.array([[2.0, 0.3, 0.0], [0.3, 1.0, -0.2], [0.0, -0.2, 0.5]])
    Q0 = np.linalg.inv(A)
    theta, _, _ = oracle.init_particles(M, d, 1, 10, 4242, mu0, Q0)
    assert np.all(np.abs(theta.mean(0) - mu0) < 5 * np.sqrt(np.diag(A) / M))
    cov = np.cov(theta.T)
    assert np.max(np.abs(cov - A)) < 0.06
    z = (theta - mu0) @ np.linalg.cholesky(Q0)  # whitened
    for c in range(d):
        assert stats.kstest(z[:, c], "norm").pvalue > 1e-4


def test_dataset_field_of_every_stream():
    """Batch members draw with their index in the counter's low 16 bits: the
    initial indices and prior normals, the resampling offset and words, and
    the move's block choice follow numpy's words at that counter."""
    M, d, m, n, seed = 4, 3, 9, 5003, 123
    for ds in (0, 1, 63, 65535):
        theta, u, _ = oracle.init_particles(M, d, m, n, seed, np.zeros(d), np.eye(d), dataset=ds)
        for i in range(M):
            for j in range(m):
                w = numpy_block(stream_counter(1, 0, 0, ds, i, j), [seed, 0])[j & 3]
                assert u[i, j] == (w * n) >> 64
        for i in range(M):
            for k in range(d):
                base = 2 * (k // 2)
                wa = numpy_block(stream_counter(0, 0, 0, ds, i, base), [seed, 0])[base & 3]
                wb = numpy_block(stream_counter(0, 0, 0, ds, i, base + 1), [seed, 0])[(base + 1) & 3]
                r = math.sqrt(-2 * math.log(((wa >> 11) + 1) * 2.0 ** -53))
                ang = 2 * math.pi * ((wb >> 11) * 2.0 ** -53)
                want = r * (math.sin(ang) if k & 1 else math.cos(ang))
                assert abs(theta[i, k] - want) <= 1e-14 * max(1.0, abs(want))
                assert oracle.normal(seed, 0, 0, 0, i, k, dataset=ds) == theta[i, k]
        off = numpy_block(stream_counter(2, 7, 0, ds, 0, 0), [seed, 0])[0] >> 32
        assert oracle.resample_offset(seed, 7, ds) == off
        lw = np.zeros(8)                               # equal weights: ancestor = floor(8 word / 2^64)
        anc = oracle.resample_multinomial(lw, seed, 7, ds)
        for k in range(8):
            wk = numpy_block(stream_counter(2, 7, 0, ds, k, 1), [seed, 0])[1]
            assert anc[k] == (wk * 8) >> 64
    a = oracle.init_particles(M, d, m, n, seed, np.zeros(d), np.eye(d), dataset=0)[1]
    b = oracle.init_particles(M, d, m, n, seed, np.zeros(d), np.eye(d), dataset=1)[1]
    assert (a != b).mean() > 0.9


def test_move_draws_use_the_dataset_field():
    """The u-refresh of a move with dataset field 9 replaces block g (purpose 3)
    by the indices of purpose 4, both at that field."""
    from paper_1805_03317_amd import workloads as W
    w = W.logistic_small(1500, 3, seed=91, M=24, m=40, G=4)
    P = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec)
    tb, _ = P.newton_mode()
    P.set_cv_centre(tb)
    ds, stage, mv = 9, 4, 1
    th0, u0, _ = oracle.init_particles(w.M, w.d, w.m, w.n, w.seed, w.prior_mean, w.prior_prec, dataset=ds)
    th0 = tb + 0.05 * (th0 - w.prior_mean)
    _, Sig, Lc = oracle.moments(th0, np.full(w.M, -math.log(w.M)))
    th1, u1, acc, _, _ = oracle.move(P, th0, u0, 0.5, 0.1, 3, w.seed, stage, mv, w.G, Sig, Lc, dataset=ds)
    assert acc[:, 0].sum() > 0
    for i in range(w.M):
        g = (numpy_block(stream_counter(3, stage, mv, ds, i, 0), [w.seed, 0])[0] * w.G) >> 64
        b0, b1 = g * w.m // w.G, (g + 1) * w.m // w.G
        outside = np.r_[0:b0, b1:w.m]
        np.testing.assert_array_equal(u1[i, outside], u0[i, outside])
        if acc[i, 0]:
            fresh = [(numpy_block(stream_counter(4, stage, mv, ds, i, j - b0), [w.seed, 0])[(j - b0) & 3] * w.n) >> 64
                     for j in range(b0, b1)]
            np.testing.assert_array_equal(u1[i, b0:b1], fresh)
        else:
            np.testing.assert_array_equal(u1[i], u0[i])
