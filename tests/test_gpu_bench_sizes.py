"""Parity at the full sizes of the benchmark configurations, on the kernels the benchmark times.

At these sizes (up to n = 5e6 rows, M = 4096 particles, m = 50,000 subsample slots, d = 116)
the oracle cannot redo a stage, so each test

* runs the library as `bench.py` does (mixed path, default kernel choice, live stages from the
  prior, or the fixed a = 1 benchmark state of the configuration table);
* hands the oracle the library's state before one move (teacher forcing: its control-variate
  centre and constants, its mass matrix and factor, and the theta and u of a block of sampled
  particles; the control variates and the mass matrix are themselves parity-tested at smaller
  sizes) and has it move those particles with the same random-number streams (Algorithm 1);
* compares the sampled particles' decisions, u, theta and the cached estimator to the bounds of
  the move-parity tests (decisions exact outside the near-tie band; u bit-exact where the
  decisions agree; theta, l_hat and sigma2_hat within 1e-5 of their scales);
* checks the stage's other steps (exponent search, mass matrix, resampling) on the whole
  population against the oracle from the library's state before each;
* checks the whole population through properties that hold at any size: the refreshed indices
  lie in [0, n) and differ from the old u only inside one of the G blocks (section 3.3); a
  rejected u-refresh leaves u unchanged and a rejected HMC step leaves theta unchanged; theta
  stays finite.
"""
import functools
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1805_03317_amd import workloads as W
from test_gpu_parity import DEV, check_decisions, oracle_move_diag, remainder_scales, say

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=1)
def _workload(name):
    w = getattr(W, name)()
    say("generated", w.name, "n", w.n, "d", w.d, "M", w.M, "m", w.m)
    return w


def _context(w):
    from paper_1805_03317_amd.binding import SubsampledSMC
    Xy = torch.tensor(w.Xy(np.float32), device=DEV)
    smc = SubsampledSMC(Xy, w.d, w.family, W.MIXED, w.M, w.m, w.G, w.prior_mean, w.prior_prec, w.seed,
                        dataset=w.dataset)
    return smc


class _Rows:
    """The library's accept flags and decision record of a block of particles (the interface
    check_decisions reads)."""

    def __init__(self, smc, i0, k):
        self.accept = smc.accept[i0:i0 + k]
        self._diag = smc.move_diag()[i0:i0 + k]

    def move_diag(self):
        return self._diag


def _check_population(w, th0, u0, th1, u1, acc):
    """Properties of one move that hold for every particle at any size."""
    n, m, G = w.n, w.m, w.G
    assert np.isfinite(th1).all()
    assert u1.min() >= 0 and u1.max() < n
    # a rejected HMC step keeps theta; a rejected u-refresh keeps u
    rej_t = acc[:, 1] == 0
    assert np.array_equal(th1[rej_t], th0[rej_t])
    changed = u1 != u0
    rej_u = acc[:, 0] == 0
    assert not changed[rej_u].any()
    # an accepted refresh changes u inside one block [floor(g m / G), floor((g + 1) m / G))
    bounds = (np.arange(G + 1, dtype=np.int64) * m) // G
    rows = np.flatnonzero(changed.any(axis=1))
    first = changed[rows].argmax(axis=1)
    last = m - 1 - changed[rows][:, ::-1].argmax(axis=1)
    g_first = np.searchsorted(bounds, first, side="right") - 1
    g_last = np.searchsorted(bounds, last, side="right") - 1
    assert np.array_equal(g_first, g_last)
    say("population: accept u", acc[:, 0].mean(), "theta", acc[:, 1].mean(), "refreshed", len(rows))


def _check_sampled(w, smc, P, i0, th0, u0, a, eps, stage, mv, Sig, Lc):
    """The sampled particles i0 .. i0 + k - 1 against the oracle's move from the same state."""
    k = len(th0)
    # the oracle's move first alone; its sensitivity to rounding-level perturbations (three more
    # runs) only if a comparison needs it (an ill-conditioned trajectory)
    out = oracle.move(P, th0, u0, a, eps, w.L, w.seed, stage, mv, w.G, Sig, Lc, i0=i0, diag=True,
                      dataset=w.dataset)
    sd, ss = remainder_scales(P, th0, u0)
    scale = 2 * (a * sd + 0.5 * a * a * ss)
    zero = {"dlogr": np.zeros((k, 2)), "dtheta": np.zeros_like(th0), "flip": np.zeros(k, dtype=bool)}
    try:
        _compare(w, smc, P, i0, out, zero, scale, a)
    except AssertionError as e:
        say("comparison needs the oracle's sensitivity:", repr(e)[:200])
        out, sens = oracle_move_diag(P, th0, u0, a, eps, w.L, w.seed, stage, mv, w.G, Sig, Lc, True, i0=i0,
                                     dataset=w.dataset)
        _compare(w, smc, P, i0, out, sens, scale, a)


def _compare(w, smc, P, i0, out, sens, scale, a):
    th1, u1, acc, _, _, dg = out
    k = len(th1)
    rows = _Rows(smc, i0, k)
    same = check_decisions(rows, acc, dg, True, a, scale, sens)
    say("sampled particles", k, "decisions equal", int(same.sum()), "accept", acc.mean(0))
    gu = smc.u[i0:i0 + k].cpu().numpy()
    np.testing.assert_array_equal(gu[same], u1[same])
    gth = smc.theta[i0:i0 + k].cpu().numpy()
    rt = 1e-5
    same2 = same & ~sens["flip"]
    tol_th = rt * np.abs(th1[same2]) + rt * np.abs(th1).max() + 10 * sens["dtheta"][same2]
    err = np.abs(gth[same2] - th1[same2])
    say("theta max error / tol", float((err / tol_th).max()) if err.size else 0.0)
    assert np.all(err <= tol_th)
    # the cached estimator at the particles' final state against the oracle's at that state
    ref = P.estimate(gth[same], gu[same])
    glh = smc.lhat[i0:i0 + k].cpu().numpy()[same]
    gs2 = smc.sig2[i0:i0 + k].cpu().numpy()[same]
    sd, ss = remainder_scales(P, gth[same], gu[same])
    e_l = np.abs(glh - ref["lhat"]) / (np.abs(ref["lhat"]) + sd)
    fl = (1e-12 * np.abs(ref["lhat"])) ** 2
    e_s = np.abs(gs2 - ref["sig2"]) / (ss + fl)
    say("l_hat error / scale", float(e_l.max()), "sigma2_hat error / scale", float(e_s.max()))
    assert np.all(e_l <= 1e-5) and np.all(e_s <= 1e-5)


def _check_stage_steps(w, smc):
    """The stage's steps before its move, each against the oracle from the library's state
    before the step: the exponent search (section 2.1, exponent to 1e-12, log-weights and the
    log-evidence increment to 1e-9), the mass matrix (particle covariance to 1e-10 of its
    largest entry, and its factor) and systematic resampling (ancestors, hence theta, u and the
    caches, bit for bit; weights reset to 1/M)."""
    lh, s2, lw = (x.cpu().numpy() for x in (smc.lhat, smc.sig2, smc.logw))
    a_prev = smc.info()["a"]
    a, dz, ess = smc.temper()
    a_o, dz_o, ess_o, lw_o = oracle.temper(lh, s2, lw, a_prev, w.ess_frac)
    say("temper", a_prev, "->", a, "oracle", a_o, "ess", ess, ess_o)
    assert abs(a - a_o) <= 1e-12 * max(1.0, a_o)
    assert abs(dz - dz_o) <= 1e-9 * max(1.0, abs(dz_o))
    assert abs(ess - ess_o) <= 1e-9 * w.M
    lw1 = smc.logw.cpu().numpy()
    np.testing.assert_allclose(lw1, lw_o, rtol=1e-9, atol=1e-9)
    th = smc.theta.cpu().numpy()
    smc.mass()
    S, Lc, _ = smc.get_mass()
    _, S_o, L_o = oracle.moments(th, lw1)
    np.testing.assert_allclose(S, S_o, rtol=1e-10, atol=1e-10 * np.abs(S_o).max())
    np.testing.assert_allclose(Lc, L_o, rtol=1e-9, atol=1e-9 * np.abs(L_o).max())
    u = smc.u.cpu().numpy()
    lh = smc.lhat.cpu().numpy()
    smc.resample()
    anc = oracle.resample_ancestors(lw1, oracle.resample_offset(w.seed, smc.info()["stage"], w.dataset))
    np.testing.assert_array_equal(smc.theta.cpu().numpy(), th[anc])
    np.testing.assert_array_equal(smc.u.cpu().numpy(), u[anc])
    np.testing.assert_array_equal(smc.lhat.cpu().numpy(), lh[anc])
    np.testing.assert_allclose(smc.logw.cpu().numpy(), -math.log(w.M), rtol=0, atol=1e-15)
    say("resample: distinct ancestors", len(np.unique(anc)))


def _oracle_problem(w, smc):
    tb, A, B, Cm = smc.get_cv()
    P = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec)
    P.set_cv(tb, A, B, Cm)
    return P


def test_benchmark_state_move_at_full_size():
    """The fixed benchmark state of the largest configuration (a = 1, theta from the Laplace
    approximation at the control-variate centre, u uniform, the inverse mass matrix its
    covariance), the state whose move the benchmark reports beside the live stages."""
    w = _workload("config5")
    smc = _context(w)
    eps = 1.0 / w.L
    tb, _, _, Cm = smc.get_cv()
    cov = np.linalg.inv(w.prior_prec - Cm)
    cov = 0.5 * (cov + cov.T)
    g = np.random.Generator(np.random.Philox(key=77))
    th0_all = tb + g.standard_normal((w.M, w.d)) @ np.linalg.cholesky(cov).T
    u0_all = g.integers(0, w.n, size=(w.M, w.m), dtype=np.int64).astype(np.int32)
    smc.theta.copy_(torch.tensor(th0_all, device=DEV))
    smc.u.copy_(torch.tensor(u0_all, device=DEV))
    smc.refresh()
    smc.set_mass(cov)
    Sig, Lc, _ = smc.get_mass()
    stage, mv, a = 4, 0, 1.0
    smc.set_stage(stage, mv, a)
    smc.move(eps, w.L, 1)
    torch.cuda.synchronize()
    _check_population(w, th0_all, u0_all, smc.theta.cpu().numpy(), smc.u.cpu().numpy(),
                      smc.accept.cpu().numpy())
    P = _oracle_problem(w, smc)
    i0, k = 2048, 8
    _check_sampled(w, smc, P, i0, th0_all[i0:i0 + k], u0_all[i0:i0 + k], a, eps, stage, mv, Sig, Lc)
    smc.close()


# (workload, sampled particles, first sampled particle)
LIVE = [("config5", 8, 1365), ("config4", 16, 2730), ("config2", 32, 1000)]


@pytest.mark.parametrize("name,k,i0", LIVE, ids=[c[0] for c in LIVE])
def test_live_stage_move_at_benchmark_size(name, k, i0):
    """The third stage of a run from the prior, as the benchmark's steps run it: two whole
    stages, then the third stage's exponent search, mass matrix and resampling (each checked),
    and its move."""
    w = _workload(name)
    smc = _context(w)
    say("kernel", smc.info())
    eps = 1.0 / w.L
    smc.stage(eps, w.L, 1)
    smc.stage(eps, w.L, 1)
    _check_stage_steps(w, smc)
    info = smc.info()
    a, stage, mv = info["a"], info["stage"], info["move"]
    th0_all = smc.theta.cpu().numpy()
    u0_all = smc.u.cpu().numpy()
    Sig, Lc, _ = smc.get_mass()
    smc.move(eps, w.L, 1)
    torch.cuda.synchronize()
    say("stage", stage, "a", a, "move", mv)
    _check_population(w, th0_all, u0_all, smc.theta.cpu().numpy(), smc.u.cpu().numpy(),
                      smc.accept.cpu().numpy())
    P = _oracle_problem(w, smc)
    _check_sampled(w, smc, P, i0, th0_all[i0:i0 + k], u0_all[i0:i0 + k], a, eps, stage, mv, Sig, Lc)
    smc.close()


def test_batched_persistent_move_at_full_size():
    """The 64-dataset batch as the benchmark runs it (mixed path, one persistent move launch for
    every member's particles, replayed from a HIP graph, eight streams for the per-member
    steps): two whole stages, then the third stage's exponent search, mass matrix and resampling
    checked on every member, and its move checked on every member through the population
    properties and on sampled particles of the largest member of each kernel body (narrow,
    lane-group, resident) against the oracle."""
    from paper_1805_03317_amd.binding import SMCBatch
    count = 64
    ws, members = [], []
    for b in range(count):
        w = W.config3_member(b, count)
        members.append(_context(w))
        ws.append(w)
    batch = SMCBatch(members)
    batch.set_graph(True)
    batch.set_streams(8)
    batch.set_persistent(True)
    eps = np.array([1.0 / w.L for w in ws])
    L = ws[0].L
    for _ in range(2):
        batch.temper()
        batch.mass()
        batch.resample()
        batch.move(eps, L, 1)
    torch.cuda.synchronize()
    # the third stage's steps, each against the oracle on every member
    pre = [(c.lhat.cpu().numpy(), c.sig2.cpu().numpy(), c.logw.cpu().numpy(), c.info()["a"]) for c in members]
    a, dz, ess, act = batch.temper()
    torch.cuda.synchronize()
    for b, (w, c) in enumerate(zip(ws, members)):
        lh, s2, lw, a_prev = pre[b]
        a_o, dz_o, ess_o, lw_o = oracle.temper(lh, s2, lw, a_prev, w.ess_frac)
        assert abs(a[b] - a_o) <= 1e-12 * max(1.0, a_o), b
        assert abs(dz[b] - dz_o) <= 1e-9 * max(1.0, abs(dz_o)), b
        np.testing.assert_allclose(c.logw.cpu().numpy(), lw_o, rtol=1e-9, atol=1e-9)
    lw1 = [c.logw.cpu().numpy() for c in members]
    th = [c.theta.cpu().numpy() for c in members]
    batch.mass()
    torch.cuda.synchronize()
    for b, c in enumerate(members):
        S, Lc, _ = c.get_mass()
        _, S_o, L_o = oracle.moments(th[b], lw1[b])
        np.testing.assert_allclose(S, S_o, rtol=1e-10, atol=1e-10 * np.abs(S_o).max())
    u = [c.u.cpu().numpy() for c in members]
    batch.resample()
    torch.cuda.synchronize()
    for b, (w, c) in enumerate(zip(ws, members)):
        anc = oracle.resample_ancestors(lw1[b], oracle.resample_offset(w.seed, c.info()["stage"], w.dataset))
        np.testing.assert_array_equal(c.theta.cpu().numpy(), th[b][anc])
        np.testing.assert_array_equal(c.u.cpu().numpy(), u[b][anc])
    # the move
    kinds = batch.member_kernels()
    say("member kernel bodies", np.bincount(kinds, minlength=3))
    state = []
    for w, c in zip(ws, members):
        i = c.info()
        Sig, Lc, _ = c.get_mass()
        state.append((c.theta.cpu().numpy(), c.u.cpu().numpy(), i["a"], i["stage"], i["move"], Sig, Lc))
    batch.move(eps, L, 1)
    torch.cuda.synchronize()
    for b, (w, c) in enumerate(zip(ws, members)):
        th0, u0 = state[b][:2]
        _check_population(w, th0, u0, c.theta.cpu().numpy(), c.u.cpu().numpy(), c.accept.cpu().numpy())
    for kind in np.unique(kinds):
        b = max(np.flatnonzero(kinds == kind), key=lambda j: ws[j].m)
        w, c = ws[b], members[b]
        th0, u0, a_b, stage, mv, Sig, Lc = state[b]
        say("member", b, "body", int(kind), "n", w.n, "d", w.d, "m", w.m, "a", a_b)
        P = _oracle_problem(w, c)
        i0, k = 500, 8
        _check_sampled(w, c, P, i0, th0[i0:i0 + k], u0[i0:i0 + k], a_b, eps[b], stage, mv, Sig, Lc)
    batch.close()
    for c in members:
        c.close()
