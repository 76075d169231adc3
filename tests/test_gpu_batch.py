"""GPU parity of the batched entry points (smc_batch_*): many datasets of
uneven n and d advanced together, one launch per step (per kernel shape for
the move).

Each member of a batch must give exactly what its own context gives with the
single-context calls (the same kernels and arguments, so bit for bit), and
what the oracle gives for that dataset with its dataset counter field (within
the full-run tolerances of the single-context tests). Members reach a = 1 at
different stages, so later stages run with part of the batch inactive."""
import math

import numpy as np
import pytest

import oracle
from paper_1805_03317_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def _binding():
    from paper_1805_03317_amd import binding
    return binding


def _oracle_problem(w):
    P = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec)
    tb, _ = P.newton_mode()
    P.set_cv_centre(tb)
    return P, tb


def _context(w, theta_bar, move_path=0):
    B = _binding()
    dt = np.float32 if w.precision == W.MIXED else np.float64
    Xy = torch.tensor(w.Xy(dt), device=DEV)
    return B.SubsampledSMC(Xy, w.d, w.family, w.precision, w.M, w.m, w.G, w.prior_mean, w.prior_prec, w.seed,
                           theta_bar=theta_bar, move_path=move_path, dataset=w.dataset)


def _eps(st, a, d):
    return 0.8 / math.sqrt(d)


def _state(smc):
    torch.cuda.synchronize()
    return (smc.theta.cpu().numpy().copy(), smc.u.cpu().numpy().copy(), smc.logw.cpu().numpy().copy(),
            smc.lhat.cpu().numpy().copy(), smc.sig2.cpu().numpy().copy())


@pytest.mark.parametrize("precision", [W.FP64, W.MIXED], ids=["fp64", "mixed"])
def test_batch_equals_single_context_runs(precision):
    """Full runs: the batch against each member run alone, bit for bit. The
    members span the narrow, lane-group and resident move kernels (one member
    forced onto the streaming path), so the move takes several launches."""
    B = _binding()
    ws = W.batched_small(6, seed=1, precision=precision, d_values=[3, 9, 17, 36, 24, 9])
    paths = [0, 0, B.MOVE_STREAMING, 0, 0, B.MOVE_STREAMING]
    say("batch members", [(w.n, w.d, w.m) for w in ws])
    centres = [_oracle_problem(w)[1] for w in ws]
    singles = []
    for w, tb, mp in zip(ws, centres, paths):
        smc = _context(w, tb, mp)
        logz, rec = smc.run(_eps, L=w.L, R=2)
        singles.append((logz, [r["a"] for r in rec], _state(smc)))
        smc.close()
    members = [_context(w, tb, mp) for w, tb, mp in zip(ws, centres, paths)]
    batch = B.SMCBatch(members)
    launches = []
    logzs, recs = batch.run(_eps, L=ws[0].L, R=2, callback=lambda b, a, act: launches.append(b.launches()))
    say("move launches per stage", launches)
    assert max(launches) >= 3
    stages = [len(r) for r in recs]
    say("stages per member", stages)
    assert len(set(stages)) > 1                        # members finish at different stages
    for k, (w, s) in enumerate(zip(ws, singles)):
        logz1, temps1, st1 = s
        assert [r["a"] for r in recs[k]] == temps1, k
        assert logzs[k] == logz1, k
        for got, ref in zip(_state(members[k]), st1):
            np.testing.assert_array_equal(got, ref)
    batch.close()
    for m in members:
        m.close()


def test_batch_matches_oracle_runs():
    """Twelve stages of a batch against the oracle run of every member with its
    dataset field: same temperatures, evidence, particles and subsample
    indices (member 0 reaches a = 1 within them). Longer runs drift apart
    through rounding: a difference in the last bits of a weight eventually
    flips an accept decision or a halving of the exponent search."""
    B = _binding()
    ws = W.batched_small(4, seed=2, precision=W.FP64, d_values=[2, 6, 35, 13])
    say("batch members", [(w.n, w.d, w.m) for w in ws])
    probs = [_oracle_problem(w) for w in ws]
    members = [_context(w, tb) for w, (P, tb) in zip(ws, probs)]
    batch = B.SMCBatch(members)
    S = 12
    logzs, recs = batch.run(_eps, L=ws[0].L, R=2, max_stages=S)
    assert sum(len(r) < S for r in recs) >= 1 and sum(len(r) == S for r in recs) >= 1
    for k, (w, (P, tb)) in enumerate(zip(ws, probs)):
        ref = oracle.run_smc(P, M=w.M, m=w.m, G=w.G, seed=w.seed, eps_fn=_eps, L=w.L, R=2, dataset=w.dataset,
                             max_stages=S)
        temps = np.array([r["a"] for r in recs[k]])
        say("member", k, "stages", len(temps), "logz", logzs[k], ref["logz"])
        assert len(temps) == len(ref["temps"])
        np.testing.assert_allclose(temps, ref["temps"], rtol=1e-8, atol=1e-10)
        assert abs(logzs[k] - ref["logz"]) <= 1e-7 * abs(ref["logz"])
        th, u, lw, _, _ = _state(members[k])
        np.testing.assert_allclose(th, ref["theta"], rtol=1e-6, atol=1e-8)
        np.testing.assert_array_equal(u, ref["u"])
    batch.close()
    for m in members:
        m.close()


def test_dataset_field_separates_streams():
    """Two contexts on identical data and seed draw different particles when
    their dataset fields differ, and the oracle's init with the same field
    agrees with each."""
    w = W.logistic_small(2000, 4, seed=81, M=32, m=60, G=4)
    P, tb = _oracle_problem(w)
    got = []
    for ds in (0, 5):
        w.dataset = ds
        smc = _context(w, tb)
        th, u, _, _, _ = _state(smc)
        th0, u0, _ = oracle.init_particles(w.M, w.d, w.m, w.n, w.seed, w.prior_mean, w.prior_prec, dataset=ds)
        np.testing.assert_array_equal(u, u0)
        np.testing.assert_allclose(th, th0, rtol=1e-13, atol=1e-13)
        got.append(u)
        smc.close()
    assert (got[0] != got[1]).mean() > 0.9


def test_batch_errors():
    B = _binding()
    ws = W.batched_small(2, seed=3, precision=W.FP64, d_values=[3, 4])
    members = [_context(w, _oracle_problem(w)[1]) for w in ws]
    batch = B.SMCBatch(members)
    with pytest.raises(B.SMCError):
        batch.move(0.1, 4)                             # no tempered stage yet
    with pytest.raises(B.SMCError):
        batch.mass()
    batch.temper()
    with pytest.raises(B.SMCError):
        batch.move(0.1, 4)                             # no mass matrix for this stage
    batch.mass()
    with pytest.raises(B.SMCError):
        batch.move([0.1, -1.0], 4)                     # a non-positive step
    batch.resample()
    batch.move(0.1, 4)
    batch.close()
    L = B.lib()
    assert L.smc_batch_workspace_size(0) == 0
    import ctypes as C
    h = C.c_void_p()
    handles = (C.c_void_p * 2)(members[0]._h.value, members[0]._h.value)
    ws_t = torch.empty(L.smc_batch_workspace_size(2) + 256, dtype=torch.uint8, device=DEV)
    base = (ws_t.data_ptr() + 255) & ~255
    assert L.smc_batch_create(handles, 2, C.c_void_p(base), L.smc_batch_workspace_size(2), C.byref(h)) != 0
    handles = (C.c_void_p * 2)(members[0]._h.value, members[1]._h.value)
    assert L.smc_batch_create(handles, 2, C.c_void_p(base), 64, C.byref(h)) != 0
    for m in members:
        m.close()


def test_graph_replay_equals_direct_launches():
    """The batched move replayed from a captured HIP graph gives the direct
    launches' results bit for bit, over a full run in which members reach
    a = 1 (so the graph is captured again) and with the stage's eager work
    (tempering, mass matrix, resampling) between replays."""
    B = _binding()
    ws = W.batched_small(5, seed=4, precision=W.MIXED, d_values=[4, 11, 34, 20, 7])
    centres = [_oracle_problem(w)[1] for w in ws]
    out = []
    for graph in (False, True):
        members = [_context(w, tb) for w, tb in zip(ws, centres)]
        batch = B.SMCBatch(members)
        batch.set_graph(graph)
        logzs, recs = batch.run(_eps, L=ws[0].L, R=3)
        say("graph", graph, "captures", batch.graph_captures(), "stages", [len(r) for r in recs])
        if graph:
            assert batch.graph_captures() >= 2
        else:
            assert batch.graph_captures() == 0
        out.append((logzs, [[r["a"] for r in rec] for rec in recs], [_state(m) for m in members]))
        batch.close()
        for m in members:
            m.close()
    (lz0, t0, s0), (lz1, t1, s1) = out
    assert lz0 == lz1 and t0 == t1
    for a, b in zip(s0, s1):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
def test_concurrent_launches_equal_serial(graph):
    """The move's launches spread over several streams (forked from and
    joined back to the batch's stream) give the one-stream results bit for
    bit, with and without graph replay."""
    B = _binding()
    ws = W.batched_small(6, seed=5, precision=W.MIXED, d_values=[4, 11, 34, 20, 45, 7])
    paths = [0, B.MOVE_STREAMING, 0, 0, 0, B.MOVE_STREAMING]
    centres = [_oracle_problem(w)[1] for w in ws]
    out = []
    for n in (1, 4, 8):
        members = [_context(w, tb, mp) for w, tb, mp in zip(ws, centres, paths)]
        batch = B.SMCBatch(members)
        batch.set_graph(graph)
        batch.set_streams(n)
        logzs, recs = batch.run(_eps, L=ws[0].L, R=2, max_stages=10)
        say("streams", n, "launches", batch.launches(), "stages", [len(r) for r in recs])
        out.append((logzs, [[r["a"] for r in rec] for rec in recs], [_state(m) for m in members]))
        batch.close()
        for m in members:
            m.close()
    for lz, t, st in out[1:]:
        assert lz == out[0][0] and t == out[0][1]
        for a, b in zip(st, out[0][2]):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)
    B2 = _binding()
    with pytest.raises(B2.SMCError):
        mem = [_context(ws[0], centres[0])]
        bt = B2.SMCBatch(mem)
        try:
            bt.set_streams(9)
        finally:
            bt.close()
            mem[0].close()


def test_heterogeneous_batch_equals_single_context_runs():
    """One batch mixing families (logistic, Poisson, Student-t), precisions
    (FP64 and mixed) and widths (narrow, lane-group and resident kernels):
    every member's run equals its own single-context run bit for bit."""
    B = _binding()
    ws = [W.logistic_small(1500, 5, seed=91, M=40, m=60, G=4, L=5),
          W.poisson_small(2500, 8, seed=92, precision=W.MIXED, M=48, m=80, G=4, L=5),
          W.student_small(2000, 6, seed=93, M=32, m=70, G=5, L=5),
          W.student_small(1800, 40, seed=94, precision=W.MIXED, M=24, m=90, G=3, L=5, theta_scale=0.3),
          W.poisson_small(3000, 3, seed=95, M=56, m=50, G=2, L=5)]
    for k, w in enumerate(ws):
        w.dataset = 10 + k
    paths = [0, 0, B.MOVE_STREAMING, 0, B.MOVE_STREAMING]
    P = [oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec) for w in ws]
    centres = [p.newton_mode()[0] for p in P]
    singles = []
    for w, tb, mp in zip(ws, centres, paths):
        smc = _context(w, tb, mp)
        logz, rec = smc.run(_eps, L=w.L, R=1, max_stages=8)
        singles.append((logz, [r["a"] for r in rec], _state(smc)))
        smc.close()
    members = [_context(w, tb, mp) for w, tb, mp in zip(ws, centres, paths)]
    batch = B.SMCBatch(members)
    batch.set_graph(True)
    logzs, recs = batch.run(_eps, L=ws[0].L, R=1, max_stages=8)
    say("launches", batch.launches(), "stages", [len(r) for r in recs])
    for k, s in enumerate(singles):
        logz1, temps1, st1 = s
        assert [r["a"] for r in recs[k]] == temps1, k
        assert logzs[k] == logz1, k
        for got, ref in zip(_state(members[k]), st1):
            np.testing.assert_array_equal(got, ref)
    batch.close()
    for m in members:
        m.close()


def _persistent_members(precision):
    """Members spanning every body of the persistent move: resident (subsample in LDS), a
    resident member whose layout needs more LDS than the launch's share and one that needs
    register rows (both moved by their streaming kernel in the launch), narrow and lane-group
    streaming members, particle counts that are not multiples of four, and a second family
    (a second launch)."""
    ws = [W.logistic_small(3000, 3, seed=301, precision=precision, M=50, m=300, G=4, L=4),
          W.logistic_small(20000, 5, seed=302, precision=precision, M=40, m=6000, G=20, L=4),
          W.logistic_small(12000, 12, seed=303, precision=precision, M=33, m=2500, G=10, L=4, theta_scale=0.3),
          W.logistic_small(4000, 28, seed=304, precision=precision, M=37, m=200, G=4, L=4, theta_scale=0.3),
          W.logistic_small(4000, 40, seed=305, precision=precision, M=30, m=150, G=5, L=4, theta_scale=0.25),
          W.poisson_small(3000, 6, seed=306, precision=precision, M=21, m=100, G=4, L=4)]
    for k, w in enumerate(ws):
        w.dataset = 20 + k
    return ws


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
@pytest.mark.parametrize("precision", [W.FP64, W.MIXED], ids=["fp64", "mixed"])
def test_persistent_batch_equals_single_context_runs(precision, graph):
    """The persistent move (one launch per row type and family, a device work queue over
    every member's particles, costliest member first) against each member run alone with the
    kernel the launch gave it, bit for bit over eight stages of two moves each (the queue is
    back at zero after every launch, or the next move would skip work)."""
    B = _binding()
    ws = _persistent_members(precision)
    centres = [_oracle_problem(w)[1] for w in ws]
    members = [_context(w, tb) for w, tb in zip(ws, centres)]
    batch = B.SMCBatch(members)
    batch.set_persistent(True)
    batch.set_graph(graph)
    kinds = []
    logzs, recs = batch.run(_eps, L=ws[0].L, R=2, max_stages=8,
                            callback=lambda b, a, act: kinds.append((b.member_kernels().tolist(), b.launches())))
    say("member kernels, launches per stage", kinds[:2], "stages", [len(r) for r in recs])
    first = np.array(kinds[0][0])
    assert kinds[0][1] == 2                                   # two families: two launches
    assert (first == 2).any() and (first == 0).any() and (first == 1).any()
    assert first[1] != 2                                      # register-row layout: streaming in the launch
    if precision == W.MIXED:
        assert first[2] != 2                                  # more LDS than two workgroups per CU leave
    for k, (w, tb) in enumerate(zip(ws, centres)):
        smc = _context(w, tb, 0 if first[k] == 2 else B.MOVE_STREAMING)
        logz1, rec1 = smc.run(_eps, L=ws[0].L, R=2, max_stages=8)
        assert [r["a"] for r in recs[k]] == [r["a"] for r in rec1], k
        assert logzs[k] == logz1, k
        for got, ref in zip(_state(members[k]), _state(smc)):
            np.testing.assert_array_equal(got, ref)
        smc.close()
    if graph:
        assert batch.graph_captures() >= 1
    batch.close()
    for m in members:
        m.close()


def test_persistent_batch_timing_and_launch_count():
    """With timing on, the persistent move reports one timed launch per row type and family
    (kind 3) and its results equal the untimed launches'."""
    B = _binding()
    ws = _persistent_members(W.MIXED)[:5]                     # one family: one launch
    centres = [_oracle_problem(w)[1] for w in ws]
    out = []
    for timing in (False, True):
        members = [_context(w, tb) for w, tb in zip(ws, centres)]
        batch = B.SMCBatch(members)
        batch.set_persistent(True)
        batch.set_timing(timing)
        logzs, recs = batch.run(_eps, L=ws[0].L, R=1, max_stages=3)
        if timing:
            kind, ms, ml = batch.move_timing()
            say("persistent launch", kind, ms, ml)
            assert list(kind) == [3] and ms[0] > 0 and set(ml) == {0}
        out.append((logzs, [_state(m) for m in members]))
        batch.close()
        for m in members:
            m.close()
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1], out[1][1]):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("precision", [W.FP64, W.MIXED], ids=["fp64", "mixed"])
def test_persistent_batch_edge_members(precision):
    """The persistent move at the edges of its items and bodies: a resident member of three
    particles, streaming members whose last item leaves one to three wavefronts idle (9, 7 and 6
    particles), the widest rows (d = 128), and the Gaussian and Student-t families beside
    logistic rows (three launches); each member equals its own run bit for bit."""
    B = _binding()
    ws = [W.logistic_small(2000, 5, seed=311, precision=precision, M=3, m=120, G=4, L=4),
          W.logistic_small(3000, 128, seed=312, precision=precision, M=7, m=90, G=3, L=4, theta_scale=0.1),
          W.gaussian_small(800, 3, seed=313, precision=precision, M=5, m=40, G=4, L=4),
          W.student_small(2500, 40, seed=314, precision=precision, M=9, m=110, G=5, L=4, theta_scale=0.3),
          W.logistic_small(2500, 20, seed=315, precision=precision, M=6, m=100, G=4, L=4, theta_scale=0.3)]
    for k, w in enumerate(ws):
        w.dataset = 40 + k
    P = [oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec, gauss_s2=w.gauss_s2)
         for w in ws]
    centres = [p.newton_mode()[0] for p in P]
    dt = np.float32 if precision == W.MIXED else np.float64

    def ctx(w, tb, path):
        return B.SubsampledSMC(torch.tensor(w.Xy(dt), device=DEV), w.d, w.family, w.precision, w.M, w.m, w.G,
                               w.prior_mean, w.prior_prec, w.seed, theta_bar=tb, move_path=path,
                               dataset=w.dataset, gauss_s2=w.gauss_s2)

    members = [ctx(w, tb, 0) for w, tb in zip(ws, centres)]
    batch = B.SMCBatch(members)
    batch.set_persistent(True)
    kinds = []
    logzs, recs = batch.run(_eps, L=ws[0].L, R=2, max_stages=5,
                            callback=lambda b, a, act: kinds.append((b.member_kernels().tolist(), b.launches())))
    say("member kernels, launches", kinds[0])
    first = np.array(kinds[0][0])
    assert kinds[0][1] == 3
    for k, (w, tb) in enumerate(zip(ws, centres)):
        smc = ctx(w, tb, 0 if first[k] == 2 else B.MOVE_STREAMING)
        logz1, rec1 = smc.run(_eps, L=ws[0].L, R=2, max_stages=5)
        assert [r["a"] for r in recs[k]] == [r["a"] for r in rec1], k
        assert logzs[k] == logz1, k
        for got, ref in zip(_state(members[k]), _state(smc)):
            np.testing.assert_array_equal(got, ref)
        smc.close()
    batch.close()
    for m in members:
        m.close()
