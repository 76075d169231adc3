"""Checkpoint and resume at the C ABI (smc_get_state / smc_set_state).

A run of Algorithm 2 stopped after some stages and resumed from its blob in a
fresh context continues bit for bit as the uninterrupted run: every stage
after the resume gives the same exponent, evidence increment, particles,
subsample indices, weights, cached estimator and accept flags."""
import numpy as np
import pytest

from paper_1805_03317_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _binding():
    from paper_1805_03317_amd import binding
    return binding


def make(w, precision=None, move_path=0):
    B = _binding()
    prec = w.precision if precision is None else precision
    data_dt = np.float32 if w.precision == W.MIXED else np.float64
    Xy = torch.tensor(w.Xy(data_dt), device=DEV)
    return B.SubsampledSMC(Xy, w.d, w.family, prec, w.M, w.m, w.G, w.prior_mean, w.prior_prec, w.seed,
                           move_path=move_path)


def snapshot(smc):
    torch.cuda.synchronize()
    return [t.clone() for t in (smc.theta, smc.u, smc.logw, smc.lhat, smc.sig2, smc.accept)]


def same(s1, s2):
    return all(torch.equal(a, b) for a, b in zip(s1, s2))


CASES = [
    ("logistic_fp64_streaming", lambda: W.logistic_small(3000, 3, seed=91, M=64, m=150, G=4, L=5), 1),
    ("logistic_fp64_auto", lambda: W.logistic_small(3000, 3, seed=91, M=64, m=150, G=4, L=5), 0),
    ("poisson_mixed_m5000", lambda: W.poisson_small(30000, 20, seed=92, precision=W.MIXED, M=32, m=5000, G=100,
                                                    L=4), 0),
    ("logistic_mixed_d50", lambda: W.logistic_small(4000, 50, seed=93, precision=W.MIXED, M=32, m=300, G=10, L=4,
                                                    theta_scale=0.15), 0),
]


@pytest.mark.parametrize("name,mk,path", CASES, ids=[c[0] for c in CASES])
def test_resume_is_bit_identical(name, mk, path):
    w = mk()
    print("resume case", name, flush=True)
    eps, L = 1.0 / w.L, w.L
    a_run = make(w, move_path=path)
    for _ in range(3):
        a_run.stage(eps, L, 1)
    blob = a_run.get_state()
    info_at = a_run.info()
    ref = []
    for _ in range(3):
        out = a_run.stage(eps, L, 1)
        ref.append((out, snapshot(a_run), a_run.info()))
    # a fresh context, and one that has run stages of its own, both resumed from the blob
    for pre in (0, 5):
        b_run = make(w, move_path=path)
        for _ in range(pre):
            b_run.stage(eps, L, 1)
        b_run.set_state(blob)
        assert b_run.info() == info_at
        for k in range(3):
            out = b_run.stage(eps, L, 1)
            assert out == ref[k][0], (pre, k)
            assert same(snapshot(b_run), ref[k][1]), (pre, k)
            assert b_run.info() == ref[k][2], (pre, k)
        b_run.close()
    a_run.close()


def test_resume_after_recentre_and_autotune():
    """The blob carries the control-variate centre (a different centre is
    rebuilt on resume, bit for bit) and the move kernel chosen by measurement."""
    w = W.poisson_small(30000, 20, seed=94, precision=W.MIXED, M=48, m=5000, G=100, L=4)
    eps, L = 1.0 / w.L, w.L
    a_run = make(w)
    for _ in range(2):
        a_run.stage(eps, L, 1)
    a_run.temper()
    a_run.mass()
    a_run.recentre()                  # centre moved to the weighted mean of this stage
    a_run.resample()
    a_run.autotune_move(eps, L)
    a_run.move(eps, L, 1)
    blob = a_run.get_state()
    cv = a_run.get_cv()
    ref = []
    for _ in range(2):
        out = a_run.stage(eps, L, 1)
        ref.append((out, snapshot(a_run)))
    b_run = make(w)
    b_run.set_state(blob)
    cv_b = b_run.get_cv()
    assert np.array_equal(cv[0], cv_b[0]) and cv[1] == cv_b[1]
    assert np.array_equal(cv[2], cv_b[2]) and np.array_equal(cv[3], cv_b[3])
    assert b_run.info()["res_rows"] == a_run.info()["res_rows"]
    for k in range(2):
        out = b_run.stage(eps, L, 1)
        assert out == ref[k][0] and same(snapshot(b_run), ref[k][1]), k
    b_run.close()
    a_run.close()


def test_state_of_another_problem_is_refused():
    B = _binding()
    w = W.logistic_small(2000, 3, seed=95, M=32, m=100, G=4, L=4)
    a_run = make(w)
    a_run.stage(0.25, 4, 1)
    blob = a_run.get_state()
    w2 = W.logistic_small(2000, 3, seed=95, M=16, m=100, G=4, L=4)
    b_run = make(w2)
    with pytest.raises(B.SMCError) as e:
        b_run.set_state(blob)
    assert e.value.status == 1
    with pytest.raises(B.SMCError):
        a_run.set_state(blob[:-8])      # truncated
    bad = bytearray(blob)
    bad[0] ^= 0xFF                      # not a state blob
    with pytest.raises(B.SMCError):
        a_run.set_state(bytes(bad))
    # the refused calls left the context as it was
    a_run.set_state(blob)
    a_run.stage(0.25, 4, 1)
    a_run.close()
    b_run.close()


def test_move_stats_before_and_after_a_move():
    B = _binding()
    w = W.logistic_small(2000, 3, seed=96, M=64, m=100, G=4, L=4)
    smc = make(w)
    with pytest.raises(B.SMCError) as e:
        smc.move_stats()
    assert e.value.status == 2
    smc.stage(0.25, 4, 1)
    st = smc.move_stats()
    acc = smc.accept.cpu().numpy()
    assert st["accept_u"] == acc[:, 0].mean() and st["accept_theta"] == acc[:, 1].mean()
    assert st["near_ties_u"] >= 0 and st["near_ties_theta"] >= 0
    smc.close()
