"""The allocation-free entry point smc_temper_noalloc through the C ABI,
against smc_temper on the same inputs: two calls in a row (the second with
fewer particles, so the shared scratch holds the first call's contents), the
all-non-finite case, and the refused sizes."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_1805_03317_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _binding():
    from paper_1805_03317_amd import binding
    return binding


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _inputs(M, seed):
    g = np.random.default_rng(seed)
    lhat = -3000 + 30 * g.standard_normal(M)
    sig2 = np.abs(g.standard_normal(M)) * 3
    lw = 0.3 * g.standard_normal(M)
    lw -= np.log(np.exp(lw - lw.max()).sum()) + lw.max()
    return lhat, sig2, lw


def _noalloc(M, lhat, sig2, logw, a_prev, ess_frac=0.5):
    B = _binding()
    out = torch.full((5,), -7.0, dtype=torch.float64, device=DEV)
    stream = torch.cuda.current_stream().cuda_stream
    st = B.lib().smc_temper_noalloc(int(M), _ptr(lhat), _ptr(sig2), _ptr(logw), float(a_prev), float(ess_frac),
                                    _ptr(out), C.c_void_p(stream))
    return st, out


@pytest.mark.parametrize("order", [(3000, 700), (4096, 1)], ids=["3000_then_700", "4096_then_1"])
def test_noalloc_temper_equals_smc_temper(order):
    B = _binding()
    for call, M in enumerate(order):
        w = W.logistic_small(500, 2, seed=41, M=M, m=16, G=2)
        Xy = torch.tensor(w.Xy(np.float64), device=DEV)
        smc = B.SubsampledSMC(Xy, w.d, w.family, W.FP64, M, w.m, w.G, w.prior_mean, w.prior_prec, w.seed,
                              theta_bar=w.theta_true)
        lhat, sig2, lw = _inputs(M, 100 + call)
        a_prev = 0.05 * (call + 1)
        smc.lhat.copy_(torch.tensor(lhat))
        smc.sig2.copy_(torch.tensor(sig2))
        smc.logw.copy_(torch.tensor(lw))
        smc.set_stage(4, 0, a_prev)
        a, dz, ess = smc.temper()
        lh_d, s2_d, lw_d = (torch.tensor(x, device=DEV) for x in (lhat, sig2, lw))
        st, out = _noalloc(M, lh_d, s2_d, lw_d, a_prev)
        assert st == 0
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        print("call", call, "M", M, "a", a, o[0], flush=True)
        assert o[0] == a and o[1] == dz and o[2] == ess and o[3] == 0.0
        assert torch.equal(lw_d, smc.logw)
        smc.close()


def test_noalloc_all_nonfinite_and_refused_sizes():
    B = _binding()
    M = 64
    lh_d = torch.full((M,), float("nan"), dtype=torch.float64, device=DEV)
    s2_d = torch.zeros(M, dtype=torch.float64, device=DEV)
    lw0 = torch.full((M,), -math.log(M), dtype=torch.float64, device=DEV)
    lw_d = lw0.clone()
    st, out = _noalloc(M, lh_d, s2_d, lw_d, 0.2)
    assert st == 0
    torch.cuda.synchronize()
    assert out[3].item() == 1.0 and torch.equal(lw_d, lw0)
    for bad_M in (0, 8193):
        st, _ = _noalloc(bad_M, lh_d, s2_d, lw_d, 0.2)
        assert st == 1
    st, _ = _noalloc(M, lh_d, s2_d, lw_d, 1.0)          # a_prev must be below 1
    assert st == 1
