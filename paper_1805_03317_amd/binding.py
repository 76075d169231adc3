"""ctypes binding of libsubsmc.so (include/subsmc.h): argument marshalling only.

PyTorch provides device memory and the stream; every step of the method runs
in the HIP library. Loading fails loudly when the library has not been built.
"""
import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsubsmc.so")

LOGISTIC, POISSON, GAUSSIAN, STUDENT_T = 0, 1, 2, 3
FP64, MIXED = 0, 1
MOVE_AUTO, MOVE_STREAMING, MOVE_RESIDENT, MOVE_RESIDENT_MFMA = 0, 1, 2, 3
STATUS = {0: "ok", 1: "invalid argument", 2: "call out of order", 3: "device error",
          4: "matrix not positive definite", 5: "non-finite weights", 6: "unsupported"}


class _Problem(C.Structure):
    _fields_ = [
        ("family", C.c_int32), ("precision", C.c_int32), ("cv_order", C.c_int32), ("d", C.c_int32),
        ("n", C.c_int64), ("ld", C.c_int32), ("xy_fp32", C.c_int32), ("Xy", C.c_void_p),
        ("gauss_s2", C.c_double), ("M", C.c_int32), ("m", C.c_int32), ("G", C.c_int32),
        ("move_path", C.c_int32), ("seed", C.c_uint64), ("dataset", C.c_uint32), ("ess_frac", C.c_double),
        ("prior_mean", C.c_void_p), ("prior_prec", C.c_void_p), ("theta_bar", C.c_void_p),
        ("theta", C.c_void_p), ("u", C.c_void_p), ("logw", C.c_void_p), ("lhat", C.c_void_p),
        ("sig2", C.c_void_p), ("accept", C.c_void_p), ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t),
    ]


class _Info(C.Structure):
    _fields_ = [("a", C.c_double), ("logz", C.c_double), ("stage", C.c_int32), ("move", C.c_int32),
                ("have_mass", C.c_int32), ("newton_iters", C.c_int32), ("move_path", C.c_int32),
                ("res_rows", C.c_int32), ("res_mfma", C.c_int32), ("stream_tile", C.c_int32)]


EXPORTS = [
    "smc_workspace_size", "smc_init", "smc_temper", "smc_temper_grid", "smc_mass", "smc_resample",
    "smc_resample_multinomial", "smc_recentre", "smc_move", "smc_stage", "smc_autotune_move", "smc_set_move_option",
    "smc_set_move_timing", "smc_move_times",
    "loglik_est", "loglik_grad", "loglik_lambda", "smc_move_stats", "smc_move_diag", "smc_get_state", "smc_set_state",
    "smc_refresh", "smc_get_info", "smc_set_stage", "smc_set_mass",
    "smc_get_mass", "smc_get_cv", "smc_full_loglik", "smc_destroy", "smc_status_string",
    "smc_last_error", "smc_batch_workspace_size", "smc_batch_create", "smc_batch_temper", "smc_batch_mass",
    "smc_batch_resample", "smc_batch_move", "smc_batch_launches", "smc_batch_set_graph", "smc_batch_set_streams", "smc_batch_graph_captures",
    "smc_batch_set_timing", "smc_batch_move_timing", "smc_temper_noalloc", "smc_batch_set_persistent",
    "smc_batch_member_kernels",
    "smc_batch_destroy", "smc_batch_last_error",
]

_lib = None


def lib():
    """Load libsubsmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_03317_amd.build` "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    L.smc_workspace_size.restype = C.c_size_t
    L.smc_workspace_size.argtypes = [C.POINTER(_Problem)]
    L.smc_init.argtypes = [C.POINTER(_Problem), vp, C.POINTER(vp)]
    L.smc_temper.argtypes = [vp, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl)]
    L.smc_temper_grid.argtypes = [vp, i32, dbl, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl), vp]
    L.smc_temper_noalloc.argtypes = [i32, vp, vp, vp, dbl, dbl, vp, vp]
    L.smc_mass.argtypes = [vp]
    L.smc_resample.argtypes = [vp]
    L.smc_resample_multinomial.argtypes = [vp]
    L.smc_recentre.argtypes = [vp, vp]
    L.smc_move.argtypes = [vp, dbl, i32, i32]
    L.smc_stage.argtypes = [vp, dbl, i32, i32, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl)]
    L.smc_autotune_move.argtypes = [vp, dbl, i32, C.POINTER(i32), vp]
    L.smc_set_move_option.argtypes = [vp, i32, i32, i32]
    L.smc_set_move_timing.argtypes = [vp, i32]
    L.smc_move_times.argtypes = [vp, i32, vp, C.POINTER(i32)]
    L.loglik_est.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.loglik_grad.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.loglik_lambda.argtypes = [vp, i32, vp, vp, dbl, vp, vp, vp]
    L.smc_move_stats.argtypes = [vp, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.smc_get_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.smc_move_diag.argtypes = [vp, vp]
    L.smc_set_state.argtypes = [vp, vp, C.c_size_t]
    L.smc_refresh.argtypes = [vp]
    L.smc_get_info.argtypes = [vp, C.POINTER(_Info)]
    L.smc_set_stage.argtypes = [vp, i32, i32, dbl, dbl]
    L.smc_set_mass.argtypes = [vp, vp]
    L.smc_get_mass.argtypes = [vp, vp, vp, vp]
    L.smc_get_cv.argtypes = [vp, vp, vp, vp, vp]
    L.smc_full_loglik.argtypes = [vp, vp, vp, vp, vp]
    L.smc_destroy.argtypes = [vp]
    L.smc_destroy.restype = None
    L.smc_status_string.restype = C.c_char_p
    L.smc_status_string.argtypes = [C.c_int]
    L.smc_last_error.restype = C.c_char_p
    L.smc_last_error.argtypes = [vp]
    L.smc_batch_workspace_size.restype = C.c_size_t
    L.smc_batch_workspace_size.argtypes = [i32]
    L.smc_batch_create.argtypes = [vp, i32, vp, C.c_size_t, C.POINTER(vp)]
    L.smc_batch_temper.argtypes = [vp, vp, vp, vp, vp]
    L.smc_batch_mass.argtypes = [vp]
    L.smc_batch_resample.argtypes = [vp, i32]
    L.smc_batch_move.argtypes = [vp, vp, i32, i32]
    L.smc_batch_launches.argtypes = [vp]
    L.smc_batch_set_graph.argtypes = [vp, i32]
    L.smc_batch_set_persistent.argtypes = [vp, i32]
    L.smc_batch_member_kernels.argtypes = [vp, vp]
    L.smc_batch_set_streams.argtypes = [vp, i32]
    L.smc_batch_graph_captures.argtypes = [vp]
    L.smc_batch_set_timing.argtypes = [vp, i32]
    L.smc_batch_move_timing.argtypes = [vp, i32, vp, vp, vp, vp]
    L.smc_batch_destroy.argtypes = [vp]
    L.smc_batch_destroy.restype = None
    L.smc_batch_last_error.restype = C.c_char_p
    L.smc_batch_last_error.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("smc_workspace_size", "smc_destroy", "smc_status_string", "smc_last_error",
                        "smc_batch_workspace_size", "smc_batch_destroy", "smc_batch_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class SMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _host_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class SubsampledSMC:
    """One Subsampling SMC run (Algorithm 2) on one GPU.

    Xy: device tensor (n, ld) float64 or float32 with rows [x_k | y_k | ...].
    Particle buffers are torch tensors owned here and filled by the library.
    """

    def __init__(self, Xy, d, family, precision, M, m, G, prior_mean, prior_prec, seed,
                 ess_frac=0.5, cv_order=2, theta_bar=None, gauss_s2=1.0, move_path=MOVE_AUTO, dataset=0):
        import numpy as np

        L = lib()
        assert Xy.is_cuda and Xy.dim() == 2 and Xy.is_contiguous()
        self.device = Xy.device
        self.Xy = Xy
        self.d, self.M, self.m, self.G = int(d), int(M), int(m), int(G)
        self.n = int(Xy.shape[0])
        dev = self.device
        self.theta = torch.zeros((M, d), dtype=torch.float64, device=dev)
        self.u = torch.zeros((M, m), dtype=torch.int32, device=dev)
        self.logw = torch.zeros(M, dtype=torch.float64, device=dev)
        self.lhat = torch.zeros(M, dtype=torch.float64, device=dev)
        self.sig2 = torch.zeros(M, dtype=torch.float64, device=dev)
        self.accept = torch.zeros((M, 2), dtype=torch.int32, device=dev)
        self._mu0 = np.ascontiguousarray(prior_mean, dtype=np.float64)
        self._Q0 = np.ascontiguousarray(prior_prec, dtype=np.float64)
        self._tb = None if theta_bar is None else np.ascontiguousarray(theta_bar, dtype=np.float64)
        pb = _Problem()
        pb.family, pb.precision, pb.cv_order, pb.d = int(family), int(precision), int(cv_order), self.d
        pb.n, pb.ld = self.n, int(Xy.shape[1])
        pb.xy_fp32 = 1 if Xy.dtype == torch.float32 else 0
        pb.Xy = Xy.data_ptr()
        pb.gauss_s2 = float(gauss_s2)
        pb.M, pb.m, pb.G = self.M, self.m, self.G
        pb.move_path = int(move_path)
        pb.seed, pb.ess_frac = int(seed), float(ess_frac)
        pb.dataset = int(dataset)
        self.dataset = int(dataset)
        pb.prior_mean = self._mu0.ctypes.data
        pb.prior_prec = self._Q0.ctypes.data
        pb.theta_bar = None if self._tb is None else self._tb.ctypes.data
        pb.theta, pb.u, pb.logw = self.theta.data_ptr(), self.u.data_ptr(), self.logw.data_ptr()
        pb.lhat, pb.sig2, pb.accept = self.lhat.data_ptr(), self.sig2.data_ptr(), self.accept.data_ptr()
        pb.workspace = 1
        nbytes = L.smc_workspace_size(C.byref(pb))
        if nbytes == 0:
            raise SMCError(1, "invalid problem (smc_workspace_size returned 0)")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        pb.workspace = (base + 255) & ~255
        pb.workspace_bytes = nbytes
        self._pb = pb
        self.stream = torch.cuda.current_stream(dev)
        h = C.c_void_p()
        st = L.smc_init(C.byref(pb), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._h = h
        if st != 0:
            msg = L.smc_last_error(h).decode() if h.value else ""
            raise SMCError(st, msg)

    # -- lifecycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().smc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise SMCError(st, lib().smc_last_error(self._h).decode())

    # -- the stage of Algorithm 2 ---------------------------------------------
    def temper(self):
        a, dz, ess = C.c_double(), C.c_double(), C.c_double()
        self._check(lib().smc_temper(self._h, C.byref(a), C.byref(dz), C.byref(ess)))
        return a.value, dz.value, ess.value

    def temper_grid(self, grid_points=129, ess_frac=0.8):
        """The paper's grid rule for the next exponent; returns a, dlogz, ess and the ESS on the grid."""
        import numpy as np
        a, dz, ess = C.c_double(), C.c_double(), C.c_double()
        grid = np.zeros(int(grid_points))
        self._check(lib().smc_temper_grid(self._h, int(grid_points), float(ess_frac), C.byref(a), C.byref(dz),
                                          C.byref(ess), _host_ptr(grid)))
        return a.value, dz.value, ess.value, grid

    def mass(self):
        self._check(lib().smc_mass(self._h))

    def resample(self, multinomial=False):
        if multinomial:
            self._check(lib().smc_resample_multinomial(self._h))
        else:
            self._check(lib().smc_resample(self._h))

    def move(self, eps, L, R=1):
        self._check(lib().smc_move(self._h, float(eps), int(L), int(R)))

    def autotune_move(self, eps, L):
        """Time the allowed move kernels from the current state (restored
        afterwards) and keep the fastest; returns (register rows per lane or
        -1 for streaming, the timed ms of each option)."""
        import numpy as np
        rpl = C.c_int32()
        ms = np.zeros(8, dtype=np.float32)
        self._check(lib().smc_autotune_move(self._h, float(eps), int(L), C.byref(rpl), _host_ptr(ms)))
        return rpl.value, ms

    def set_move_option(self, res_rows=-1, res_mfma=0, stream_tile=0):
        """Pick the move kernel: res_rows = -1 streaming (tile form stream_tile), else resident."""
        self._check(lib().smc_set_move_option(self._h, int(res_rows), int(res_mfma), int(stream_tile)))

    def set_move_timing(self, n):
        self._check(lib().smc_set_move_timing(self._h, int(n)))

    def move_times(self, cap=4096):
        """Device ms of the last timed move launches, oldest first."""
        import numpy as np
        ms = np.zeros(int(cap), dtype=np.float32)
        cnt = C.c_int32()
        self._check(lib().smc_move_times(self._h, int(cap), _host_ptr(ms), C.byref(cnt)))
        return ms[:cnt.value].astype(np.float64)

    def stage(self, eps, L, R=1):
        """temper (until a = 1), mass, resample and move in one call; returns a, dlogz, ess."""
        a, dz, ess = C.c_double(), C.c_double(), C.c_double()
        self._check(lib().smc_stage(self._h, float(eps), int(L), int(R), C.byref(a), C.byref(dz), C.byref(ess)))
        return a.value, dz.value, ess.value

    def recentre(self, theta_bar=None):
        """Move the control-variate centre (default: this stage's weighted mean) and re-evaluate the caches."""
        import numpy as np
        if theta_bar is None:
            self._check(lib().smc_recentre(self._h, None))
        else:
            tb = np.ascontiguousarray(theta_bar, dtype=np.float64)
            self._check(lib().smc_recentre(self._h, _host_ptr(tb)))

    def refresh(self):
        self._check(lib().smc_refresh(self._h))

    # -- estimator entry points -------------------------------------------------
    def loglik_est(self, theta, u):
        theta = theta.contiguous()
        u = u.contiguous()
        cnt = theta.shape[0]
        lh = torch.empty(cnt, dtype=torch.float64, device=self.device)
        s2 = torch.empty_like(lh)
        dh = torch.empty_like(lh)
        self._check(lib().loglik_est(self._h, cnt, _ptr(theta), _ptr(u), _ptr(lh), _ptr(s2), _ptr(dh)))
        return lh, s2, dh

    def loglik_grad(self, theta, u, g_lhat=None, g_sig2=None, separate=False):
        theta = theta.contiguous()
        u = u.contiguous()
        cnt = theta.shape[0]
        grad = torch.empty((cnt, self.d), dtype=torch.float64, device=self.device)
        gl = torch.empty_like(grad) if separate else None
        gs = torch.empty_like(grad) if separate else None
        gl_in = None if g_lhat is None else g_lhat.to(torch.float64).contiguous()
        gs_in = None if g_sig2 is None else g_sig2.to(torch.float64).contiguous()
        self._check(lib().loglik_grad(self._h, cnt, _ptr(theta), _ptr(u), _ptr(gl_in), _ptr(gs_in),
                                      _ptr(grad), _ptr(gl), _ptr(gs)))
        return (grad, gl, gs) if separate else grad

    def loglik_lambda(self, theta, u, a):
        """lambda_a = a l_hat - a^2 sigma2_hat / 2 per particle; returns (lam, lhat, sig2)."""
        theta = theta.contiguous()
        u = u.contiguous()
        cnt = theta.shape[0]
        lam = torch.empty(cnt, dtype=torch.float64, device=self.device)
        lh = torch.empty_like(lam)
        s2 = torch.empty_like(lam)
        self._check(lib().loglik_lambda(self._h, cnt, _ptr(theta), _ptr(u), float(a), _ptr(lam), _ptr(lh),
                                        _ptr(s2)))
        return lam, lh, s2

    # -- state access -----------------------------------------------------------
    def move_stats(self):
        """Last move: accept rates of the u refresh and of HMC, near-tie counts of both."""
        au, at = C.c_double(), C.c_double()
        tu, tt = C.c_int64(), C.c_int64()
        self._check(lib().smc_move_stats(self._h, C.byref(au), C.byref(at), C.byref(tu), C.byref(tt)))
        return {"accept_u": au.value, "accept_theta": at.value, "near_ties_u": tu.value,
                "near_ties_theta": tt.value}

    def move_diag(self):
        """Last move, per particle: [log r, log U] of the u refresh, then of the HMC step (M x 4)."""
        import numpy as np
        out = np.zeros((self.M, 4))
        self._check(lib().smc_move_diag(self._h, _host_ptr(out)))
        return out

    def get_state(self):
        """Checkpoint of the run as bytes (smc_get_state)."""
        n = C.c_size_t(0)
        self._check(lib().smc_get_state(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(lib().smc_get_state(self._h, buf, C.byref(n)))
        return bytes(buf.raw[:n.value])

    def set_state(self, blob):
        """Resume from bytes written by get_state of a context of the same problem."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self._check(lib().smc_set_state(self._h, buf, len(blob)))

    def info(self):
        o = _Info()
        self._check(lib().smc_get_info(self._h, C.byref(o)))
        return {"a": o.a, "logz": o.logz, "stage": o.stage, "move": o.move, "have_mass": o.have_mass,
                "newton_iters": o.newton_iters, "move_path": o.move_path, "res_rows": o.res_rows,
                "res_mfma": o.res_mfma, "stream_tile": o.stream_tile}

    def set_stage(self, stage, move, a, logz=0.0):
        self._check(lib().smc_set_stage(self._h, int(stage), int(move), float(a), float(logz)))

    def set_mass(self, Sigma):
        import numpy as np
        S = np.ascontiguousarray(Sigma, dtype=np.float64)
        self._check(lib().smc_set_mass(self._h, _host_ptr(S)))

    def get_mass(self):
        import numpy as np
        d = self.d
        S, Lc, Li = np.zeros((d, d)), np.zeros((d, d)), np.zeros((d, d))
        self._check(lib().smc_get_mass(self._h, _host_ptr(S), _host_ptr(Lc), _host_ptr(Li)))
        return S, Lc, Li

    def get_cv(self):
        import numpy as np
        d = self.d
        tb, A, B, Cm = np.zeros(d), np.zeros(1), np.zeros(d), np.zeros((d, d))
        self._check(lib().smc_get_cv(self._h, _host_ptr(tb), _host_ptr(A), _host_ptr(B), _host_ptr(Cm)))
        return tb, float(A[0]), B, Cm

    def full_loglik(self, theta):
        import numpy as np
        d = self.d
        th = np.ascontiguousarray(theta, dtype=np.float64)
        A, B, Cm = np.zeros(1), np.zeros(d), np.zeros((d, d))
        self._check(lib().smc_full_loglik(self._h, _host_ptr(th), _host_ptr(A), _host_ptr(B), _host_ptr(Cm)))
        return float(A[0]), B, Cm

    # -- a full run ---------------------------------------------------------------
    def run(self, eps_fn, L, R, max_stages=100000, callback=None, schemes="default", grid_points=129,
            grid_ess_frac=0.8, recentre=False):
        """Algorithm 2 until a = 1; returns log Z and the per-stage record.

        schemes="paper" uses the paper's grid rule for the exponent (target
        grid_ess_frac * M) and multinomial resampling. recentre=True moves the
        control-variate centre to each stage's weighted mean (step d)."""
        paper = schemes == "paper"
        fused = not paper and not recentre
        rec = []
        a = self.info()["a"]
        while a < 1.0 and len(rec) < max_stages:
            if fused and not eps_depends_on_a(eps_fn):
                # one library call per stage: the same steps and results, without
                # the device waiting for the host between them
                eps = eps_fn(len(rec) + 1, None, self.d)
                a, dz, ess = self.stage(eps, L, R)
            else:
                if paper:
                    a, dz, ess, _ = self.temper_grid(grid_points, grid_ess_frac)
                else:
                    a, dz, ess = self.temper()
                self.mass()
                if recentre:
                    self.recentre()
                self.resample(multinomial=paper)
                eps = eps_fn(len(rec) + 1, a, self.d)
                self.move(eps, L, R)
            rec.append({"a": a, "dlogz": dz, "ess": ess, "eps": eps})
            if callback:
                callback(self, rec[-1])
        return self.info()["logz"], rec


def eps_depends_on_a(eps_fn):
    """True unless eps_fn(stage, a, d) ignores a (tried with two exponents)."""
    try:
        return eps_fn(1, 0.25, 2) != eps_fn(1, 0.75, 2)
    except Exception:
        return True


class SMCBatch:
    """Many SubsampledSMC runs advanced together (one launch per step for all
    of them; the move: one launch per kernel shape among the members).

    Each member's results are those of its own single-context run."""

    def __init__(self, members):
        import numpy as np
        L = lib()
        self.members = list(members)
        self.count = len(self.members)
        handles = (C.c_void_p * self.count)(*[m._h.value for m in self.members])
        self._handles = handles
        nbytes = L.smc_batch_workspace_size(self.count)
        if nbytes == 0:
            raise SMCError(1, "invalid batch size")
        dev = self.members[0].device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = (self.workspace.data_ptr() + 255) & ~255
        h = C.c_void_p()
        st = L.smc_batch_create(handles, self.count, C.c_void_p(base), nbytes, C.byref(h))
        if st != 0:
            raise SMCError(st, "smc_batch_create")
        self._h = h
        self._a = np.zeros(self.count)
        self._dz = np.zeros(self.count)
        self._ess = np.zeros(self.count)
        self._act = np.zeros(self.count, dtype=np.int32)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().smc_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise SMCError(st, lib().smc_batch_last_error(self._h).decode())

    def temper(self):
        """Returns (a, dlogz, ess, active) arrays over the members."""
        self._check(lib().smc_batch_temper(self._h, _host_ptr(self._a), _host_ptr(self._dz), _host_ptr(self._ess),
                                           _host_ptr(self._act)))
        return self._a.copy(), self._dz.copy(), self._ess.copy(), self._act.astype(bool)

    def mass(self):
        self._check(lib().smc_batch_mass(self._h))

    def resample(self, multinomial=False):
        self._check(lib().smc_batch_resample(self._h, 1 if multinomial else 0))

    def move(self, eps, L, R=1):
        import numpy as np
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (self.count,)))
        self._check(lib().smc_batch_move(self._h, _host_ptr(e), int(L), int(R)))

    def launches(self):
        return int(lib().smc_batch_launches(self._h))

    def set_graph(self, on=True):
        self._check(lib().smc_batch_set_graph(self._h, 1 if on else 0))

    def set_streams(self, n):
        """Streams the move's launches are spread over (1..8)."""
        self._check(lib().smc_batch_set_streams(self._h, int(n)))

    def set_persistent(self, on=True):
        """One persistent move launch per row type and family, with a device work queue."""
        self._check(lib().smc_batch_set_persistent(self._h, 1 if on else 0))

    def member_kernels(self):
        """The kernel each member's last move ran: 0 narrow, 1 lane-group, 2 resident, -1 none."""
        import numpy as np
        kind = np.zeros(self.count, dtype=np.int32)
        self._check(lib().smc_batch_member_kernels(self._h, _host_ptr(kind)))
        return kind

    def graph_captures(self):
        return int(lib().smc_batch_graph_captures(self._h))

    def set_timing(self, on=True):
        self._check(lib().smc_batch_set_timing(self._h, 1 if on else 0))

    def move_timing(self):
        """Launches of the last move: (kind per launch, device ms per launch, launch per member)."""
        import numpy as np
        cap = 64
        n = C.c_int32()
        kind = np.zeros(cap, dtype=np.int32)
        ms = np.zeros(cap)
        ml = np.zeros(self.count, dtype=np.int32)
        self._check(lib().smc_batch_move_timing(self._h, cap, C.byref(n), _host_ptr(kind), _host_ptr(ms),
                                                _host_ptr(ml)))
        return kind[:n.value].copy(), ms[:n.value].copy(), ml

    def run(self, eps_fn, L, R, max_stages=100000, callback=None):
        """Algorithm 2 for every member until all reach a = 1; returns the
        members' log Z and per-member stage records."""
        import numpy as np
        recs = [[] for _ in range(self.count)]
        steps = 0
        while steps < max_stages and any(m.info()["a"] < 1.0 for m in self.members):
            a, dz, ess, act = self.temper()
            self.mass()
            self.resample()
            eps = np.array([eps_fn(len(recs[k]) + 1, a[k], m.d) if act[k] else 1.0
                            for k, m in enumerate(self.members)])
            self.move(eps, L, R)
            for k in np.flatnonzero(act):
                recs[k].append({"a": a[k], "dlogz": dz[k], "ess": ess[k], "eps": eps[k]})
            steps += 1
            if callback:
                callback(self, a, act)
        return [m.info()["logz"] for m in self.members], recs


class LogLikEstimate(torch.autograd.Function):
    """(l_hat, sigma2_hat) per particle with the hand-written HIP backward."""

    @staticmethod
    def forward(ctx, theta, u, smc):
        lh, s2, _ = smc.loglik_est(theta.detach(), u)
        ctx.save_for_backward(theta.detach(), u)
        ctx.smc = smc
        return lh, s2

    @staticmethod
    def backward(ctx, g_lhat, g_sig2):
        theta, u = ctx.saved_tensors
        grad = ctx.smc.loglik_grad(theta, u, g_lhat, g_sig2)
        return grad, None, None


def loglik(theta, u, smc):
    return LogLikEstimate.apply(theta, u, smc)
