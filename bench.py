"""Throughput of the Subsampling SMC hot path on one MI355X.

One step = one stage of Algorithm 2 on a live run: tempering exponent by ESS
bisection + reweighting, mass matrix (weighted covariance + Cholesky),
systematic resampling, and one fused Markov move (block pseudo-marginal
refresh of u + HMC with L leapfrog steps). The control-variate summaries and
packed rows are built once in setup (the centre is fixed at the posterior
mode). Inputs are resident in HBM before timing starts.

Metric: particle x subsample-slot log-likelihood + gradient evaluations per
second; a move does M * m * (L + 1) of them (one estimator pass for the
u-refresh and one per leapfrog step). `value` is the mixed-precision path
(FP32 data and per-observation terms, FP64 control variates, reductions and
accept ratios); the plain FP64 path on the same data is reported beside it.

With no flags the line is the additive logistic model (n = 5e6, d = 116,
M = 4096, m = 50,000, L = 20), the largest configuration; the logistic
d = 50 (n = 1e7) and Poisson d = 20 (n = 1e6) configurations are reported
beside it under "beside".
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Published FP32 vector peak of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (FMA) x 2 (packed dual FP32) x 2.4 GHz. The kernels issue no packed FP32
# instructions, so their attainable vector rate is half of it (78.6 TFLOP/s,
# also the FP64 vector peak); that view is reported beside the fraction.
PEAK_FP32_TFLOPS = 157.3
PEAK_VALU_NONPACKED_TFLOPS = 78.6
MOVE_STREAMING, MOVE_RESIDENT = 1, 2
HEADLINE = "config5"
BESIDE = ("config4", "config2")
METRIC = "particle-obs loglik+grad evals/s (mixed vs FP64 plain, <=1e-5 rel err)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-e2e", action="store_true", help="skip the whole run to a = 1 (configurations 1 and 2)")
    ap.add_argument("--cpu-particles", type=int, default=256)
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None, help="time one path only (profiling)")
    ap.add_argument("--batch", type=int, default=64, help="members of the batched workload")
    ap.add_argument("--no-graph", action="store_true", help="batched workload: direct launches instead of graph replay")
    ap.add_argument("--per-shape", action="store_true",
                    help="batched workload: one move launch per kernel shape instead of the persistent launch")
    ap.add_argument("--streams", type=int, default=8,
                    help="batched workload: streams the move's launches are spread over (1 = one after another)")
    ap.add_argument("--workload", choices=["config1", "config2", "batched", "config4", "config5", "student"],
                    default=HEADLINE,
                    help="config5 (additive logistic n=5e6 d=116, the largest configuration) is the default "
                         "line, with config4 and config2 beside it; the others are the logistic d=5 FP64, "
                         "Poisson d=20, logistic d=50 configurations, the 64-dataset batch and the Student-t "
                         "regression n=5e5 d=50")
    ap.add_argument("--no-beside", action="store_true", help="default line only: skip config4 and config2")
    ap.add_argument("--move-path", type=int, choices=[0, 1, 2, 3], default=0,
                    help="move kernel: 0 automatic, 1 streaming, 2 resident, 3 resident with x'delta on the "
                         "matrix cores")
    ap.add_argument("--autotune", action="store_true",
                    help="after the warm-up steps, time every move kernel option on the live state "
                         "(smc_autotune_move), report the times and keep the fastest for the timed steps")
    ap.add_argument("--schemes", choices=["default", "paper"], default="default",
                    help="default: ESS root search (target M/2) and systematic resampling; paper: the grid "
                         "rule with target 0.8 M (129 points) and multinomial resampling")
    ap.add_argument("--recentre", action="store_true",
                    help="move the control-variate centre to every stage's weighted mean (Algorithm 2 step d: "
                         "a full-data CV rebuild and a re-evaluation of every particle per step)")
    ap.add_argument("--cv-order", type=int, choices=[1, 2], default=2,
                    help="2: the second-order control variate (default); 1: the first-order one of Experiment 4")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (the reference kernel for scaling "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def algorithmic_bytes_per_eval(d, fp32):
    """x_k (d values) + y_k + the 4-byte subsample index."""
    s = 4 if fp32 else 8
    return d * s + s + 4


def algorithmic_flops_per_eval(d):
    """Four length-d contractions per eval (2 flops per element each): the
    linear predictor at the centre and at theta (x'theta_bar, x'delta), and the
    two gradient sums S1 += d' x and T1 += (d - shift) d' x. The kernels store
    x'theta_bar in the packed row, so they execute 6d of these 8d; the scalar
    remainder and the FP64 sums are not counted."""
    return 8 * d


def calibrate_copy():
    import torch
    n = 256 * 1024 * 1024  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "dispatches": 3}), flush=True)


def run_path(w, precision, Xy_dev, args, eps):
    import torch
    from paper_1805_03317_amd.binding import SubsampledSMC

    path = args.move_path if (precision == 1 or args.move_path != 3) else 0
    smc = SubsampledSMC(Xy_dev, w.d, w.family, precision, w.M, w.m, w.G, w.prior_mean, w.prior_prec, w.seed,
                        cv_order=args.cv_order, move_path=path)
    evals_per_move = w.M * w.m * (w.L + 1)
    state = {"tempered": 0}

    paper = args.schemes == "paper"
    # the default schemes run as one library call per stage (the device does
    # not wait for the host between its steps); the variants call the steps
    fused = not paper and not args.recentre

    def step():
        if smc.info()["a"] < 1.0:
            state["tempered"] += 1
            if not fused:
                if paper:
                    smc.temper_grid(129, 0.8)
                else:
                    smc.temper()
        if fused:
            smc.stage(eps, w.L, 1)
            return
        smc.mass()
        if args.recentre:
            smc.recentre()
        smc.resample(multinomial=paper)
        smc.move(eps, w.L, 1)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tuned = None
    if args.autotune:
        if smc.info()["have_mass"] == 0:
            smc.mass()
        rpl, ms = smc.autotune_move(eps, w.L)
        i = smc.info()
        tuned = {"ms": [round(float(x), 4) for x in ms if x > 0], "res_rows": rpl, "res_mfma": i["res_mfma"],
                 "stream_tile": i["stream_tile"]}
    # every timed move launch is bracketed by HIP events on the context's stream
    smc.set_move_timing(args.steps)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    move_ms = float(np.mean(smc.move_times()))
    smc.set_move_timing(0)
    info = smc.info()
    acc = smc.accept.float().mean(0).cpu().numpy()
    ms = smc.move_stats()
    res = {
        "evals_per_s": args.steps * evals_per_move / elapsed,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "move_ms": move_ms,
        "move_evals_per_s": evals_per_move / (move_ms * 1e-3),
        "a": info["a"],
        "stage": info["stage"],
        "stages_tempered": state["tempered"],
        "accept_u": float(acc[0]),
        "accept_theta": float(acc[1]),
        "newton_iters": info["newton_iters"],
        "move_path": info["move_path"],
        "res_rows": info["res_rows"],
        "res_mfma": info["res_mfma"],
        "stream_tile": info["stream_tile"],
        "near_ties_last_move": [ms["near_ties_u"], ms["near_ties_theta"]],
    }
    if tuned is not None:
        res["autotune"] = tuned
    return smc, res


def laplace_state_move(smc, w, eps, reps=10, warm=3, seed=77):
    """The move on the fixed benchmark state at a = 1: theta_i ~ N(theta_bar, (-C - Q0)^{-1}) (the
    Laplace approximation at the control-variate centre), u uniform, inverse mass matrix
    (-C - Q0)^{-1}; `warm` untimed moves, then the median device time of `reps` moves, each
    from the same state."""
    import torch
    tb, _, _, Cm = smc.get_cv()
    prec = -Cm + w.prior_prec
    cov = np.linalg.inv(prec)
    cov = 0.5 * (cov + cov.T)
    g = np.random.Generator(np.random.Philox(key=seed))
    th = tb + g.standard_normal((w.M, w.d)) @ np.linalg.cholesky(cov).T
    u = g.integers(0, w.n, size=(w.M, w.m), dtype=np.int64).astype(np.int32)
    th_d = torch.tensor(th, device=smc.device)
    u_d = torch.tensor(u, device=smc.device)
    smc.set_mass(cov)
    info = smc.info()
    smc.set_move_timing(reps)
    for r in range(warm + reps):
        if r == warm:
            smc.set_move_timing(reps)          # clears the ring: only the timed moves remain
        smc.theta.copy_(th_d)
        smc.u.copy_(u_d)
        smc.refresh()
        smc.set_stage(info["stage"], 0, 1.0, info["logz"])
        smc.move(eps, w.L, 1)
    torch.cuda.synchronize()
    ms = float(np.median(smc.move_times()))
    smc.set_move_timing(0)
    st = smc.move_stats()
    return {"move_ms_median": ms, "move_evals_per_s": w.M * w.m * (w.L + 1) / (ms * 1e-3),
            "accept_u": st["accept_u"], "accept_theta": st["accept_theta"],
            "state": "a = 1, theta ~ Laplace approximation at the centre, u uniform, Sigma = (-C - Q0)^-1"}


# the device sources each move kernel is compiled from: a committed PMC summary
# counts only while these are unchanged
_COMMON_SOURCES = ["kernels.hpp", "xlane.hpp", "glm.hpp", "rng.hpp"]
DEVICE_SOURCES = {
    "move_kernel": _COMMON_SOURCES,
    "move_kernel_wide": _COMMON_SOURCES + ["kernels_wide.hpp"],
    "move_kernel_wide_group": _COMMON_SOURCES + ["kernels_wide.hpp"],
    "move_kernel_res": _COMMON_SOURCES + ["kernels_resident.hpp"],
    "move_kernel_persist": _COMMON_SOURCES + ["kernels_wide.hpp", "kernels_resident.hpp", "kernels_persist.hpp",
                                              "launch_persist.hpp"],
}


def device_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in DEVICE_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1805_03317_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def move_kernel_name(w, move_path, stream_tile=0):
    if move_path == MOVE_RESIDENT:
        return "move_kernel_res"
    if w.d <= 32:
        return "move_kernel"
    # tile form 2: the lane-group move with four particles per workgroup
    return "move_kernel_wide_group" if stream_tile == 2 else "move_kernel_wide"


def measured_traffic(w, precision, kernel, state="live"):
    """HBM bytes per move launch from the committed PMC summary, if it was
    taken on the current device sources (else None): the live stages' mean, or
    with state="a1" the mean over the moves of the fixed a = 1 state."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{w.name}_{precision}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#") and len(ln.split()) == 2:
                k, v = ln.split()
                kv[k] = v
    if kv.get("device_source_sha256") != device_source_hash(kernel):
        return None
    key = "traffic_bytes_per_launch" + ("_a1" if state == "a1" else "")
    return float(kv[key]) if key in kv else None


def roofline(w, fp32, move_ms, move_path, stream_tile=0, state="live"):
    """The move kernel against its bound. The streaming kernels re-read every
    row on every pass and are bounded by memory bandwidth; the resident kernel
    gathers the rows once per move and keeps them on chip, so its passes are
    bounded by the vector ALU."""
    evals = w.M * w.m * (w.L + 1)
    kernel = move_kernel_name(w, move_path, stream_tile)
    traffic = measured_traffic(w, "mixed" if fp32 else "fp64", kernel, state)
    if move_path == MOVE_RESIDENT:
        fpe = algorithmic_flops_per_eval(w.d)
        achieved = fpe * evals / (move_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic, "kernel": kernel,
                "flops_per_eval": fpe, "evals_per_launch": evals,
                "frac_of_nonpacked_fp32_peak": round(achieved / PEAK_VALU_NONPACKED_TFLOPS, 4)}
    bpe = algorithmic_bytes_per_eval(w.d, fp32)
    achieved = bpe * evals / (move_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": kernel, "bytes_per_eval": bpe, "evals_per_launch": evals}


def run_to_end(w, precision, Xy_dev, eps, cv_order=2):
    """A whole run of Algorithm 2 from the prior to a = 1 on a fresh context
    (one move per stage), wall clock from the first tempering step."""
    import torch
    from paper_1805_03317_amd.binding import SubsampledSMC

    smc = SubsampledSMC(Xy_dev, w.d, w.family, precision, w.M, w.m, w.G, w.prior_mean, w.prior_prec, w.seed,
                        cv_order=cv_order)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    logz, rec = smc.run(lambda st, a, d: eps, w.L, 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    acc = smc.accept.float().mean(0).cpu().numpy()
    smc.close()
    return {"stages": len(rec), "wall_s": round(wall, 4), "logz": logz, "final_accept_u": float(acc[0]),
            "final_accept_theta": float(acc[1])}


def oracle_problem(w, cv_order=2, max_cost=4e8):
    """The oracle on the workload's data with control variates at a centre near the mode: the
    generating parameter where known, else the oracle's Newton mode. When a full-data pass of the
    oracle (n d^2 extended-precision products, one thread) would take minutes, the summaries are
    built from the first rows and scaled to n (the timed move does not depend on their values
    beyond the branch mix of the remainders), at the prior mean where no generating parameter is
    known."""
    import oracle
    P = oracle.Problem(w.Xy(np.float64), w.d, w.family, w.prior_mean, w.prior_prec, cv_order=cv_order)
    cost = float(w.n) * w.d * w.d
    if cost <= max_cost:
        tb = w.theta_true if w.theta_true is not None else P.newton_mode()[0]
        P.set_cv_centre(tb)
        return P, "full-data control variates"
    n_sub = max(1000, int(max_cost / (w.d * w.d)))
    sub = oracle.Problem(w.Xy(np.float64)[:n_sub], w.d, w.family, w.prior_mean, w.prior_prec, cv_order=cv_order)
    tb = w.theta_true if w.theta_true is not None else np.array(w.prior_mean, dtype=np.float64)
    A, B, Cm = sub.cv_build(tb)
    f = w.n / n_sub
    P.set_cv(tb, A * f, B * f, Cm * f)
    return P, f"control variates from the first {n_sub} rows scaled to n"


def cpu_baseline(w, eps, budget_s=12.0, cv_order=2, one_thread=True):
    """The oracle on a bounded sample of the workload: the estimator pass with both gradients
    (eq. difference_estimator_logl and its derivative; the eval the metric counts, m per
    particle) of particles at the a = 1 benchmark state (Laplace approximation at the oracle's
    centre, u uniform), a batch of one particle per host thread at a time while the budget
    lasts; then the same on one thread. A whole move is L + 1 such passes plus the HMC
    arithmetic (one config-5 particle's move is about a minute of one core)."""
    import oracle
    P, cv_note = oracle_problem(w, cv_order)
    thp, u0, _ = oracle.init_particles(w.M, w.d, w.m, w.n, w.seed, w.prior_mean, w.prior_prec)
    cov = np.linalg.inv(-P.C + w.prior_prec)
    cov = 0.5 * (cov + cov.T)
    Lc = np.linalg.cholesky(cov)
    z = (thp - w.prior_mean) @ np.linalg.cholesky(w.prior_prec)   # standard normals
    th0 = P.theta_bar + z @ Lc.T                                   # Laplace approximation draws

    def timed(threads, budget):
        oracle.set_num_threads(threads)
        dt, done = 0.0, 0
        while done < w.M and (done == 0 or dt < budget):
            k = min(threads, w.M - done)
            t0 = time.perf_counter()
            P.estimate(th0[done:done + k], u0[done:done + k], grad=True)
            dt += time.perf_counter() - t0
            done += k
        return done, dt

    threads = oracle.num_threads()
    done, dt = timed(threads, budget_s)
    out = {"value": done * w.m / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
           "sample": f"the estimator pass with gradients of {done} of the {w.M} particles ({threads} at a time; "
                     f"same data, a=1 Laplace-approximation state, {cv_note}), {done * w.m} evals "
                     f"in {dt:.2f} s wall",
           "evals": done * w.m, "seconds": dt}
    if one_thread:
        done1, dt1 = timed(1, budget_s / 2)
        out["one_thread"] = {"value": done1 * w.m / dt1, "cores": 1,
                             "sample": f"the same pass for {done1} particles on one thread, {done1 * w.m} evals "
                                       f"in {dt1:.2f} s"}
    oracle.set_num_threads(threads)
    return out

BATCH_KINDS = {0: "move_kernel_batch", 1: "move_kernel_wide_batch", 2: "move_kernel_res_batch",
               3: "move_kernel_persist"}


def run_batched_path(ws, Xys, precision, args):
    """One batch of contexts (one per dataset) stepped together; the move's
    launches are timed with HIP events on the batch's stream."""
    import torch
    from paper_1805_03317_amd.binding import SMCBatch, SubsampledSMC

    members = [SubsampledSMC(Xy, w.d, w.family, precision, w.M, w.m, w.G, w.prior_mean, w.prior_prec, w.seed,
                             dataset=w.dataset) for w, Xy in zip(ws, Xys)]
    batch = SMCBatch(members)
    batch.set_graph(not args.no_graph)
    batch.set_streams(args.streams)
    batch.set_persistent(not args.per_shape)
    eps = np.array([1.0 / w.L for w in ws])
    L = ws[0].L
    per_member = np.array([w.M * w.m * (w.L + 1) for w in ws], dtype=np.float64)
    stream = torch.cuda.current_stream()
    state = {"evals": 0.0, "active": []}

    def step(events=None, timed=False):
        _, _, _, act = batch.temper()
        batch.mass()
        batch.resample()
        if events is not None:
            events[0].record(stream)
        batch.move(eps, L, 1)
        if events is not None:
            events[1].record(stream)
        if timed:
            state["evals"] += float(per_member[act].sum())
            state["active"].append(int(act.sum()))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k], timed=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    move_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    # one more stage with the move's launches timed one by one
    batch.set_timing(True)
    step()
    kinds, launch_ms, member_launch = batch.move_timing()
    batch.set_timing(False)
    torch.cuda.synchronize()
    acc = np.array([m.accept.float().mean(0).cpu().numpy() for m in members])
    res = {
        "evals_per_s": state["evals"] / elapsed,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "move_ms": move_ms,
        "move_evals_per_s": state["evals"] / args.steps / (move_ms * 1e-3),
        "active_members": state["active"],
        "launch_kind": kinds.tolist(),
        "member_kernels": batch.member_kernels().tolist(),
        "launch_ms": launch_ms.tolist(),
        "member_launch": member_launch.tolist(),
        "stage": [m.info()["stage"] for m in members],
        "graph_captures": batch.graph_captures(),
        "accept_u": float(acc[:, 0].mean()),
        "accept_theta": float(acc[:, 1].mean()),
    }
    return batch, members, res


def batched_launches(ws, fp32, r):
    """Per-launch algorithmic work and rate of the last timed batch move."""
    out = []
    ml = np.array(r["member_launch"])
    for g, (kind, ms) in enumerate(zip(r["launch_kind"], r["launch_ms"])):
        mem = [w for w, l in zip(ws, ml) if l == g]
        evals = sum(w.M * w.m * (w.L + 1) for w in mem)
        byts = sum(algorithmic_bytes_per_eval(w.d, fp32) * w.M * w.m * (w.L + 1) for w in mem)
        flops = sum(algorithmic_flops_per_eval(w.d) * w.M * w.m * (w.L + 1) for w in mem)
        out.append({"kernel": BATCH_KINDS[kind], "members": len(mem), "d": sorted({w.d for w in mem}),
                    "evals": evals, "ms": round(ms, 4), "alg_bytes": byts, "alg_flops": flops})
    return out


def batched_roofline(launches):
    """The dominant launch (largest device time) against its bound (a persistent launch, which
    moves every member, against HBM with every member's algorithmic bytes)."""
    g = max(launches, key=lambda x: x["ms"])
    t = g["ms"] * 1e-3
    if g["kernel"] == "move_kernel_res_batch":
        achieved = g["alg_flops"] / t / 1e12
        return {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None, "kernel": g["kernel"],
                "evals_per_launch": g["evals"], "share_of_move_time": round(g["ms"] / sum(x["ms"] for x in launches), 3)}
    achieved = g["alg_bytes"] / t / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "kernel": g["kernel"],
            "evals_per_launch": g["evals"], "share_of_move_time": round(g["ms"] / sum(x["ms"] for x in launches), 3)}


def main_batched(args):
    import torch
    from paper_1805_03317_amd import workloads as W

    t_gen = time.perf_counter()
    ws, Xf, Xd = [], [], []
    paths = ["mixed", "fp64"] if args.only is None else [args.only]
    if args.no_fp64 and args.only is None:
        paths = ["mixed"]
    for k in range(args.batch):
        w = W.config3_member(k, args.batch)
        if "mixed" in paths:
            Xf.append(torch.tensor(w.Xy(np.float32), device="cuda:0"))
        if "fp64" in paths:
            Xd.append(torch.tensor(w.Xy(np.float64), device="cuda:0"))
        w.X = w.y = None                                 # host copies no longer needed
        ws.append(w)
    torch.cuda.synchronize()
    print(f"# generated {len(ws)} datasets in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    results = {}
    for p in paths:
        prec = W.MIXED if p == "mixed" else W.FP64
        t0 = time.perf_counter()
        batch, members, res = run_batched_path(ws, Xf if p == "mixed" else Xd, prec, args)
        batch.close()
        for m in members:
            m.close()
        del batch, members
        torch.cuda.synchronize()
        res["launches"] = batched_launches(ws, p == "mixed", res)
        results[p] = res
        print(f"# {p} ({time.perf_counter() - t0:.1f} s): {res}", file=sys.stderr, flush=True)
    head = "mixed" if "mixed" in results else "fp64"
    r = results[head]
    sizes = [(w.n, w.d, w.m) for w in ws]
    out = {
        "metric": "particle-obs loglik+grad evals/s (mixed vs FP64 plain, <=1e-5 rel err)",
        "value": r["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"batched{len(ws)}_logistic_nloguniform1e4_2e6_d5_50", "members": len(ws),
                   "n_total": int(sum(n for n, _, _ in sizes)), "M": ws[0].M, "m": "max(200, 0.01 n)",
                   "G": ws[0].G, "L": ws[0].L, "R": 1, "eps": "1/L", "precision": head,
                   "step": "batched temper+mass+resample+move",
                   "move_launch": ("per kernel shape, " if args.per_shape else "persistent, ")
                   + ("direct" if args.no_graph else "hip graph replay")},
        "roofline": batched_roofline(r["launches"]),
        "move_ms": r["move_ms"],
        "move_evals_per_s": r["move_evals_per_s"],
        "launches": r["launches"],
        "run": {k: r[k] for k in ("active_members", "accept_u", "accept_theta", "graph_captures")},
        "note": "not the benchmark workload (Poisson n=1e6 d=20); reported for the configuration table",
    }
    if "fp64" in results and head == "mixed":
        f = results["fp64"]
        out["fp64"] = {"value": f["evals_per_s"], "ms_per_step": f["ms_per_step"], "move_ms": f["move_ms"],
                       "roofline": batched_roofline(f["launches"]), "launches": f["launches"],
                       "mixed_over_fp64": r["evals_per_s"] / f["evals_per_s"]}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_batched(args.batch)
    print(json.dumps(out), flush=True)


def cpu_baseline_batched(count, budget_s=12.0):
    """The oracle's move on particles of members 0, 1, ... of the batch (each as in cpu_baseline,
    all host threads) until about budget_s seconds of CPU work (at least one member)."""
    from paper_1805_03317_amd import workloads as W
    evals, secs, used, cores = 0, 0.0, [], 1
    for b in range(count):
        w = W.config3_member(b, count)
        r = cpu_baseline(w, 1.0 / w.L, budget_s=max(0.5, budget_s - secs), one_thread=False)
        evals += r["evals"]
        secs += r["seconds"]
        used.append(f"{b} (n={w.n}, d={w.d})")
        cores = r["cores"]
        if secs >= budget_s:
            break
    return {"value": evals / secs, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"the estimator pass with gradients of particles of members {', '.join(used)} (same "
                      f"data, a=1 Laplace-approximation state), {evals} evals in {secs:.1f} s wall"}


WORKLOADS = {"config1": "config1", "config2": "config2", "config4": "config4", "config5": "config5",
             "student": "student_t"}


def bench_workload(name, args, cpu, e2e):
    """Timed steps of one workload on the mixed and FP64 paths; the result line's fields."""
    import torch
    from paper_1805_03317_amd import workloads as W

    t_gen = time.perf_counter()
    w = getattr(W, WORKLOADS[name])()
    print(f"# generated {w.name} in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    eps = 1.0 / w.L
    Xy = torch.tensor(w.Xy(np.float32 if w.precision == W.MIXED else np.float64), device="cuda:0")
    torch.cuda.synchronize()

    if w.precision == W.FP64:
        paths = ["fp64"]
    else:
        paths = ["mixed", "fp64"] if args.only is None else [args.only]
    if args.no_fp64 and len(paths) > 1 and args.only is None:  # FP64-only workloads keep their path
        paths.remove("fp64")
    results = {}
    ctxs = {}
    for p in paths:
        prec = W.MIXED if p == "mixed" else W.FP64
        ctxs[p], results[p] = run_path(w, prec, Xy, args, eps)
        print(f"# {w.name} {p}: {results[p]}", file=sys.stderr, flush=True)

    head = "mixed" if "mixed" in results else "fp64"
    r = results[head]
    out = {
        "metric": METRIC,
        "value": r["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "M": w.M, "m": w.m, "G": w.G, "L": w.L,
                   "R": 1, "eps": eps, "precision": head, "step": "temper+mass+resample+move",
                   "schemes": args.schemes, "recentre": bool(args.recentre), "cv_order": args.cv_order},
        "roofline": roofline(w, head == "mixed", r["move_ms"], r["move_path"], r.get("stream_tile", 0)),
        "move_ms": r["move_ms"],
        "move_evals_per_s": r["move_evals_per_s"],
        "run": {k: r[k] for k in ("a", "stage", "stages_tempered", "accept_u", "accept_theta", "newton_iters",
                                  "move_path", "res_rows", "res_mfma", "stream_tile", "near_ties_last_move",
                                  "autotune") if k in r},
    }
    if "fp64" in results and head == "mixed":
        f = results["fp64"]
        out["fp64"] = {"value": f["evals_per_s"], "ms_per_step": f["ms_per_step"], "move_ms": f["move_ms"],
                       "roofline": roofline(w, False, f["move_ms"], f["move_path"], f.get("stream_tile", 0)),
                       "mixed_over_fp64": r["evals_per_s"] / f["evals_per_s"]}
        # error of the mixed path against the FP64 path on the same particles: l_hat (dominated by
        # the exact FP64 constant A), and its FP32-computed part d_hat = (n/m) sum_j d_j on its own
        sm, sf = ctxs["mixed"], ctxs["fp64"]
        th = sm.theta[:256].clone()
        u = sm.u[:256].clone()
        lm, s2m, dm = sm.loglik_est(th, u)
        lf, s2f, df = sf.loglik_est(th, u)
        out["mixed_rel_err"] = {
            "lhat_max": float(((lm - lf).abs() / lf.abs()).max()),
            "dhat_max": float(((dm - df).abs() / df.abs().clamp_min(1e-300)).max()),
            "dhat_over_max_dhat": float((dm - df).abs().max() / df.abs().max()),
            "sig2_max": float(((s2m - s2f).abs() / s2f.abs().clamp_min(1e-300)).max()),
            "particles": int(th.shape[0]),
        }
    # the move on the fixed benchmark state (a = 1, Laplace approximation) for the dominant path
    out["laplace_a1"] = laplace_state_move(ctxs[head], w, eps)
    out["laplace_a1"]["roofline"] = roofline(w, head == "mixed", out["laplace_a1"]["move_ms_median"],
                                             r["move_path"], r.get("stream_tile", 0), state="a1")
    if name in ("config1", "config2") and e2e:
        out["run_to_end"] = run_to_end(w, W.MIXED if head == "mixed" else W.FP64, Xy, eps, args.cv_order)
    for c in ctxs.values():
        c.close()
    del ctxs, Xy
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if cpu:
        out["cpu_baseline"] = cpu_baseline(w, eps, cv_order=args.cv_order)
    if args.recentre or args.schemes != "default" or args.cv_order != 2:
        out["note"] = (" variant: per-stage CV centre" * bool(args.recentre)
                       + " variant: first-order control variate" * (args.cv_order == 1)
                       + " variant: paper schemes (grid tempering 0.8M, multinomial)" * (args.schemes == "paper")).strip()
    return out


BESIDE_KEYS = ("value", "ms_per_step", "move_ms", "move_evals_per_s", "dtype", "config", "roofline", "fp64",
               "mixed_rel_err", "laplace_a1", "run", "run_to_end")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): sharding the particles over "
              "several GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "batched":
        main_batched(args)
        return
    out = bench_workload(args.workload, args, cpu=not args.no_cpu, e2e=not args.no_e2e)
    if args.workload == HEADLINE and not args.no_beside:
        # the other single-GPU configurations, timed with the same steps (not part of `value`)
        out["beside"] = {}
        for name in BESIDE:
            o = bench_workload(name, args, cpu=False, e2e=not args.no_e2e)
            out["beside"][name] = {k: o[k] for k in BESIDE_KEYS if k in o}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
