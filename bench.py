"""Benchmark: ANOVA fast-summation matvecs/s on one MI355X.

Default workload (the headline): N = 1e6 points, d = 9 features uniform in
[-1/4, 1/4), three windows of three features (weights 1/3), Gaussian width
ell = 0.2, beta = 1, float32 NFFT stages with float64 accumulation, plan
parameters chosen for a per-entry error estimate <= 1e-4.  One "step" is one
full (K~ + beta I) alpha over all windows for one right-hand side, with all
inputs resident in HBM.

Prints one JSON line with the throughput, the roofline of the dominant
kernel (per-launch durations from HIP events recorded on the launching
stream over the timed region), the same product at the fixed bandwidth
M = 64, m = 6, n = 128, and the oracle's CPU time on a bounded sample of
rows (the only use of the oracle here), whose rows also give the error of
the GPU result.  Further legs (each can be skipped): the measured
parameter choice, the precision split, the batched and large
configurations, the lambda grid by shifted CG, the regularised kernel,
the end-to-end classifier (fit / predict / accuracy), prediction at 1e6
test points, and served solves.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# float32 FMA without packed instructions (the library is built without
# them): 256 CUs x 64 lanes x 2 flop x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 78.6
# the chip's float32 vector peak counting packed instructions (which this
# library does not emit), reported beside the fraction for reference
VALU_FP32_PACKED_PEAK_TFLOPS = 157.3
C_EVAL = 8  # flops charged per window evaluation (a fixed charge, not the kernels' own count)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "headline_pmc_traffic.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000, help="points")
    ap.add_argument("--target", type=float, default=1e-4)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate oracle CPU time for the baseline sample")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fixed", action="store_true")
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests of the serving stream (first 10%% are warm-up)")
    ap.add_argument("--serve-load", type=float, default=0.75,
                    help="Poisson arrival rate as a fraction of the measured capacity")
    ap.add_argument("--serve-n-hi", type=int, default=500_000)
    ap.add_argument("--serve-budget-gb", type=float, default=32.0,
                    help="device memory the live requests may hold together")
    ap.add_argument("--serve-round", type=int, default=4,
                    help="CG iterations per scheduling round of the serving loop")
    ap.add_argument("--sweep-requests", type=int, default=300,
                    help="requests per arrival rate of the serving rate sweep (0: no sweep)")
    ap.add_argument("--sweep-n-hi", type=int, default=50_000,
                    help="largest N of the rate sweep's requests")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-tuned", action="store_true")
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--skip-predict", action="store_true")
    ap.add_argument("--skip-grid", action="store_true")
    ap.add_argument("--skip-e2e", action="store_true")
    ap.add_argument("--skip-reg", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run 5 device-to-device copies of 1 GiB (counter calibration)")
    return ap.parse_args()


def alg_bytes(stage: str, N: int, G: int, elem: int, P: int = 3, per_cell: bool = True) -> float:
    """Algorithmic HBM bytes of a stage for one window (the combine: for the
    whole product).  elem = 4 B (float32 NFFT) or 8 B (float64):
    permute (per-point kernels only): permutation index 4 B, the gathered
              float64 coefficient 8 B and the sorted coefficient written;
    spread  : per-cell (float32): the point's three offsets 12 B, its
              permutation index 4 B and float64 coefficient 8 B; per-point:
              node record (16 B f32 / 32 B f64) + sorted coefficient; one
              write of each grid value;
    tile_sum, fold : one write of each grid value (the tile regions they read
              are traffic of this implementation, not of the method);
    convolve (one axis pass): one read and one write of the grid;
    gather  : the offsets (12 B per-cell, the node record per-point), the
              permutation index 4 B and one value written (in the caller's
              order) per point, one read of each grid value;
    combine (all windows): alpha read and output write 16 B per point, plus
              each window's value per point."""
    node = 16 if elem == 4 else 32
    if stage == "permute":
        return N * (4 + 8 + elem)
    if stage == "spread":
        return (N * (12 + 4 + 8) if per_cell else N * (node + elem)) + G * elem
    if stage == "gather":
        return N * ((12 if per_cell else node) + 4 + elem) + G * elem
    if stage == "combine":
        return N * (16 + P * elem)
    if stage == "convolve":
        return 2.0 * G * elem
    return float(G * elem)  # tile_sum, fold


def alg_flops(N: int, dA: int, W: int) -> float:
    """Algorithmic flops of one window's spread or gather (an FMA counts 2):
    per point, 2 W^d_A for the tensor-product sum over the W^d_A support
    points, plus d_A W window evaluations at C_EVAL flops each.  The
    kernels' own instruction counts (degree-7 polynomials evaluated in
    mirror pairs, weight products) are not what is charged."""
    return float(N) * (2 * W ** dA + dA * W * C_EVAL)


def measured_traffic(kernel_stage: str):
    """HBM bytes per launch of a stage from the committed counter summary,
    if it was taken from the current kernel source (else None)."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    src = os.path.join(ROOT, "paper_2111_10140_amd", "csrc", "kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if f"kernel_source_sha256: {digest}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"traffic {kernel_stage}:"):
            return float(line.split(":")[1].split()[0])
    return None


def time_matvecs(A, torch, plan, a, out, beta, steps, warmup):
    for _ in range(warmup):
        A.anova_matvec(plan, a, out, beta)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        A.anova_matvec(plan, a, out, beta)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def graph_timing(A, torch, plan, a, out, beta, steps, warmup):
    """One product captured into a graph (the launch tables are built by an
    eager product first, so nothing is allocated or uploaded inside the
    capture), `warmup` replays, then `steps` back-to-back replays timed
    together, then `steps` more each bracketed by events on the replaying
    stream.  Returns (graph, mean ms over the timed region, sorted
    per-replay ms, every replay equal to the eager result)."""
    A.anova_matvec(plan, a, out, beta)
    torch.cuda.synchronize()
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.anova_matvec(plan, a, out, beta)
    ok = True
    for _ in range(max(warmup, 1)):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        ok = ok and torch.equal(out, ref)
    # the timed region: `steps` back-to-back replays between two events
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        g.replay()
    t1.record()
    torch.cuda.synchronize()
    # the distribution: the same number of replays, each between events of
    # its own (the extra event records are outside the timed region above)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for e0, e1 in ev:
        e0.record()
        g.replay()
        e1.record()
    torch.cuda.synchronize()
    per = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    ok = ok and torch.equal(out, ref)
    return g, t0.elapsed_time(t1) / steps, per, ok


def cold_timing(torch, g, reps=20):
    """Replays of the captured product, each after 512 MiB of writes that
    evict the 256 MB Infinity Cache and the L2 caches: sorted ms."""
    flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for r, (e0, e1) in enumerate(ev):
        flush.fill_(float(r))
        e0.record()
        g.replay()
        e1.record()
    torch.cuda.synchronize()
    del flush
    return sorted(e0.elapsed_time(e1) for e0, e1 in ev)


def pct(v, q):
    return float(np.percentile(np.asarray(v), q))


def stage_profile(A, torch, plan, a, out, beta, steps):
    plan.set_timing(True)
    for _ in range(steps):
        A.anova_matvec(plan, a, out, beta)
    torch.cuda.synchronize()
    t = plan.stage_times()
    plan.set_timing(False)
    return t


def serve_stream(Server, ex, reqs, arrivals, budget, max_live, round_iters=4):
    """Feed requests to a server at the given arrival offsets (seconds) in
    real time; returns the server once every request is done."""
    srv = Server(ex, budget=budget, max_live=max_live, iters_per_round=round_iters, planners=4)
    order = sorted(range(len(reqs)), key=lambda k: arrivals[k])
    t0 = time.perf_counter()
    k = 0
    while k < len(order) or srv.busy():
        now = time.perf_counter() - t0
        while k < len(order) and arrivals[order[k]] <= now:
            p = reqs[order[k]].problem
            srv.submit(p.X, p.windows, p.ell, p.beta, p.y, tol=1e-6, maxit=2000,
                       arrival=t0 + arrivals[order[k]])
            k += 1
        if srv.busy():
            srv.step()
        elif k < len(order):
            time.sleep(max(0.0, arrivals[order[k]] - (time.perf_counter() - t0)))
    srv.close()
    return srv


def precision_split(A, torch, X, p, a, out, plan32, target):
    """The float32-NFFT path (float64 CG, float64 residuals) against the
    plain float64 path on the same GPU, both planned for the same per-entry
    error target: matvecs/s and one full CG solve of the headline system."""
    y = torch.from_numpy(np.ascontiguousarray(p.y[:, 0])).cuda()
    res, xs = {}, {}
    plan64 = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, A.ANOVA_FP64,
                                                              target_err=target))
    for name, plan in [("fp32_nfft", plan32), ("fp64_plain", plan64)]:
        ms = time_matvecs(A, torch, plan, a, out, p.beta, 50, 5)
        x = torch.empty_like(y)
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = A.krr_cg_solve(plan, y, x, p.beta, 1e-6, 3000, allow_not_converged=True)
        torch.cuda.synchronize()
        t_cg = time.perf_counter() - t
        xs[name] = x.cpu().numpy()
        i0 = plan.info(0)
        res[name] = {"matvecs_per_s": round(1e3 / ms, 2), "ms_per_matvec": round(ms, 4),
                     "params": dict(M=i0.M, n=i0.n, m=i0.m), "err_estimate": plan.err_estimate(),
                     "cg_iters": info[0]["iters"], "cg_true_relres": info[0]["true_relres"],
                     "cg_seconds": round(t_cg, 4)}
    plan64.destroy()
    d = np.linalg.norm(xs["fp32_nfft"] - xs["fp64_plain"]) / np.linalg.norm(xs["fp64_plain"])
    res["solution_rel_diff"] = float(d)
    # precision alone: the float64 path at the float32 plan's (M, n, m, h)
    i0 = plan32.info(0)
    plan64s = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, A.ANOVA_FP64, M=i0.M, n=i0.n,
                                                               m=i0.m, h=i0.h))
    x64s = torch.empty_like(y)
    A.krr_cg_solve(plan64s, y, x64s, p.beta, 1e-6, 3000, allow_not_converged=True)
    torch.cuda.synchronize()
    plan64s.destroy()
    x64s = x64s.cpu().numpy()
    res["solution_rel_diff_same_params"] = float(np.linalg.norm(xs["fp32_nfft"] - x64s) /
                                                 np.linalg.norm(x64s))
    res["cg"] = ("tol 1e-6 on y of the headline workload, beta=1, x0=0; each path plans its own "
                 "parameters for the same error target, so the solutions differ by both "
                 "approximations as well as by precision")
    return res


def cg_iteration_timing(A, torch, plan, p, product_ms, iters=400, warmup=20):
    """Device time of CG iterations on the headline system: one solve
    advanced by krr_cg_iterate (one captured graph per iteration: the
    product, whose combine also reduces p.q, the fused x/r update with its
    r.r reduction, and the p update; every 50th iteration adds the float64
    residual product), timed with events on the stream over `iters`
    iterations after `warmup`; tol 0 keeps every iteration active."""
    y = torch.from_numpy(np.ascontiguousarray(p.y[:, 0])).cuda()
    x = torch.empty_like(y)
    sv = A.Solve(plan, y, x, p.beta, 0.0, iters + warmup + 10)
    A.krr_cg_iterate([sv], warmup)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    A.krr_cg_iterate([sv], iters)
    t1.record()
    torch.cuda.synchronize()
    us = t0.elapsed_time(t1) * 1e3 / iters
    sv.destroy()
    return {"us_per_iteration": round(us, 2), "iterations": iters,
            "product_us": round(product_ms * 1e3, 2),
            "iteration_over_product": round(us / (product_ms * 1e3), 3),
            "includes": "float64 residual product every 50th iteration"}


def batched_config(A, torch):
    """The batched configuration (64 problems, N log-uniform in [5000,
    200000], windows of 3, 2 and 1 features, 4 right-hand sides, float32
    products with float64 CG): all problems solved together (one launch per
    stage and kernel signature per CG iteration, captured in a hipGraph)
    against the same solves one after another."""
    import workloads
    probs = workloads.batched()
    t = time.perf_counter()
    plans = [A.anova_fastsum_plan_host(p.X, p.windows, A.make_params(p.ell, A.ANOVA_FP32_NFFT,
                                                                     target_err=1e-4))
             for p in probs]
    plan_s = time.perf_counter() - t

    def cols(a):
        return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().T

    ys = [cols(p.y) for p in probs]
    xs = [torch.empty((p.nrhs, p.N), dtype=torch.float64, device="cuda").T for p in probs]
    A.krr_cg_solve_batched(plans[:2], ys[:2], xs[:2], [1.0, 1.0], 1e-6, 3000)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    infos = A.krr_cg_solve_batched(plans, ys, xs, [p.beta for p in probs], 1e-6, 3000)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    t = time.perf_counter()
    for k, p in enumerate(probs):
        A.krr_cg_solve(plans[k], ys[k], xs[k], p.beta, 1e-6, 3000)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    ms = [dict(d_A=i.d_A, M=i.M, n=i.n, m=i.m, per_cell=i.per_cell)
          for i in (plans[0].info(w) for w in range(plans[0].P))]
    cols_info = [i for inf in infos for i in inf]
    work = sum(i["iters"] * p.N * len(p.windows) for p, inf in zip(probs, infos) for i in inf)
    for pl in plans:
        pl.destroy()
    return {"workload": "64 problems, N log-uniform in [5000, 200000], d=6 windows {0,1,2},"
                        "{3,4},{5}, 4 RHS, ell in {0.1,0.2,0.4}, beta=1, tol 1e-6",
            "sum_N": int(sum(p.N for p in probs)), "plan_seconds": round(plan_s, 3),
            "solve_seconds_together": round(t_batch, 4),
            "solve_seconds_one_by_one": round(t_seq, 4),
            "speedup_together": round(t_seq / t_batch, 3),
            "solves_per_s_together": round(len(probs) / t_batch, 2),
            "point_window_products_per_s": work / t_batch,
            "all_converged": all(i["converged"] for i in cols_info),
            "max_true_relres": max(i["true_relres"] for i in cols_info),
            "max_iters": max(i["iters"] for i in cols_info),
            "first_problem_params": ms}


def large_config(A, torch):
    """The large configuration (N = 2e6, mixture in R^15, five windows of
    three features, ell = 0.15, beta = 0.5) at M = 64, m = 6, n = 128:
    float32 products (float64 CG and residuals) against the plain float64
    path on the same GPU: matvecs/s and a CG solve to 1e-6."""
    import workloads
    p = workloads.large()
    X = torch.from_numpy(p.X).cuda()
    a = torch.from_numpy(np.ascontiguousarray(p.alpha[:, 0])).cuda()
    y = torch.from_numpy(np.ascontiguousarray(p.y[:, 0])).cuda()
    out = torch.empty_like(a)
    res, xs = {}, {}
    for name, prec in (("fp32_nfft", A.ANOVA_FP32_NFFT), ("fp64_plain", A.ANOVA_FP64)):
        t = time.perf_counter()
        plan = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, prec, M=64, m=6, n=128))
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t
        ms = time_matvecs(A, torch, plan, a, out, p.beta, 10, 2)
        x = torch.empty_like(y)
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = A.krr_cg_solve(plan, y, x, p.beta, 1e-6, 3000, allow_not_converged=True)
        torch.cuda.synchronize()
        xs[name] = x.cpu().numpy()
        res[name] = {"matvecs_per_s": round(1e3 / ms, 2), "plan_seconds": round(plan_s, 3),
                     "err_estimate": plan.err_estimate(), "cg_iters": info[0]["iters"],
                     "cg_true_relres": info[0]["true_relres"],
                     "cg_seconds": round(time.perf_counter() - t, 3),
                     "per_cell": plan.info(0).per_cell}
        plan.destroy()
        print(f"# large {name}: {json.dumps(res[name])}", file=sys.stderr, flush=True)
    res["solution_rel_diff"] = float(np.linalg.norm(xs["fp32_nfft"] - xs["fp64_plain"]) /
                                     np.linalg.norm(xs["fp64_plain"]))
    res["workload"] = ("N=2e6 mixture in R^15, 5 windows of 3 features, ell=0.15, beta=0.5, "
                       "M=64 m=6 n=128, CG tol 1e-6")
    return res


def predict_config(A, torch, steps):
    """Prediction at new points: 1e6 training and 1e6 test points of the
    headline distribution (the paper's experiments split each sample into
    training and test halves), float32 plan for a per-entry estimate <= 1e-4;
    predictions/s (one = all test points for one coefficient vector), the
    per-stage split.  Its parity with the oracle is a test, not part of this
    timing."""
    import workloads
    p, Zn = workloads.train_test(1_000_000, 1_000_000, seed=31)
    X = torch.from_numpy(p.X).cuda()
    Z = torch.from_numpy(Zn).cuda()
    a_np = np.ascontiguousarray(p.alpha[:, 0])
    a = torch.from_numpy(a_np.copy()).cuda()
    out = torch.empty(Zn.shape[0], dtype=torch.float64, device="cuda")
    t = time.perf_counter()
    plan = A.anova_predict_plan(X, Z, p.windows, A.make_params(p.ell, A.ANOVA_FP32_NFFT,
                                                               target_err=1e-4))
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t
    for _ in range(3):
        A.anova_predict(plan, a, out)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        A.anova_predict(plan, a, out)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / steps
    plan.set_timing(True)
    for _ in range(10):
        A.anova_predict(plan, a, out)
    torch.cuda.synchronize()
    st = plan.stage_times()
    plan.set_timing(False)
    res = {"workload": "train N=1e6, test Nz=1e6, d=9, 3 windows of 3 features, ell=0.2, "
                       "float32, per-entry estimate <= 1e-4",
           "ms_per_predict": round(ms, 4), "predicts_per_s": round(1e3 / ms, 2),
           "test_points_per_s": round(Zn.shape[0] / (ms * 1e-3), 1),
           "plan_seconds": round(plan_s, 3),
           "params": [dict(M=i.M, n=i.n, m=i.m, h=round(i.h, 4), per_cell=i.per_cell)
                      for i in (plan.info(l) for l in range(plan.P))],
           "err_estimate": plan.err_estimate(),
           "stage_avg_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in st.items() if v[1]}}
    plan.destroy()
    return res


def grid_config(A, torch, N=100_000, seed=1):
    """The regularisation grid of the paper's grid search (lambda in {1, 10,
    100, 1000}) on the feature-grouped workload (float32 plan, CG tol 1e-6):
    one shifted-CG solve for all four systems, against the four systems
    solved together by the batched single-shift solver and one after
    another."""
    import workloads
    p = workloads.feature_grouped(N, seed=seed)
    grid = [1.0, 10.0, 100.0, 1000.0]
    X = torch.from_numpy(p.X).cuda()
    y = torch.from_numpy(np.ascontiguousarray(p.y[:, 0])).cuda()
    plan = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, A.ANOVA_FP32_NFFT))
    xs = torch.empty((len(grid), p.N), dtype=torch.float64, device="cuda").T
    A.krr_cg_solve_shifts(plan, y, xs, grid, 1e-6, 5000)  # warm-up (graphs, work space)
    torch.cuda.synchronize()
    t = time.perf_counter()
    info = A.krr_cg_solve_shifts(plan, y, xs, grid, 1e-6, 5000)
    torch.cuda.synchronize()
    t_shift = time.perf_counter() - t
    xb = [torch.empty_like(y) for _ in grid]
    A.krr_cg_solve_batched([plan] * len(grid), [y] * len(grid), xb, grid, 1e-6, 5000)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ib = A.krr_cg_solve_batched([plan] * len(grid), [y] * len(grid), xb, grid, 1e-6, 5000)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    t = time.perf_counter()
    iters_one = []
    for lam, xo in zip(grid, xb):
        iters_one.append(A.krr_cg_solve(plan, y, xo, lam, 1e-6, 5000)[0]["iters"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    diff = max(float(torch.linalg.norm(xs[:, k] - xb[k]) / torch.linalg.norm(xb[k]))
               for k in range(len(grid)))
    plan.destroy()
    return {"workload": f"feature_grouped N={N}, float32 plan, lambda in {{1,10,100,1000}}, "
                        "CG tol 1e-6",
            "shifted_seconds": round(t_shift, 4), "batched_seconds": round(t_batch, 4),
            "sequential_seconds": round(t_seq, 4),
            "speedup_vs_batched": round(t_batch / t_shift, 2),
            "speedup_vs_sequential": round(t_seq / t_shift, 2),
            "shifted_iters": [i["iters"] for i in info],
            "single_iters": iters_one,
            "true_relres": [i["true_relres"] for i in info],
            "max_rel_diff_vs_single": diff}


def regularised_config(A, torch, X, p, a, out, steps):
    """The headline product with the regularised kernel (boundary
    polynomial of order 8, period chosen by the plan) for the same 1e-4
    estimate: matvecs/s and the chosen parameters."""
    plan = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, A.ANOVA_FP32_NFFT,
                                                            target_err=1e-4, reg_q=8))
    ms = time_matvecs(A, torch, plan, a, out, p.beta, steps, 3)
    res = {"workload": "headline points, float32, per-entry estimate <= 1e-4, reg_q = 8",
           "matvecs_per_s": round(1e3 / ms, 2), "ms_per_step": round(ms, 4),
           "params": [dict(M=i.M, n=i.n, m=i.m, h=round(i.h, 4), per_cell=i.per_cell)
                      for i in (plan.info(l) for l in range(plan.P))],
           "err_estimate": plan.err_estimate()}
    plan.destroy()
    return res


def e2e_config(torch):
    """The paper's measured quantities end to end (Sec. 6): fit time (z-score,
    MIS windows, plan, CG to 1e-3), predict time (prediction plan and sum at
    the test points) and test accuracy, on 1e6 training and 1e6 test points
    of labelled synthetic data (nine raw features, three informative)."""
    import workloads
    from paper_2111_10140_amd import krr
    X, y, Z, yz = workloads.labelled(1_000_000, 1_000_000)
    torch.cuda.synchronize()
    t = time.perf_counter()
    m = krr.KernelRidge(sigma=1.0, lam=1.0, tol=1e-3).fit(X, y)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t
    t = time.perf_counter()
    pred = m.predict(Z)
    t_pred = time.perf_counter() - t
    return {"workload": "labelled N=1e6 train + 1e6 test, d=9 raw features, sigma=1, lambda=1, "
                        "float32 plans (1e-4), CG tol 1e-3",
            "fit_seconds": round(t_fit, 3), "predict_seconds": round(t_pred, 3),
            "accuracy": float(np.mean(pred == yz)), "cg_iters": m.fit_info_["iters"],
            "windows": [list(w[0]) for w in m.windows_]}


def serving(args, A):
    """Served KRR solves: closed-loop capacity (every request queued at t=0),
    the same with one request at a time, then Poisson arrivals at
    serve_load x capacity; latency = result time - arrival."""
    import workloads
    from paper_2111_10140_amd.serve import HipExecutor, Server
    R = args.serve_requests
    reqs = workloads.serving_stream(R, rate=1.0, n_hi=args.serve_n_hi)  # unit-rate arrivals
    ex = HipExecutor(A.ANOVA_FP32_NFFT, target_err=1e-4)
    budget = int(args.serve_budget_gb * (1 << 30))
    closed = serve_stream(Server, ex, reqs, [0.0] * R, budget, 64, args.serve_round)
    cap = closed.stats(0.0)["solves_per_s"]
    print(f"# serving: capacity {cap:.2f} solves/s (closed loop, {R} requests)", file=sys.stderr,
          flush=True)
    seq = serve_stream(Server, ex, reqs, [0.0] * R, budget, 1, args.serve_round)
    seq_rate = seq.stats(0.0)["solves_per_s"]
    rate = args.serve_load * cap
    srv = serve_stream(Server, ex, reqs, [r.arrival / rate for r in reqs], budget, 64,
                       args.serve_round)
    st = srv.stats(0.1)
    statuses = {}
    for r in srv.results.values():
        statuses[r.status] = statuses.get(r.status, 0) + 1
    iters = [max(i["iters"] for i in r.info) for r in srv.results.values() if r.info]
    return {
        "workload": f"Poisson stream of {R} KRR solves: N uniform in [1000, {args.serve_n_hi}], "
                    "d in {6,9,12} (consecutive triples), ell uniform in [0.1, 0.4], beta=1, "
                    "1-8 RHS, fp32 NFFT + fp64 CG, tol 1e-6, plan for err<=1e-4",
        "requests": R, "load": args.serve_load, "rate_per_s": round(rate, 3),
        "capacity_solves_per_s": round(cap, 3),
        "one_at_a_time_solves_per_s": round(seq_rate, 3),
        "p50_ms": round(st["p50_s"] * 1e3, 2), "p99_ms": round(st["p99_s"] * 1e3, 2),
        "mean_ms": round(st["mean_s"] * 1e3, 2), "solves_per_s": round(st["solves_per_s"], 3),
        "latency_from": "arrival (queueing, planning, CG, result copy); first 10% excluded",
        "peak_live": st["peak_live"], "budget_gb": args.serve_budget_gb,
        "iters_per_round": args.serve_round,
        "peak_reserved_gb": round(st["peak_reserved_bytes"] / 2**30, 3),
        "statuses": statuses, "errors": error_counts(srv),
        "cg_iters_median": int(np.median(iters)) if iters else None,
    }


def error_counts(srv):
    """Requests that did not end OK, by status and message."""
    out = {}
    for r in srv.results.values():
        if r.status != "OK":
            key = f"{r.status}: {r.error[:160]}" if r.error else r.status
            out[key] = out.get(key, 0) + 1
    return out


SWEEP_LOADS = (0.25, 0.5, 0.75, 0.9, 1.0, 1.2)


def serving_sweep(args, A):
    """Served solves at Poisson arrival rates of SWEEP_LOADS x the measured
    closed-loop capacity, the same `--sweep-requests` requests at every rate
    (N uniform in [1000, --sweep-n-hi], the request mix of the serving
    stream otherwise); p50/p99 over the requests after the first 10%."""
    import workloads
    from paper_2111_10140_amd.serve import HipExecutor, Server
    R = args.sweep_requests
    reqs = workloads.serving_stream(R, rate=1.0, n_hi=args.sweep_n_hi)
    ex = HipExecutor(A.ANOVA_FP32_NFFT, target_err=1e-4)
    budget = int(args.serve_budget_gb * (1 << 30))
    closed = serve_stream(Server, ex, reqs, [0.0] * R, budget, 64, args.serve_round)
    cap = closed.stats(0.0)["solves_per_s"]
    rows = []
    for f in SWEEP_LOADS:
        rate = f * cap
        srv = serve_stream(Server, ex, reqs, [r.arrival / rate for r in reqs], budget, 64,
                           args.serve_round)
        st = srv.stats(0.1)
        ok = sum(1 for r in srv.results.values() if r.status == "OK")
        rows.append({"load": f, "rate_per_s": round(rate, 3),
                     "p50_ms": round(st["p50_s"] * 1e3, 2), "p99_ms": round(st["p99_s"] * 1e3, 2),
                     "mean_ms": round(st["mean_s"] * 1e3, 2),
                     "solves_per_s": round(st["solves_per_s"], 3), "peak_live": st["peak_live"],
                     "ok": ok, "not_ok": error_counts(srv)})
        print(f"# serving sweep: {json.dumps(rows[-1])}", file=sys.stderr, flush=True)
    return {"workload": f"{R} KRR solves per rate: N uniform in [1000, {args.sweep_n_hi}], "
                        "d in {6,9,12}, ell uniform in [0.1, 0.4], beta=1, 1-8 RHS, fp32 NFFT + "
                        "fp64 CG, tol 1e-6, plan for err<=1e-4",
            "requests_per_rate": R, "capacity_solves_per_s": round(cap, 3),
            "latency_from": "arrival (queueing, planning, CG, result copy); first 10% excluded",
            "rates": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4,
                          "copy_probe_bytes_written": b.numel() * 4, "copies": 5}))
        return

    import workloads
    from paper_2111_10140_amd import _lib as A

    A.load()
    torch.cuda.set_device(0)
    p = workloads.headline(args.n)
    N = p.N
    X = torch.from_numpy(p.X).cuda()
    a_np = np.ascontiguousarray(p.alpha[:, 0])
    a = torch.from_numpy(a_np.copy()).cuda()
    out = torch.empty_like(a)

    t0 = time.perf_counter()
    plan = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, A.ANOVA_FP32_NFFT,
                                                            target_err=args.target))
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    infos = [plan.info(l) for l in range(plan.P)]

    ms_eager = time_matvecs(A, torch, plan, a, out, p.beta, max(10, args.steps // 2),
                            args.warmup)
    graph, ms, per_replay, graph_ok = graph_timing(A, torch, plan, a, out, p.beta, args.steps,
                                                   args.warmup)
    cold = cold_timing(torch, graph)
    del graph
    stages = stage_profile(A, torch, plan, a, out, p.beta, max(10, args.steps // 2))
    A.anova_matvec(plan, a, out, p.beta)
    torch.cuda.synchronize()
    gpu_out = out.cpu().numpy()

    G = infos[0].n ** infos[0].d_A
    P = plan.P
    per_launch = {}
    for k, (tot, cnt) in stages.items():
        if cnt:
            # one launch group covers all P windows (combine: the whole product)
            avg_ms = tot / cnt
            b = alg_bytes(k, N, G, 4, P, bool(infos[0].per_cell)) * (1 if k == "combine" else P)
            per_launch[k] = dict(avg_us=avg_ms * 1e3, launches=cnt, alg_bytes=b,
                                 gbs=b / (avg_ms * 1e-3) / 1e9,
                                 hbm_frac=b / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
    W = 2 * infos[0].m
    for k in ("spread", "gather"):
        if k in per_launch:
            f = alg_flops(N, infos[0].d_A, W) * P
            per_launch[k]["alg_flops"] = f
            per_launch[k]["tflops"] = f / (per_launch[k]["avg_us"] * 1e-6) / 1e12
            per_launch[k]["valu_frac"] = per_launch[k]["tflops"] / VALU_FP32_PEAK_TFLOPS
    dom = max(per_launch, key=lambda k: per_launch[k]["avg_us"])
    traffic = measured_traffic(dom)
    count = (f"spread/gather: 2 W^d_A + {C_EVAL} d_A W flop per point and window (W = {W}, "
             f"d_A = {infos[0].d_A}: {2 * W ** infos[0].d_A + C_EVAL * infos[0].d_A * W}); "
             "bytes as alg_bytes in bench.py")
    kernels = {k: {"avg_us": round(v["avg_us"], 3), "tflops": round(v["tflops"], 3),
                   "valu_frac": round(v["valu_frac"], 4), "gbs": round(v["gbs"], 1),
                   "hbm_frac": round(v["hbm_frac"], 4)}
               for k, v in per_launch.items() if "tflops" in v}
    if "tflops" in per_launch[dom]:
        # at m = 3 spread and gather do ~24 flop per algorithmic byte, above
        # the float32 ridge (78.6 TFLOP/s / 8 TB/s ~ 10): the vector ALUs bind
        roof = {"bound": "alu", "kernel": dom, "achieved": round(per_launch[dom]["tflops"], 2),
                "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(per_launch[dom]["valu_frac"], 4),
                "frac_of_packed_fp32_peak": round(per_launch[dom]["tflops"] /
                                                  VALU_FP32_PACKED_PEAK_TFLOPS, 4),
                "traffic": traffic,
                "traffic_source": ("FETCH_SIZE + WRITE_SIZE per launch from the committed "
                                   "counter runs in profiles/headline_pmc_traffic.txt, taken "
                                   "on this kernel source (not measured in this run)")
                if traffic is not None else "none for this kernel source",
                "alg_flops": per_launch[dom]["alg_flops"], "alg_bytes": per_launch[dom]["alg_bytes"],
                "hbm_achieved_gbs": round(per_launch[dom]["gbs"], 1),
                "hbm_frac": round(per_launch[dom]["hbm_frac"], 4),
                "count": count, "kernels": kernels}
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(per_launch[dom]["gbs"], 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(per_launch[dom]["hbm_frac"], 4), "traffic": traffic}
    timing = {"unit": "ms per product", "graph_replays": args.steps,
              "median": round(pct(per_replay, 50), 4), "p10": round(pct(per_replay, 10), 4),
              "p90": round(pct(per_replay, 90), 4),
              "matvecs_per_s_at_median": round(1e3 / pct(per_replay, 50), 2),
              "replays_equal_eager_product": bool(graph_ok),
              "eager_mean": round(ms_eager, 4),
              "cold_cache": {"reps": len(cold), "median": round(pct(cold, 50), 4),
                             "p10": round(pct(cold, 10), 4), "p90": round(pct(cold, 90), 4),
                             "matvecs_per_s": round(1e3 / pct(cold, 50), 2),
                             "flush": "512 MiB written before each replay"}}

    cg_iter = cg_iteration_timing(A, torch, plan, p, pct(per_replay, 50))
    print(f"# cg iteration: {json.dumps(cg_iter)}", file=sys.stderr, flush=True)

    fixed = None
    if not args.skip_fixed:
        plan_f = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, A.ANOVA_FP32_NFFT, M=64,
                                                                  m=6, n=128))
        ms_f = time_matvecs(A, torch, plan_f, a, out, p.beta, max(10, args.steps // 4), 3)
        st_f = stage_profile(A, torch, plan_f, a, out, p.beta, 10)
        A.anova_matvec(plan_f, a, out, p.beta)
        torch.cuda.synchronize()
        fixed_out = out.cpu().numpy()
        fixed = {"M": 64, "m": 6, "n": 128, "ms_per_step": round(ms_f, 4),
                 "matvecs_per_s": round(1e3 / ms_f, 2),
                 "stage_avg_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in st_f.items() if v[1]}}
        plan_f.destroy()

    cpu = None
    if not args.skip_cpu:
        import oracle
        rng = np.random.default_rng(7)
        # the probe holds enough rows to occupy every host thread
        probe = rng.choice(N, 256, replace=False)
        t1 = time.perf_counter()
        oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, a_np, rows=probe)
        per_row = (time.perf_counter() - t1) / 256
        S = int(max(64, min(32768, args.cpu_seconds / max(per_row, 1e-6))))
        rows = rng.choice(N, S, replace=False)
        t1 = time.perf_counter()
        ref, threads = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, a_np, rows=rows,
                                                  return_threads=True)
        t_cpu = time.perf_counter() - t1
        err = float(np.max(np.abs(gpu_out[rows] - ref)) / np.abs(a_np).sum())
        rel = float(np.max(np.abs(gpu_out[rows] - ref)) / np.max(np.abs(ref)))
        # one thread, on a sample sized for about a third of the time
        S1 = int(max(16, min(S, S / max(threads, 1) / 3)))
        oracle.direct.set_threads(1)
        t1 = time.perf_counter()
        oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, a_np, rows=rows[:S1])
        t_one = time.perf_counter() - t1
        oracle.direct.set_threads(threads)
        cpu = {"value": S / (t_cpu * N), "unit": "matvecs/s", "cores": int(threads),
               "kind": "oracle",
               "sample": f"{S} random rows of the N={N} direct float64 sum ({t_cpu:.1f} s), "
                         f"extrapolated as rows/(time*N)",
               "single_core_value": S1 / (t_one * N),
               "single_core_sample": f"{S1} of those rows on one thread ({t_one:.1f} s)"}
        if fixed is not None:
            fixed["err_sampled_rows"] = float(np.max(np.abs(fixed_out[rows] - ref)) / np.abs(a_np).sum())
    else:
        err = rel = None

    # the measured parameter choice on the same points
    tuned = None
    if not args.skip_tuned:
        t0 = time.perf_counter()
        plan_t = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, A.ANOVA_FP32_NFFT,
                                                                  target_err=args.target, tune=1))
        torch.cuda.synchronize()
        tuned = {"plan_seconds": round(time.perf_counter() - t0, 3),
                 "params": [dict(M=i.M, n=i.n, m=i.m, per_cell=i.per_cell)
                            for i in (plan_t.info(l) for l in range(plan_t.P))],
                 "err_estimate": plan_t.err_estimate()}
        tuned["matvecs_per_s"] = round(1e3 / time_matvecs(A, torch, plan_t, a, out, p.beta,
                                                          args.steps, args.warmup), 2)
        plan_t.destroy()
        print(f"# measured parameter choice: {json.dumps(tuned)}", file=sys.stderr, flush=True)

    split = None
    if not args.skip_fixed:
        split = precision_split(A, torch, X, p, a, out, plan, args.target)
        print(f"# precision split: {json.dumps(split)}", file=sys.stderr, flush=True)
    batched = None
    if not args.skip_batched:
        batched = batched_config(A, torch)
        print(f"# batched: {json.dumps(batched)}", file=sys.stderr, flush=True)
    large = None if args.skip_large else large_config(A, torch)
    gridded = None
    if not args.skip_grid:
        gridded = [grid_config(A, torch), grid_config(A, torch, N, 2)]
        print(f"# grid: {json.dumps(gridded)}", file=sys.stderr, flush=True)
    regd = None
    if not args.skip_reg:
        regd = regularised_config(A, torch, X, p, a, out, max(10, args.steps // 2))
        print(f"# regularised: {json.dumps(regd)}", file=sys.stderr, flush=True)
    e2e = None
    if not args.skip_e2e:
        e2e = e2e_config(torch)
        print(f"# end to end: {json.dumps(e2e)}", file=sys.stderr, flush=True)
    predicted = None
    if not args.skip_predict:
        predicted = predict_config(A, torch, max(10, args.steps // 2))
        print(f"# predict: {json.dumps(predicted)}", file=sys.stderr, flush=True)
    served = None if args.skip_serve else serving(args, A)
    if served is not None and args.sweep_requests > 0:
        served["rate_sweep"] = serving_sweep(args, A)

    res = {
        "metric": "ANOVA matvecs/s N=1M,3 windows d_A=3 (err<=1e-4)",
        "value": round(1e3 / ms, 2), "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded uniform points, stand-in for the paper's datasets)",
        "config": {"workload": f"feature_grouped N={N} d=9 windows 3x(d_A=3) ell=0.2 beta=1",
                   "precision": "fp32 spread/FFT/gather, fp64 accumulation",
                   "params": [dict(M=i.M, n=i.n, m=i.m, h=round(i.h, 4)) for i in infos],
                   "err_estimate": plan.err_estimate(), "err_sampled_rows": err,
                   "rel_err_sampled_rows": rel, "plan_seconds": round(plan_s, 3)},
        "roofline": roof,
        "timing": timing,
        "cg_iteration": cg_iter,
        "stages_per_launch": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                                  for kk, vv in v.items()} for k, v in per_launch.items()},
        "fixed_params": fixed,
        "tuned": tuned,
        "precision_split": split,
        "batched": batched,
        "large": large,
        "predict": predicted,
        "lambda_grid": gridded,
        "regularised": regd,
        "end_to_end": e2e,
        "serving": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))
    plan.destroy()


if __name__ == "__main__":
    main()
