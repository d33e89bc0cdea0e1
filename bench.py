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
the GPU result.
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
    return ap.parse_args()


def alg_bytes(stage: str, N: int, G: int, elem: int, P: int = 3) -> float:
    """Algorithmic HBM bytes of a stage for one window (the combine: for the
    whole product).  elem = 4 B (float32 NFFT) or 8 B (float64):
    permute : permutation index 4 B, the gathered float64 coefficient 8 B and
              the sorted coefficient written (elem) per point;
    spread  : node record (16 B f32 / 32 B f64) + sorted coefficient per
              point, one write of each grid value;
    tile_sum, fold : one write of each grid value (the tile regions they read
              are traffic of this implementation, not of the method);
    convolve (one axis pass): one read and one write of the grid;
    gather  : node record + one value written per point, one read of each
              grid value;
    combine (all windows): alpha read and output write 16 B per point, plus
              the inverse permutation and the window's value per point and
              window."""
    node = 16 if elem == 4 else 32
    if stage == "permute":
        return N * (4 + 8 + elem)
    if stage == "spread":
        return N * (node + elem) + G * elem
    if stage == "gather":
        return N * (node + elem) + G * elem
    if stage == "combine":
        return N * (16 + P * (4 + elem))
    if stage == "convolve":
        return 2.0 * G * elem
    return float(G * elem)  # tile_sum, fold


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


def stage_profile(A, torch, plan, a, out, beta, steps):
    plan.set_timing(True)
    for _ in range(steps):
        A.anova_matvec(plan, a, out, beta)
    torch.cuda.synchronize()
    t = plan.stage_times()
    plan.set_timing(False)
    return t


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

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

    ms = time_matvecs(A, torch, plan, a, out, p.beta, args.steps, args.warmup)
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
            b = alg_bytes(k, N, G, 4, P) * (1 if k == "combine" else P)
            per_launch[k] = dict(avg_us=avg_ms * 1e3, launches=cnt, alg_bytes=b,
                                 gbs=b / (avg_ms * 1e-3) / 1e9)
    dom = max(per_launch, key=lambda k: per_launch[k]["avg_us"])
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(per_launch[dom]["gbs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(per_launch[dom]["gbs"] / HBM_PEAK_GBS, 4), "traffic": None}

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
        probe = rng.choice(N, 8, replace=False)
        t1 = time.perf_counter()
        oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, a_np, rows=probe)
        per_row = (time.perf_counter() - t1) / 8
        S = int(max(16, min(4096, args.cpu_seconds / max(per_row, 1e-6))))
        rows = rng.choice(N, S, replace=False)
        t1 = time.perf_counter()
        ref, threads = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, a_np, rows=rows,
                                                  return_threads=True)
        t_cpu = time.perf_counter() - t1
        err = float(np.max(np.abs(gpu_out[rows] - ref)) / np.abs(a_np).sum())
        cpu = {"value": S / (t_cpu * N), "unit": "matvecs/s", "cores": int(threads),
               "kind": "oracle",
               "sample": f"{S} random rows of the N={N} direct float64 sum ({t_cpu:.1f} s), "
                         f"extrapolated as rows/(time*N)"}
        if fixed is not None:
            fixed["err_sampled_rows"] = float(np.max(np.abs(fixed_out[rows] - ref)) / np.abs(a_np).sum())
    else:
        err = None

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
                   "plan_seconds": round(plan_s, 3)},
        "roofline": roof,
        "stages_per_launch": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                                  for kk, vv in v.items()} for k, v in per_launch.items()},
        "fixed_params": fixed,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))
    plan.destroy()


if __name__ == "__main__":
    main()
