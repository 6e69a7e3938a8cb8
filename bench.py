"""Benchmark: factorise + solve throughput of the regularised Newton systems on one GPU.

One step = one IPM-like iteration on the staircase augmented system (20000 x 40000,
40 periods): a fresh Theta (already resident in HBM), the numeric factorisation, and the
predictor and one corrector solve (Section 4.7: 1 + k directions with k >= 1), each refined
in FP64 to the target backward error.  Prints one JSON line.

The roofline object describes the kernel kind that takes the most time in a step: its
launches inside the timed region are bracketed with HIP events on the library's stream and
its algorithmic work per launch comes from the symbolic structure.
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

from paper_2508_04370_amd import workloads as W  # noqa: E402

PEAK_FP64 = 78.6e12   # MI355X dense FP64, matrix and vector (FLOP/s)
PEAK_FP32 = 157.3e12  # dense FP32 matrix (FLOP/s)
PEAK_HBM = 8.0e12     # HBM3E (bytes/s)

# which resource bounds each kernel kind: the dependent FP64 steps of the pivot chains (small
# fronts, windows), HBM for assembly, finalize and the solves, the matrix units for the trailing
# update
KIND_BOUND = {0: "alu", 1: "hbm", 2: "alu", 3: "mfma", 4: "hbm", 5: "hbm", 6: "hbm"}


def kernel_source_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_2508_04370_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of kernel on workload from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading on a plain copy of
    known size), or None when there is none or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic: "):
            rec = json.loads(line[len("traffic: "):])
    if not rec or rec.get("kernels_sha") != kernel_source_sha():
        return None
    return rec["fetch_kib_per_dispatch"] * 1024.0 / rec["copy_fetch_factor"] + \
        rec["write_kib_per_dispatch"] * 1024.0 / rec["copy_write_factor"]


def copy_calibration(nbytes):
    """One plain device copy of nbytes (reads nbytes, writes nbytes): the reference dispatch
    for the HBM counters."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "kernels_sha": kernel_source_sha()}))


def make_workload(name):
    if name == "as_staircase":
        return W.as_staircase(), dict()
    if name == "ne_random":
        return W.ne_random(), dict()
    if name == "ne_grid":
        lp = W.ne_grid(nrhs=8)
        return lp, dict(ordering=2, grid=lp["grid"])
    if name == "ne_grid_small":
        lp = W.ne_grid(24, 24, 20, nrhs=8)
        return lp, dict(ordering=2, grid=lp["grid"])
    if name.startswith("ne_dense_front"):  # ne_dense_front or ne_dense_front_<f>
        f = int(name.split("_")[-1]) if name[-1].isdigit() else 4096
        return W.ne_dense_front(f), dict(ordering=0)
    if name in ("as_batch", "as_batch_small"):
        lps = W.as_batch(512 if name == "as_batch" else 32)
        cat = W.concat_systems(lps)
        cat["systems"] = lps
        return cat, dict(systems=lps, ordering=0)
    if name == "as_dense_cols":
        lp = W.as_dense_cols()
        return lp, dict(ordering=2, grid=lp["grid"])
    if name == "as_staircase_qp":  # the staircase with a Hessian on half of its columns
        return W.with_hessian(W.as_staircase(), seed=1, frac=0.5, per_row=3, window=50), dict()
    raise SystemExit(f"unknown workload {name}")


def thetas(lp, k, seed):
    if "systems" in lp:  # batch: system s, iteration k draws from seed [4, s, k]
        return np.concatenate([W.as_batch_theta(q, s, k) for s, q in enumerate(lp["systems"])])
    if lp["name"].startswith("ne_dense_front"):
        return W.log_uniform(W.rng(seed, 1000 + k), 1e-2, 1e2, lp["n"])
    g = W.rng(seed, 1000 + k)
    lo, hi = (1e-10, 1e10) if lp["mode"] == W.AS else (1e-6, 1e6)
    return W.log_uniform(g, lo, hi, lp["n"])


def run_gpu(lp, opts, prec, steps, warmup, nsolves, graph):
    import torch
    from paper_2508_04370_amd import qdmf as Q
    dev = "cuda:0"
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    s = Q.Solver(lp, device=0, stream=stream.cuda_stream, **opts)
    sym = s.sym
    nth = warmup + steps + 8
    TH = [torch.from_numpy(thetas(lp, k, 7)).to(dev) for k in range(nth)]
    if "systems" in lp:  # batch: predictor right-hand sides of iteration 0, seed [4, s, 0, 0]
        rs = [W.as_batch_rhs(q, s, 0, 0) for s, q in enumerate(lp["systems"])]
        lp["r7"] = np.concatenate([r[0] for r in rs]).reshape(-1, 1)
        lp["r1"] = np.concatenate([r[1] for r in rs]).reshape(-1, 1)
    r1 = Q.to_device_colmajor(lp["r1"], dev)
    r7 = Q.to_device_colmajor(lp["r7"], dev) if lp["mode"] == W.AS else None
    nrhs = r1.shape[1]
    dx = torch.empty((nrhs, lp["n"]), dtype=torch.float64, device=dev).T
    dy = torch.empty((nrhs, lp["m"]), dtype=torch.float64, device=dev).T

    def one(k):
        s.factorise(TH[k % nth], lp["rho"], lp["delta"], prec)
        for _ in range(nsolves):
            s.solve(r7, r1, dx, dy)

    for k in range(warmup):
        one(k)
    stream.synchronize()
    # the dominant kernel kind: one profiled step per kind
    per_kind = {}
    for kind in range(7):
        Q.qdmf_profile_kind(s.h, kind)
        one(warmup + steps + (kind % 8))
        per_kind[kind] = Q.qdmf_profile_read(s.h)
    Q.qdmf_profile_kind(s.h, -1)
    dom = max(per_kind, key=lambda k: per_kind[k]["total_ms"])
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(kind):
        Q.qdmf_profile_kind(s.h, kind)
        per, steps_taken, berrs = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(warmup, warmup + steps):
            e0.record(stream)
            one(k)
            e1.record(stream)
            e1.synchronize()
            per.append(e0.elapsed_time(e1))
            ss = s.solve_stats(nrhs)
            steps_taken.append(int(ss["max_steps"]))
            berrs.append(float(ss["berr_nw"]))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = Q.qdmf_profile_read(s.h)
        Q.qdmf_profile_kind(s.h, -1)
        return per, steps_taken, berrs, prof, wall

    # the timed region: K steps; then the same K steps again with every launch of the
    # dominant kind bracketed by HIP events on the library's stream (the brackets add a
    # little time per launch, so they stay out of the step time)
    per, steps_taken, berrs, _, wall = timed(-1)
    per_p, _, _, prof, _ = timed(dom)
    fs = s.factor_stats()
    if s.systems is not None:  # the worst system of the batch
        bs = s.batch_stats(nrhs)
        fs["systems"] = len(s.systems)
        fs["worst_system_berr_nw"] = float(bs["berr_nw"].max())
        fs["inertia_ok_all_systems"] = bool(all(tuple(bs["inertia"][q][:2]) == (sy_["n"], sy_["m"])
                                               for q, sy_ in enumerate(s.systems)))
    out = dict(ms=per, wall=wall, ms_profiled=per_p, sym=sym, steps=steps_taken, berr=berrs, fstats=fs, dom=dom, prof=prof,
               per_kind={Q.KERNEL_KIND_NAMES[k]: round(v["total_ms"], 3) for k, v in per_kind.items()})
    if graph:  # the same step captured once as a HIP graph and replayed with Theta refreshed
        th = torch.empty(lp["n"], dtype=torch.float64, device=dev)
        th.copy_(TH[0])
        Q.qdmf_graph_capture(s.h, th, lp["rho"], lp["delta"], prec, nsolves, nrhs, r7, r1, dx, dy)
        gms = []
        for k in range(warmup + steps):
            e0.record(stream)
            th.copy_(TH[k % nth])
            Q.qdmf_graph_launch(s.h)
            e1.record(stream)
            e1.synchronize()
            if k >= warmup:
                gms.append(e0.elapsed_time(e1))
        out["graph_ms"] = gms
        out["graph_berr"] = float(s.solve_stats(nrhs)["berr_nw"])
    s.close()
    return out


def cpu_baseline(lp):
    """The oracle (plain C, one thread) on the same workload: factorise + one solve."""
    from oracle import oracle as O
    O.build(force=False)
    S = O.Sym(lp)
    th = thetas(lp, 0, 7)
    t0 = time.perf_counter()
    F = O.Num(S, lp["val"], th, lp["rho"], lp["delta"])
    r7 = lp["r7"] if lp["mode"] == W.AS else None
    res = F.solve(r7, lp["r1"])
    t = time.perf_counter() - t0
    nrhs = lp["r1"].shape[1]
    flops = S.flops + (1 + float(np.mean(res["steps"]))) * nrhs * (4.0 * (S.nnzL - S.N) + S.N)
    return dict(value=round(flops / t / 1e9, 4), unit="GFLOP/s", cores=1, kind="oracle",
                sample="one factorise + one solve with refinement of the full workload on one host "
                       "core (ordering and symbolic analysis excluded)",
                seconds=round(t, 3), ms_per_factorise_solve=round(t * 1e3, 1))


def run_ipm(lp, opts, prec, args):
    """The interior point driver (qdmf_ipm_solve) on the LP min c^T x, A x = b, l <= x <= u with
    the workload's A and b, c, l, u from workloads.bounded_lp (a fraction --ipm-upper of the
    columns with a finite upper bound); one untimed run (warm-up), then the timed runs;
    value = milliseconds per IPM iteration."""
    import torch
    from paper_2508_04370_amd import qdmf as Q
    lpf, b, c, l, u = W.bounded_lp(lp, seed=7, upper=args.ipm_upper)
    dev = "cuda:0"
    s = Q.Solver(lpf, device=0, **{k: v for k, v in opts.items() if k in ("ordering", "grid")})
    bd, cd, ld, ud = (torch.from_numpy(v).to(dev) for v in (b, c, l, u))
    x = torch.empty(lpf["n"], dtype=torch.float64, device=dev)
    zl = torch.empty(lpf["n"], dtype=torch.float64, device=dev)
    zu = torch.empty(lpf["n"], dtype=torch.float64, device=dev)
    y = torch.empty(lpf["m"], dtype=torch.float64, device=dev)
    opt = Q.qdmf_ipm_default_options(prec=prec)
    runs = []
    for k in range(args.warmup + args.steps):
        info, hist = Q.qdmf_ipm_solve(s.h, bd, cd, x, y, zl, opt, l=ld, u=ud, zu=zu)
        print(f"[bench] ipm run {k}: status {info['status']} iters {info['iters']} {info['ms']:.1f} ms",
              file=sys.stderr, flush=True)
        if k >= args.warmup:
            runs.append(info)
    ms_it = [r["ms"] / max(1, r["iters"]) for r in runs]
    last = runs[-1]
    out = {"metric": "interior point iteration time (factorise, predictor, correctors, vector work)",
           "value": round(float(np.median(ms_it)), 4), "unit": "ms/iteration", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if prec == 0 else "f64+f32", "data": "synthetic",
           "config": {"workload": lp["name"] + "_bounded_lp", "m": lpf["m"], "n": lpf["n"], "mode": "AS",
                      "upper_bounded_fraction": args.ipm_upper, "precision": args.prec},
           "ipm": {"status": last["status"], "iterations": last["iters"], "correctors": last["correctors"],
                   "primal_obj": last["primal_obj"], "dual_obj": last["dual_obj"], "pinf": last["pinf"],
                   "dinf": last["dinf"], "ms_total": round(last["ms"], 3)}}
    s.close()
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="as_staircase",
                    help="as_staircase | ne_random | ne_grid | ne_grid_small | as_batch | as_batch_small | "
                         "as_dense_cols | ne_dense_front[_<f>] | as_staircase_qp")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--nsolves", type=int, default=2)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ipm", action="store_true",
                    help="instead: the interior point driver on a feasible LP over the workload's A "
                         "(one JSON line, ms per IPM iteration)")
    ap.add_argument("--ipm-upper", type=float, default=0.5,
                    help="--ipm: fraction of the columns with a finite upper bound")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one plain device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU (--gpus 1): the library factorises on one device; "
              "across several, the elimination tree's subtrees would go to different GPUs and only the "
              "subtree roots' contribution blocks would travel", file=sys.stderr)
        sys.exit(2)
    lp, opts = make_workload(args.workload)
    prec = 1 if args.prec == "mixed" else 0
    if args.ipm:
        run_ipm(lp, opts, prec, args)
        return
    print(f"[bench] workload={lp['name']} prec={args.prec} steps={args.steps} warmup={args.warmup}",
          file=sys.stderr, flush=True)
    r = run_gpu(lp, opts, prec, args.steps, args.warmup, args.nsolves, not args.no_graph)
    sym = r["sym"]
    ms = r["wall"] * 1e3 / args.steps  # K steps between two device synchronisations
    nrhs = lp["r1"].shape[1]
    nnz_a = int(lp["colptr"][-1])
    # algorithmic work of one step (exact structure of L): factorisation, every solve pass
    # (the first solve and each refinement step) and each residual
    solve_passes = args.nsolves * (1 + float(np.mean(r["steps"])))
    flops = sym["flops_fact"] + solve_passes * nrhs * (sym["flops_solve"] + 4.0 * nnz_a + 2.0 * sym["N"])
    value = flops / (ms * 1e-3) / 1e9
    from paper_2508_04370_amd import qdmf as Q
    dom = r["dom"]
    pr = r["prof"]
    avg_ms = pr["total_ms"] / max(1, pr["launches"])
    bound = KIND_BOUND[dom]
    if bound == "hbm":
        per_launch = pr["bytes"] / max(1, pr["launches"])
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        peak, unit = PEAK_HBM / 1e9, "GB/s"
    else:
        per_launch = pr["flops"] / max(1, pr["launches"])
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        peak = (PEAK_FP32 if (bound == "mfma" and prec == 1) else PEAK_FP64) / 1e12
        unit = "TFLOP/s"
    out = {
        "metric": "factorise+solve GFLOP/s (ms per IPM iteration alongside)",
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": lp["name"], "m": lp["m"], "n": lp["n"], "mode": "AS" if lp["mode"] else "NE",
                   "nrhs": nrhs, "solves_per_step": args.nsolves, "precision": args.prec,
                   "N": sym["N"], "nsuper": sym["nsuper"], "nlevels": sym["nlevels"],
                   "max_front": sym["max_front"], "flops_fact": sym["flops_fact"],
                   "nnz_l": sym["nnz_l"]},
        "roofline": {"bound": bound, "kernel": Q.KERNEL_KIND_NAMES[dom], "achieved": round(achieved, 6),
                     "peak": peak, "unit": unit, "frac": round(achieved / peak, 6),
                     "traffic": measured_traffic(Q.KERNEL_KIND_NAMES[dom], args.workload),
                     "algorithmic_bytes_per_launch": round(pr["bytes"] / max(1, pr["launches"]), 1),
                     "launches": pr["launches"], "avg_launch_us": round(avg_ms * 1e3, 3),
                     "work_per_launch": round(per_launch, 1),
                     "ms_per_step_with_brackets": round(float(np.median(r["ms_profiled"])), 4)},
        "kernel_ms_per_step_by_kind": r["per_kind"],
        "berr_nw_max": max(r["berr"]),
        "refine_steps_mean": float(np.mean(r["steps"])),
        "ms_median": round(float(np.median(r["ms"])), 4), "ms_min": round(min(r["ms"]), 4),
        "ms_max": round(max(r["ms"]), 4),
        "inertia": [r["fstats"]["nneg"], r["fstats"]["npos"]],
        "batch": {k: r["fstats"][k] for k in ("systems", "worst_system_berr_nw", "inertia_ok_all_systems")}
        if "systems" in r["fstats"] else None,
    }
    if "graph_ms" in r:
        gms = float(np.median(r["graph_ms"]))
        out["graph"] = {"ms_per_step": round(gms, 4), "value": round(flops / (gms * 1e-3) / 1e9, 3),
                        "berr_nw": r["graph_berr"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lp)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
