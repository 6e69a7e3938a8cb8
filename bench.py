"""Benchmark: factorise + solve of the regularised Newton systems on one GPU, FP64 and mixed
precision in the same run.

Default workload: the dense-column augmented system (rows on an 80 x 50 x 50 grid, m = 200000,
n = 400000 with 20 dense columns at 50 % density, N = 600000; geometric nested dissection),
the largest single-GPU configuration of the build.  One step = one IPM-like iteration: a fresh
Theta (already resident in HBM), the numeric factorisation, and the predictor and one
corrector solve (Section 4.7: 1 + k directions with k >= 1), each refined in FP64 to its
backward-error target (1e-12 FP64 path, 1e-10 mixed path).  Prints one JSON line: value = the
FP64 path's algorithmic GFLOP/s, with the mixed path's time, accuracy and speedup beside it.
The mixed path runs with the workload's tuned options; when those leave no front with FP32
products, `mixed_fp32_products` also times the mixed path with them on (f_mix = 1024).

The roofline object describes the kernel kind that takes the most time in an FP64 step: its
launches inside the timed region are bracketed with HIP events on the library's stream and its
algorithmic work per launch comes from the symbolic structure.  `rooflines` gives the same for
the trailing update (matrix cores), the solves and the assembly (HBM).
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
KIND_BOUND = {0: "alu", 1: "hbm", 2: "alu", 3: "mfma", 4: "hbm", 5: "hbm", 6: "hbm", 7: "mfma"}


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
    try:
        return W.named_workload(name)
    except ValueError as e:
        raise SystemExit(str(e))


def thetas(lp, k, seed):
    return W.iteration_theta(lp, k, seed)


PRECS = {"fp64": 0, "mixed": 1}
KINDS = range(8)


def tuned_options(workload):
    """Launch parameters the autotuner chose for this workload (tuning/<workload>.json in the
    package), or {} when there is none."""
    path = os.path.join(ROOT, "paper_2508_04370_amd", "tuning", f"{workload}.json")
    if not os.path.exists(path):
        return {}, None
    rec = json.load(open(path))
    return dict(rec["options"]), os.path.relpath(path, ROOT)


def run_gpu(lp, opts, precs, steps, warmup, nsolves, graph):
    """Times the same K steps for each precision on one analysed handle."""
    import torch
    from paper_2508_04370_amd import qdmf as Q
    dev = "cuda:0"
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    t0 = time.perf_counter()
    s = Q.Solver(lp, device=0, stream=stream.cuda_stream, **opts)
    analyse_s = time.perf_counter() - t0
    sym = s.sym
    nth = warmup + steps + 8
    TH = [torch.from_numpy(thetas(lp, k, 7)).to(dev) for k in range(nth)]
    if "systems" in lp:  # batch: predictor right-hand sides of iteration 0, seed [4, s, 0, 0]
        rs = [W.as_batch_rhs(q, s_, 0, 0) for s_, q in enumerate(lp["systems"])]
        lp["r7"] = np.concatenate([r[0] for r in rs]).reshape(-1, 1)
        lp["r1"] = np.concatenate([r[1] for r in rs]).reshape(-1, 1)
    r1 = Q.to_device_colmajor(lp["r1"], dev)
    r7 = Q.to_device_colmajor(lp["r7"], dev) if lp["mode"] == W.AS else None
    nrhs = r1.shape[1]
    dx = torch.empty((nrhs, lp["n"]), dtype=torch.float64, device=dev).T
    dy = torch.empty((nrhs, lp["m"]), dtype=torch.float64, device=dev).T
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    results = {}
    for pname in precs:
        prec = PRECS[pname]

        def one(k):
            s.factorise(TH[k % nth], lp["rho"], lp["delta"], prec)
            for _ in range(nsolves):
                s.solve(r7, r1, dx, dy)

        print(f"[bench] {pname}: warm-up", file=sys.stderr, flush=True)
        for k in range(warmup):
            one(k)
        stream.synchronize()
        # time per kernel kind: one profiled step per kind
        per_kind = {}
        for kind in KINDS:
            Q.qdmf_profile_kind(s.h, kind)
            one(warmup + steps + (kind % 8))
            per_kind[kind] = Q.qdmf_profile_read(s.h)
        Q.qdmf_profile_kind(s.h, -1)
        dom = max(per_kind, key=lambda k: per_kind[k]["total_ms"])

        def timed(kind):
            Q.qdmf_profile_kind(s.h, kind)
            per, steps_taken, berrs = [], [], []
            torch.cuda.synchronize()
            t_0 = time.perf_counter()
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
            wall = time.perf_counter() - t_0
            prof = Q.qdmf_profile_read(s.h)
            Q.qdmf_profile_kind(s.h, -1)
            return per, steps_taken, berrs, prof, wall

        # the timed region: K steps; then the same K steps again with every launch of the
        # dominant kind bracketed by HIP events on the library's stream (the brackets add a
        # little time per launch, so they stay out of the step time)
        print(f"[bench] {pname}: timed steps", file=sys.stderr, flush=True)
        per, steps_taken, berrs, _, wall = timed(-1)
        per_p, _, _, prof, _ = timed(dom)
        fs = s.factor_stats()
        if s.systems is not None:  # the worst system of the batch
            bs = s.batch_stats(nrhs)
            fs["systems"] = len(s.systems)
            fs["worst_system_berr_nw"] = float(bs["berr_nw"].max())
            fs["inertia_ok_all_systems"] = bool(all(tuple(bs["inertia"][q][:2]) == (sy_["n"], sy_["m"])
                                                   for q, sy_ in enumerate(s.systems)))
        out = dict(ms=per, wall=wall, ms_profiled=per_p, steps=steps_taken, berr=berrs, fstats=fs, dom=dom,
                   prof=prof, per_kind=per_kind)
        if graph:  # the same step captured once as a HIP graph and replayed with Theta refreshed
            print(f"[bench] {pname}: graph", file=sys.stderr, flush=True)
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
        results[pname] = out
    s.close()
    return results, sym, analyse_s


def host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(workload):
    """The oracle (plain C, one thread) timed on this host over a bounded sample of the
    workload: a smaller instance of the same generator, factorised in matched mode (the
    oracle takes the library's ordering as data, so both factor the same structure)."""
    from oracle import oracle as O
    from paper_2508_04370_amd import qdmf as Q
    O.build(force=False)
    if workload == "as_dense_cols":
        lp = W.as_dense_cols(40, 25, 25)
        opts = dict(ordering=Q.QDMF_ORDER_GRID_ND, grid=lp["grid"])
        sample = ("as_dense_cols 40x25x25 (the same generator on a 40 x 25 x 25 row grid: m = 25000, "
                  "n = 50000 with 20 dense columns, N = 75000): one factorise + one refined solve")
    else:
        lp, opts = make_workload(workload)
        if "systems" in lp:
            lp, opts = lp["systems"][0], dict(ordering=0)
            sample = "the first system of the batch: one factorise + one refined solve"
        else:
            sample = "the full workload: one factorise + one refined solve"
    s = Q.Solver(lp, device=-1, **{k: v for k, v in opts.items() if k != "systems"})
    perm = np.asarray(s.sym["perm"]).copy()
    s.close()
    S = O.Sym(lp, perm)
    th = thetas(lp, 0, 7)
    t0 = time.perf_counter()
    F = O.Num(S, lp["val"], th, lp["rho"], lp["delta"])
    r7 = lp["r7"] if lp["mode"] == W.AS else None
    res = F.solve(r7, lp["r1"])
    t = time.perf_counter() - t0
    nrhs = lp["r1"].shape[1]
    flops = S.flops + (1 + float(np.mean(res["steps"]))) * nrhs * (4.0 * (S.nnzL - S.N) + S.N)
    model, ncpu, avail = host_cpu()
    return dict(value=round(flops / t / 1e9, 4), unit="GFLOP/s", cores=1, kind="oracle", sample=sample,
                seconds=round(t, 3), berr_nw=float(np.max(res["berr_nw"])), ordering="library's (matched mode)",
                cpu_model=model, host_cpus=ncpu, host_cpus_available=avail)


def roofline_of(kind, pr, prec, Q):
    bound = KIND_BOUND[kind]
    launches = max(1, pr["launches"])
    avg_ms = pr["total_ms"] / launches
    if bound == "hbm":
        per_launch = pr["bytes"] / launches
        achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
        peak, unit = PEAK_HBM / 1e9, "GB/s"
    else:
        per_launch = pr["flops"] / launches
        achieved = per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
        peak = (PEAK_FP32 if (bound == "mfma" and prec == 1) else PEAK_FP64) / 1e12
        unit = "TFLOP/s"
    return {"bound": bound, "kernel": Q.KERNEL_KIND_NAMES[kind], "achieved": round(achieved, 6), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 6), "launches": pr["launches"],
            "avg_launch_us": round(avg_ms * 1e3, 3), "work_per_launch": round(per_launch, 1),
            "algorithmic_bytes_per_launch": round(pr["bytes"] / launches, 1)}


def run_c0(args):
    """Dense-front sweep: one front of order f with p pivots (p = f: a single supernode; p < f:
    the front plus its dense parent of order f - p + 1), FP64 and mixed; one JSON line per
    (f, p) with the factorisation's GFLOP/s (work from the exact structure) and the trailing
    update's TFLOP/s against the matrix-core peak."""
    import torch
    from paper_2508_04370_amd import qdmf as Q
    dev = "cuda:0"
    sizes = [int(v) for v in args.c0_sizes.split(",")]
    for f in sizes:
        for frac in (4, 2, 1):
            p = f // frac
            lp, perm = W.dense_front_system(f, p)
            extra = json.loads(args.opts) if args.opts else {}
            s = Q.Solver(lp, device=0, perm=perm, amalgamate=0, **extra)
            th = torch.from_numpy(lp["theta"]).to(dev)
            line = {"workload": f"dense_front_{f}_{p}", "f": f, "p": p, "N": s.N,
                    "flops_fact": s.sym["flops_fact"], "nsuper": s.sym["nsuper"]}
            for pname, prec in PRECS.items():
                for _ in range(args.warmup):
                    s.factorise(th, lp["rho"], lp["delta"], prec)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.steps):
                    s.factorise(th, lp["rho"], lp["delta"], prec)
                e1.record()
                e1.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                kinds = {}
                for kind in KINDS:
                    Q.qdmf_profile_kind(s.h, kind)
                    s.factorise(th, lp["rho"], lp["delta"], prec)
                    r = Q.qdmf_profile_read(s.h)
                    if r["launches"]:
                        kinds[Q.KERNEL_KIND_NAMES[kind]] = {
                            "ms": round(r["total_ms"], 3), "launches": r["launches"],
                            "tflops": round(r["flops"] / (r["total_ms"] * 1e-3) / 1e12, 2) if r["total_ms"] else 0.0}
                Q.qdmf_profile_kind(s.h, -1)
                upd = [kinds[k] for k in ("k_syrk", "k_syrk128") if k in kinds]
                upd_ms = sum(u["ms"] for u in upd)
                upd_fl = sum(u["tflops"] * u["ms"] for u in upd)
                peak = (PEAK_FP32 if prec == 1 else PEAK_FP64) / 1e12
                line[pname] = {"ms_factorise": round(ms, 3),
                               "gflops_factorise": round(s.sym["flops_fact"] / (ms * 1e-3) / 1e9, 1),
                               "trailing_update_tflops": round(upd_fl / upd_ms, 2) if upd_ms else None,
                               "trailing_update_frac_of_peak": round(upd_fl / upd_ms / peak, 4) if upd_ms else None,
                               "kernels": kinds}
            s.close()
            print(json.dumps(line), flush=True)


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
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="as_dense_cols",
                    help="as_dense_cols | as_staircase | ne_random | ne_grid | ne_grid_small | as_batch | "
                         "as_batch_small | ne_dense_front[_<f>] | as_staircase_qp")
    ap.add_argument("--prec", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--nsolves", type=int, default=2)
    ap.add_argument("--opts", default="", help="JSON object of extra qdmf_options fields (after tuning)")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the autotuner's file for the workload")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-line", action="store_true",
                    help="skip the extra mixed run with FP32 products when the tuned mixed path has none")
    ap.add_argument("--c0", action="store_true",
                    help="instead: the dense-front sweep (one JSON line per front order and pivot count)")
    ap.add_argument("--c0-sizes", default="1024,2048,4096,8192")
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
    if args.c0:
        run_c0(args)
        return
    lp, opts = make_workload(args.workload)
    tuned, tuning_file = ({}, None) if args.no_tuning else tuned_options(args.workload)
    opts = dict(opts, **tuned)
    if args.opts:
        opts.update(json.loads(args.opts))
    precs = ["fp64", "mixed"] if args.prec == "both" else [args.prec]
    if args.ipm:
        run_ipm(lp, opts, PRECS[precs[0]], args)
        return
    print(f"[bench] workload={lp['name']} precisions={precs} steps={args.steps} warmup={args.warmup} "
          f"options={opts if 'systems' not in opts else {k: v for k, v in opts.items() if k != 'systems'}}",
          file=sys.stderr, flush=True)
    res, sym, analyse_s = run_gpu(lp, opts, precs, args.steps, args.warmup, args.nsolves, not args.no_graph)
    from paper_2508_04370_amd import qdmf as Q
    nrhs = lp["r1"].shape[1]
    nnz_a = int(lp["colptr"][-1])
    # algorithmic work of one step (exact structure of L): the factorisation and, per solve, one
    # forward/D/backward pass and one residual; the same for both precisions, so GFLOP/s compares
    # their times (refinement passes are extra work of a path, not useful work)
    work = sym["flops_fact"] + args.nsolves * nrhs * (sym["flops_solve"] + 4.0 * nnz_a + 2.0 * sym["N"])
    first = precs[0]
    r0 = res[first]
    ms = r0["wall"] * 1e3 / args.steps  # K steps between two device synchronisations
    value = work / (ms * 1e-3) / 1e9
    pr0 = PRECS[first]
    dom = r0["dom"]
    roof = roofline_of(dom, r0["prof"], pr0, Q)
    roof["traffic"] = measured_traffic(Q.KERNEL_KIND_NAMES[dom], args.workload)
    roof["ms_per_step_with_brackets"] = round(float(np.median(r0["ms_profiled"])), 4)
    roofs = {}
    pk = r0["per_kind"]
    for name, kinds in (("trailing_update", (3, 7)), ("solves", (5, 6)), ("assembly", (1,)), ("window", (2,))):
        tot = {"launches": sum(pk[k]["launches"] for k in kinds), "total_ms": sum(pk[k]["total_ms"] for k in kinds),
               "flops": sum(pk[k]["flops"] for k in kinds), "bytes": sum(pk[k]["bytes"] for k in kinds)}
        if tot["launches"]:
            rr = roofline_of(kinds[0], tot, pr0, Q)
            rr["kernel"] = "+".join(Q.KERNEL_KIND_NAMES[k] for k in kinds)
            rr["ms_per_step"] = round(tot["total_ms"], 3)
            roofs[name] = rr
    # the same fractions against peaks measured on this device (matrix instructions, vector
    # FMAs, a streaming copy), beside the datasheet ones
    try:
        measured = Q.qdmf_peak_probe(0, None)
    except Exception as exc:  # a failed probe leaves the datasheet fractions only
        print(f"[bench] peak probe failed: {exc}", file=sys.stderr, flush=True)
        measured = None
    if measured:
        for r in [roof] + list(roofs.values()):
            mp = {"mfma": measured["mfma_f32_tflops"] if (r["bound"] == "mfma" and pr0 == 1)
                  else measured["mfma_f64_tflops"], "hbm": measured["hbm_gbs"],
                  "alu": measured["valu_f64_tflops"]}[r["bound"]]
            r["peak_measured"] = round(mp, 3)
            r["frac_measured"] = round(r["achieved"] / mp, 6) if mp > 0 else None
    out = {
        "metric": "factorise+solve GFLOP/s & ms/IPM-iter, mixed vs FP64 at backward err <=1e-10",
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if first == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": lp["name"], "m": lp["m"], "n": lp["n"], "mode": "AS" if lp["mode"] else "NE",
                   "nrhs": nrhs, "solves_per_step": args.nsolves, "precision_of_value": first,
                   "N": sym["N"], "nsuper": sym["nsuper"], "nlevels": sym["nlevels"],
                   "max_front": sym["max_front"], "flops_fact": sym["flops_fact"], "nnz_l": sym["nnz_l"],
                   "work_per_step_flops": work, "analyse_s": round(analyse_s, 2),
                   "options": {k: v for k, v in opts.items() if k != "systems"}, "tuning_file": tuning_file},
        "roofline": roof,
        "rooflines": roofs,
        "kernel_ms_per_step_by_kind": {Q.KERNEL_KIND_NAMES[k]: round(v["total_ms"], 3) for k, v in pk.items()},
        "measured_peaks": measured,
    }
    for pname in precs:
        r = res[pname]
        mms = r["wall"] * 1e3 / args.steps
        target = 1e-12 if pname == "fp64" else 1e-10
        entry = {"ms_per_step": round(mms, 4), "ms_per_ipm_iteration": round(mms, 4),
                 "gflops": round(work / (mms * 1e-3) / 1e9, 3),
                 "ms_median": round(float(np.median(r["ms"])), 4), "ms_min": round(min(r["ms"]), 4),
                 "ms_max": round(max(r["ms"]), 4), "berr_nw_max": max(r["berr"]), "target_berr": target,
                 "target_met": bool(max(r["berr"]) <= target), "refine_steps_mean": float(np.mean(r["steps"])),
                 "inertia": [r["fstats"]["nneg"], r["fstats"]["npos"]], "dominant_kernel":
                 Q.KERNEL_KIND_NAMES[r["dom"]],
                 "kernel_ms_per_step_by_kind": {Q.KERNEL_KIND_NAMES[k]: round(v["total_ms"], 3)
                                                for k, v in r["per_kind"].items()}}
        if "graph_ms" in r:
            gms = float(np.median(r["graph_ms"]))
            entry["graph"] = {"ms_per_step": round(gms, 4), "gflops": round(work / (gms * 1e-3) / 1e9, 3),
                              "berr_nw": r["graph_berr"], "vs_eager": round(gms / float(np.median(r["ms"])), 4)}
        if "systems" in r["fstats"]:
            entry["batch"] = {k: r["fstats"][k] for k in ("systems", "worst_system_berr_nw",
                                                          "inertia_ok_all_systems")}
        out[pname] = entry
    if "fp64" in res and "mixed" in res:
        f64, mx = out["fp64"], out["mixed"]
        out["mixed_vs_fp64"] = {"speedup": round(f64["ms_per_step"] / mx["ms_per_step"], 4),
                                "both_within_1e-10": bool(f64["berr_nw_max"] <= 1e-10 and mx["berr_nw_max"] <= 1e-10)}
    if "fp64" in res and "mixed" in res and opts.get("f_mix", 1024) > sym["max_front"] and not args.no_fp32_line:
        # the tuned mixed configuration takes no FP32 products on this workload (they did not
        # pay): time the mixed path with them on (the default f_mix) as well, same steps
        print("[bench] mixed with FP32 products (f_mix 1024)", file=sys.stderr, flush=True)
        o32 = dict(opts, f_mix=1024)
        r32, _, _ = run_gpu(lp, o32, ["mixed"], args.steps, args.warmup, args.nsolves, False)
        r = r32["mixed"]
        mms = r["wall"] * 1e3 / args.steps
        out["mixed_fp32_products"] = {
            "f_mix": 1024, "ms_per_step": round(mms, 4), "gflops": round(work / (mms * 1e-3) / 1e9, 3),
            "berr_nw_max": max(r["berr"]), "target_met": bool(max(r["berr"]) <= 1e-10),
            "refine_steps_mean": float(np.mean(r["steps"])),
            "speedup_vs_fp64": round(out["fp64"]["ms_per_step"] / mms, 4),
            "kernel_ms_per_step_by_kind": {Q.KERNEL_KIND_NAMES[k]: round(v["total_ms"], 3)
                                           for k, v in r["per_kind"].items()}}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
