"""Autotuner of the launch shapes of one measured workload.

Coordinate descent over the options that only decide how the same arithmetic is cut into
launches, starting from the defaults: which fronts take grouped trailing updates
(syrk_group_front) and how many windows a group holds (syrk_group), which trailing matrices
take 128 x 128 tiles (syrk_tile_front), which supernodes take the many-workgroup solves
(split_solve_front), which fronts are factorised whole in LDS (small_front), which fronts
overlap their trailing updates with the next windows on a second stream (lookahead_front),
and, for the mixed path, which fronts take FP32 products (f_mix).  The block size nb, the amalgamation
rule and the pivoting parameters are never touched: they change the factor itself.

A candidate is timed over a few steps (factorise + the workload's solves, refined as in the
measured run) on freshly drawn Theta, and kept only if it is faster than the best so far
and its backward error still meets the precision's target (or is no worse than ten times
the defaults').  The result goes to <out>/<workload>.json, which bench.py reads:

    python -m paper_2508_04370_amd.autotune --workload as_dense_cols --out <dir>
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import workloads as W

SPACE = [
    ("syrk_group_front", [1024, 512, 2048, 4096, 0]),
    ("syrk_group", [4, 2, 3]),
    ("syrk_tile_front", [0, 1024, 2048, 4096]),
    ("split_solve_front", [1024, 512, 2048, 4096]),
    ("small_front", [64, 32, 16]),
    ("lookahead_front", [0, 1024]),
]
MIXED_SPACE = [("f_mix", [1024, 2048, 4096, 1 << 30])]
TARGET = {0: 1e-12, 1: 1e-10}


def _log(msg):
    print(f"[autotune] {msg}", file=sys.stderr, flush=True)


class Bench:
    """One workload on the device: Theta per iteration and the right-hand sides, resident."""

    def __init__(self, name, nsolves=2, steps=3, warmup=1):
        import torch
        self.torch = torch
        self.name = name
        self.lp, self.base = W.named_workload(name)
        lp = self.lp
        self.steps, self.warmup, self.nsolves = steps, warmup, nsolves
        dev = "cuda:0"
        self.TH = [torch.from_numpy(W.iteration_theta(lp, k, 7)).to(dev) for k in range(steps + warmup)]
        if "systems" in lp:
            rs = [W.as_batch_rhs(q, s_, 0, 0) for s_, q in enumerate(lp["systems"])]
            lp["r7"] = np.concatenate([r[0] for r in rs]).reshape(-1, 1)
            lp["r1"] = np.concatenate([r[1] for r in rs]).reshape(-1, 1)
        from . import qdmf as Q
        self.Q = Q
        self.r1 = Q.to_device_colmajor(lp["r1"], dev)
        self.r7 = Q.to_device_colmajor(lp["r7"], dev) if lp["mode"] == W.AS else None
        nrhs = self.r1.shape[1]
        self.dx = torch.empty((nrhs, lp["n"]), dtype=torch.float64, device=dev).T
        self.dy = torch.empty((nrhs, lp["m"]), dtype=torch.float64, device=dev).T
        self.perm = None  # the first analysis' ordering, reused by every candidate (not for batches)

    def run(self, opts, prec):
        """Median ms per step and the worst backward error of the timed steps."""
        torch, Q, lp = self.torch, self.Q, self.lp
        o = dict(self.base, **opts)
        if "systems" in lp:
            o["systems"] = lp["systems"]
        s = Q.Solver(lp, device=0, perm=self.perm, **o)
        if self.perm is None and "systems" not in lp:
            self.perm = s.sym["perm"].copy()
        nrhs = self.r1.shape[1]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms, berr = [], 0.0
        for k in range(self.warmup + self.steps):
            e0.record()
            s.factorise(self.TH[k], lp["rho"], lp["delta"], prec)
            for _ in range(self.nsolves):
                s.solve(self.r7, self.r1, self.dx, self.dy)
            e1.record()
            e1.synchronize()
            if k >= self.warmup:
                ms.append(e0.elapsed_time(e1))
                if s.systems is not None:
                    b = float(np.max(s.batch_stats(nrhs)["berr_nw"]))
                else:
                    b = float(s.solve_stats(nrhs)["berr_nw"])
                if berr == berr and (b != b or b > berr):  # the worst, NaN kept
                    berr = b
        s.close()
        return float(np.median(ms)), berr


def tune(name, precs=(0, 1), steps=3, warmup=1):
    b = Bench(name, steps=steps, warmup=warmup)
    chosen, trials, default = {}, [], {}
    for prec in precs:
        space = SPACE if prec == 0 else MIXED_SPACE
        if prec == 1 and 0 not in precs:
            space = SPACE + MIXED_SPACE
        t, e = b.run(chosen, prec)
        default[prec] = (t, e)
        best = t
        bound = max(TARGET[prec], 10.0 * e) if np.isfinite(e) else TARGET[prec]
        _log(f"{name} prec {prec}: start {chosen} {t:.2f} ms berr {e:.2e}")
        trials.append(dict(prec=prec, options=dict(chosen), ms=t, berr=e, kept=True))
        for key, values in space:
            for v in values:
                if chosen.get(key, values[0]) == v:
                    continue
                cand = dict(chosen, **{key: v})
                t, e = b.run(cand, prec)
                ok = bool(e <= bound)
                kept = ok and t < best * 0.99
                _log(f"{name} prec {prec}: {key}={v} {t:.2f} ms berr {e:.2e}{' kept' if kept else ''}")
                trials.append(dict(prec=prec, options=cand, ms=t, berr=e, kept=kept))
                if kept:
                    best, chosen = t, cand
    final = {prec: b.run(chosen, prec) for prec in precs}
    return dict(workload=name, options=chosen,
                default_ms={str(p): default[p][0] for p in precs},
                tuned_ms={str(p): final[p][0] for p in precs},
                tuned_berr={str(p): final[p][1] for p in precs},
                gain={str(p): default[p][0] / final[p][0] for p in precs},
                steps=steps, warmup=warmup, trials=trials)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", required=True, help="directory of the <workload>.json result")
    ap.add_argument("--precs", default="0,1", help="precisions to tune: 0 FP64, 1 mixed")
    ap.add_argument("--steps", type=int, default=3)
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    rec = tune(args.workload, tuple(int(p) for p in args.precs.split(",")), steps=args.steps)
    import torch
    rec["device"] = torch.cuda.get_device_name(0)
    rec["tuning_s"] = round(time.perf_counter() - t0, 1)
    os.makedirs(args.out, exist_ok=True)
    path = os.path.join(args.out, f"{args.workload}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    _log(f"wrote {path}: {rec['options']} gain {rec['gain']}")


if __name__ == "__main__":
    main()
