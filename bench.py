#!/usr/bin/env python3
"""Throughput of one periodic-DMK evaluation on one MI355X.

Workload: 3D triclinic cell a1=(1,0,0), a2=(0.5,4,0), a3=(0.3,0.7,17) (edge
ratio ~17), N = 1e7 sources on a thin spherical shell (radius 0.3, width 1e-3
in fractional coordinates), +-1 neutral charges, targets = sources,
eps = 1e-6.  A step is one full call (orientation, images, tree, lists, near
field, far field, assembly) with inputs resident in HBM.

Prints one JSON line.  --gpus above 1 is rejected: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Per-pair floating-point work of the residual sum (3D, FP64), counted from the
# kernel's arithmetic on every visited pair: 3 sub + 3 FMA for r^2, compare.
# Pairs inside the support add sqrt, divide and a Clenshaw series of nE terms;
# those are counted separately from the kernel's own in-support statistics.
FLOP_PER_VISITED_PAIR = 9.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=float, default=1e7)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=16)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2606_28608_amd import pdmk, workloads as W

    n = int(args.n)
    L, src, q = W.shell3d(n, seed=3)
    dev = torch.device("cuda:0")
    S = torch.tensor(src, dtype=torch.float64, device=dev)
    Q = torch.tensor(q, dtype=torch.float64, device=dev)
    plan = pdmk.Plan(L, eps=args.eps, precision=args.precision)
    g = plan.geometry()

    for _ in range(args.warmup):
        pot = plan.eval(S, Q)
    torch.cuda.synchronize()
    stage = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pot = plan.eval(S, Q)
        stage.append(plan.stats())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    value = n / (dt / args.steps)

    st = stage[-1]
    avg = {k: sum(s[k] for s in stage) / len(stage) for k in stage[0] if k.startswith("t_")}

    # dominant kernel: the residual sums (one launch per call); its duration is
    # the library's HIP-event time around that launch on the call's stream
    t_dir = avg["t_direct_ms"] * 1e-3
    pairs = st["n_direct_pairs"]
    # peak of FP64 vector arithmetic (256 CUs x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz)
    peak = 78.6
    achieved = pairs * FLOP_PER_VISITED_PAIR / t_dir / 1e12 if t_dir > 0 else 0.0
    roofline = {"bound": "alu", "kernel": "k_direct", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                "launch_ms": avg["t_direct_ms"], "pairs_per_launch": pairs,
                "flop_per_pair": FLOP_PER_VISITED_PAIR}

    err = None
    if not args.no_check:
        gold = os.path.join(ROOT, "tests", "golden", "shell3d_n1e7_seed3.txt")
        if os.path.exists(gold) and n == 10_000_000:
            data = np.loadtxt(gold)
            idx = data[:, 0].astype(np.int64)
            ref = data[:, 1]
            got = pot.cpu().numpy()[idx]
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import ewald as E
        rng = np.random.default_rng(7)
        ns = args.cpu_sample
        idx = rng.choice(n, ns, replace=False)
        t1 = time.perf_counter()
        E.ewald_sampled(L, src, q, idx)
        tc = time.perf_counter() - t1
        cpu = {"value": ns / tc, "unit": "particles/s", "cores": os.cpu_count(),
               "kind": "oracle",
               "sample": "Ewald potential at %d sampled targets of the same N=%d system "
                         "(structure factor over all sources, real-space sum over all "
                         "sources); %.1f s" % (ns, n, tc)}

    out = {
        "metric": "particles/sec, 3D triclinic N=1e7 at eps=1e-6: mixed-precision vs FP64 on 1 GPU",
        "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "mixed",
        "data": "synthetic",
        "config": {"workload": "shell3d: triclinic a1=(1,0,0) a2=(0.5,4,0) a3=(0.3,0.7,17), "
                               "N=%d thin shell r=0.3 w=1e-3, +-1 charges, eps=%g" % (n, args.eps),
                   "precision": args.precision, "kappa": g.kappa, "n_s": g.n_s,
                   "porder": g.porder, "npw": g.npw, "nufft_w": g.nufft_w,
                   "fourier_grid": list(g.fgrid)},
        "e_rel_sampled": err,
        "stages_ms": {k: round(v, 3) for k, v in avg.items()},
        "counts": {k: st[k] for k in ("n_images", "n_levels", "n_boxes", "n_leaves",
                                      "n_nonleaf", "n_direct_pairs", "n_pw_pairs")},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
