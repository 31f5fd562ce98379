#!/usr/bin/env python3
"""Throughput of one periodic-DMK evaluation on one MI355X.

Workload: 3D triclinic cell a1=(1,0,0), a2=(0.5,4,0), a3=(0.3,0.7,17) (edge
ratio ~17), N = 1e7 sources on a thin spherical shell (radius 0.3, width 1e-3
in fractional coordinates), +-1 neutral charges, targets = sources,
eps = 1e-6.  A step is one full call (orientation, images, tree, lists, near
field, far field, assembly) with inputs resident in HBM.

Both arithmetic modes are timed: the mixed-precision evaluation gives
`value`; the FP64 evaluation is reported beside it under "fp64".  Each mode
reports its relative l2 error on stored oracle values at 64 sampled sources.

Beside the timed steps each mode also reports (fewer steps each): the same
workload at eps = 1e-3 with its own planned (kappa, n_s); the default plan
(kappa = 3, image halo populated); and one run with every stage on one
stream, whose per-stage timings give the far field's stand-alone spreading,
transform and interpolation times.  A result whose sampled error exceeds eps
is reported with "parity_ok": false and no value.

Prints one JSON line.  --gpus above 1 is rejected: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks: vector ALU for the residual sums (an n-body sum with
# a compactly supported polynomial kernel), matrix cores for the plane-wave
# contractions; both are 157.3 TFLOP/s in FP32 and 78.6 TFLOP/s in FP64.
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_shell3d_n1e7_eps1e-6.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2606_28608_amd", "csrc", f)
               for f in ("near.hip", "pwmfma.hip")]


def flop_per_pair(series_len: int):
    """Arithmetic of the residual kernel, counted from its operations.

    Every visited pair: 3 subtractions, 1 multiply and 2 FMAs for r^2 (8 flop).
    A pair inside the support r < h adds the series argument u = r^2 (2/h^2) - 1
    (one FMA, 2), Horner's rule over the series (series_len - 1 FMAs), rsqrt
    (1), 1/r - E/h as one FMA (2) and the charge FMA (2): 2 * series_len + 5.
    """
    return 8.0, 2.0 * series_len + 5.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=float, default=1e7)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default (kappa, n_s) instead of planning them on the input")
    ap.add_argument("--kappa", type=float, default=0.0,
                    help="fixed kappa for the timed runs (with --n-s; skips the planner)")
    ap.add_argument("--n-s", type=int, default=0, dest="n_s",
                    help="fixed leaf capacity for the timed runs (with --kappa)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle targets for the CPU baseline (0: one per oracle thread)")
    ap.add_argument("--cpu-alpha", type=float, default=1.3,
                    help="Ewald splitting parameter of the CPU baseline run")
    ap.add_argument("--child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--child-batch", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched many-cell measurement")
    ap.add_argument("--batch-systems", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-batch-tune", action="store_true",
                    help="skip the batch autotuner (per-size-class kappa, n_s)")
    ap.add_argument("--batch-workers", type=int, default=8,
                    help="host workers of the batched measurement")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the eps=1e-3, default-plan and one-stream runs")
    ap.add_argument("--cpu-full", default="10000,100000",
                    help="sizes of the full-N uniform oracle runs ('' to skip)")
    ap.add_argument("--paper-tables", action="store_true",
                    help="instead of the benchmark line: the paper's nine cells at N=1e7 and "
                         "eps 1e-3..1e-12 (FP64, default plans), one JSON line")
    ap.add_argument("--paper-steps", type=int, default=3)
    ap.add_argument("--paper-cells", default="",
                    help="comma-separated subset of the paper's cells (default: all nine)")
    ap.add_argument("--paper-eps", default="",
                    help="comma-separated subset of eps (default: 1e-3,1e-6,1e-9,1e-12)")
    ap.add_argument("--paper-n", type=float, default=1e7)
    ap.add_argument("--child-paper", action="store_true", help=argparse.SUPPRESS)
    return ap.parse_args()


def progress(msg):
    """A progress line on stderr (the JSON result goes to stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for src in KERNEL_SRCS:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(mode, kernel, kappa, n_s):
    """HBM bytes per launch of `kernel` from the committed counter runs, or
    None when the kernel sources have changed since they were taken or the
    runs used other (kappa, n_s)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256_16") != kernel_source_hash():
        return None
    for run in t.get("runs", []):
        if (run["precision"] == mode and abs(run["kappa"] - kappa) < 1e-12
                and run["n_s"] == n_s):
            m = run["kernels"].get(kernel)
            return None if m is None else m.get("bytes_per_launch")
    return None


def run_mode(pdmk, L, S, Q, n, eps, precision, steps, warmup, gold, over=None):
    import numpy as np
    import torch
    progress("%s eps=%g %s: %d warm-up + %d timed steps" % (precision, eps, over or "defaults",
                                                          warmup, steps))
    plan = pdmk.Plan(L, eps=eps, precision=precision, **(over or {}))
    g = plan.geometry()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pot = plan.eval(S, Q)
    torch.cuda.synchronize()
    cold_ms = 1e3 * (time.perf_counter() - t0)
    for _ in range(max(0, warmup - 1)):
        pot = plan.eval(S, Q)
    torch.cuda.synchronize()
    stage, per = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        pot = plan.eval(S, Q)          # blocks until the results are written
        per.append(1e3 * (time.perf_counter() - t1))
        stage.append(plan.stats())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = None
    if gold is not None:
        idx, ref = gold
        got = pot.cpu().numpy()[idx]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    st = stage[-1]
    avg = {k: sum(s[k] for s in stage) / len(stage) for k in stage[0] if k.startswith("t_")}
    return {"plan": g, "ms_per_step": 1e3 * dt / steps, "median_ms": statistics.median(per),
            "step_ms": [round(x, 2) for x in per],
            "cold_first_call_ms": cold_ms, "value": n / (dt / steps), "e_rel_sampled": err,
            "stats": st, "stages_ms": {k: round(v, 3) for k, v in avg.items()}}


def run_bloch(pdmk, L, S, Q, n, eps, precision, steps, warmup, over):
    """Quasi-periodic evaluation (pdmk_plan_eval_bloch) of the same input and
    plan, Bloch vector (0.7, -1.1, 0.4), against the stored Bloch oracle values
    when present."""
    import numpy as np
    import torch
    beta = np.array([0.7, -1.1, 0.4])
    progress("bloch %s eps=%g %s: %d warm-up + %d timed steps" % (precision, eps, over,
                                                                warmup, steps))
    plan = pdmk.Plan(L, eps=eps, precision=precision, bloch=beta, **over)
    for _ in range(warmup):
        pot = plan.eval_bloch(S, Q)
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        pot = plan.eval_bloch(S, Q)
        per.append(1e3 * (time.perf_counter() - t1))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = None
    path = os.path.join(ROOT, "tests", "golden", "shell3d_n1e7_seed3_bloch.txt")
    if n == 10_000_000 and os.path.exists(path):
        data = np.loadtxt(path)
        idx = data[:, 0].astype(np.int64)
        ref = data[:, 1] + 1j * data[:, 2]
        got = pot.cpu().numpy()[idx]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return {"value": n / (dt / steps), "ms_per_step": 1e3 * dt / steps,
            "median_ms": statistics.median(per), "e_rel_sampled": err,
            "parity_ok": err is None or err <= eps, "beta": list(beta),
            "fourier_grid": list(plan.geometry().fgrid)}


def run_cube(pdmk, n, eps, precision, steps):
    """The cube-cell construction of rem:cube against physical images on the
    same input: N clustered sources in the unit cube, kappa = 4 (r_c a
    quarter of the side), n_s = 300."""
    import numpy as np
    import torch
    from paper_2606_28608_amd import workloads as W
    L, src, q = W.clustered3d(n, seed=2, cell="cubic")
    dev = torch.device("cuda:0")
    S = torch.tensor(src, dtype=torch.float64, device=dev)
    Q = torch.tensor(q, dtype=torch.float64, device=dev)
    out, pots = {}, {}
    for name, vi in (("physical_images", False), ("virtual_images", True)):
        progress("cube %s %s eps=%g: 1 warm-up + %d timed steps" % (name, precision, eps, steps))
        plan = pdmk.Plan(L, eps=eps, precision=precision, kappa=4.0, n_s=300, virtual_images=vi)
        plan.eval(S, Q)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            pot = plan.eval(S, Q)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = plan.stats()
        pots[name] = pot.cpu().numpy()
        out[name] = {"ms_per_step": 1e3 * dt, "value": n / dt, "n_images": st["n_images"],
                     "t_build_ms": round(st["t_build_ms"], 3), "t_near_ms": round(st["t_near_ms"], 3)}
    a, b = pots["virtual_images"], pots["physical_images"]
    out["rel_diff"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out["workload"] = "clustered3d cubic, N=%d, kappa=4, n_s=300, eps=%g" % (n, eps)
    return out


def _ball_modes(J):
    """Modes of the Hermitian half ball |j| <= J (j0 >= 0)."""
    n = 0
    for j0 in range(J + 1):
        for j1 in range(-J, J + 1):
            for j2 in range(-J, J + 1):
                n += j0 * j0 + j1 * j1 + j2 * j2 <= J * J
    return n


def pw_fma_per_box(P, J):
    """Useful real multiply-adds of the three axis contractions of one box
    (one direction), counted from the shapes: (J+1) slabs of N1 x N1 modes,
    P^3 proxy points, complex arithmetic as real products."""
    N1 = 2 * J + 1
    return (2 * (J + 1) * P * P * P + 2 * N1 * 2 * P * (J + 1) * P
            + (J + 1) * N1 * 2 * P * 2 * N1)


def roofline_all(r, mode, plan):
    """Achieved rate of the main kernels: algorithmic flops of one call /
    summed HIP-event duration of the kernel's launches in that call."""
    st, sm = r["stats"], r["stages_ms"]
    out = {}
    fv, fs = flop_per_pair(st["series_len"])
    # pairs evaluated once (targets = sources): each in-support pair also forms
    # q_t R for its source end and adds it into that source's sum (2 flop)
    if st.get("pairs_once"):
        fs += 2
    # pairs the kernel evaluates: the list pairs left after the per-pass reach
    # test (a source farther than h + rho from the centre of a pass's targets
    # is not staged); the test itself costs 9 flop per candidate source and pass
    staged = st.get("n_staged_pairs", 0) or st["n_direct_pairs"]
    flop = staged * fv + st["n_support_pairs"] * fs + st["n_direct_pairs"] / 64.0 * 9.0
    t = sm["t_direct_ms"] * 1e-3
    out["k_direct"] = {"bound": "alu", "achieved": flop / t / 1e12 if t > 0 else 0.0,
                       "peak": PEAK_TFLOPS[mode], "unit": "TFLOP/s", "launch_ms": sm["t_direct_ms"],
                       "launches": 1, "flop_per_launch": flop,
                       "pairs_listed": st["n_direct_pairs"], "pairs_staged": staged,
                       "pairs_in_support": st["n_support_pairs"],
                       "flop_per_staged_pair": fv, "flop_per_support_pair": fs,
                       "pairs_once": bool(st.get("pairs_once"))}
    P, J = plan["porder"], plan["npw"]
    nb = _ball_modes(J)
    tr = pw_fma_per_box(P, J)
    flop_in = 2.0 * tr * st["n_pwin_boxes"]
    flop_out = 2.0 * tr * st["n_pwout_boxes"]
    nlev = st["n_levels"] - 1
    for name, f, tms in (("k_pw_in", flop_in, sm.get("t_pwin_ms", 0.0)),
                         ("k_pw_out", flop_out, sm.get("t_pwout_ms", 0.0))):
        t = tms * 1e-3
        out[name] = {"bound": "mfma", "achieved": f / t / 1e12 if t > 0 else 0.0,
                     "peak": PEAK_TFLOPS[mode], "unit": "TFLOP/s", "launch_ms": tms / max(1, nlev),
                     "launches": nlev, "flop_per_launch": f / max(1, nlev),
                     "flop_per_box": 2.0 * tr}
    # colleague translation: compulsory bytes = every outgoing expansion of
    # the level read once + every incoming expansion written once (half-ball
    # modes, complex FP32 or FP64)
    cb = 8 if mode == "mixed" else 16
    tms = sm.get("t_pwtr_ms", 0.0)
    if tms > 0:
        by = float(nb * cb * (st["n_pwout_boxes"] + st["n_pwin_boxes"]))
        t = tms * 1e-3
        out["k_pw_trans"] = {"bound": "hbm", "achieved": by / t / 1e9, "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "launch_ms": tms / max(1, nlev), "launches": nlev,
                             "bytes_per_launch": by / max(1, nlev),
                             "bytes_per_box": nb * cb,
                             "flop_per_launch": 8.0 * nb * st["n_pw_pairs"] / max(1, nlev)}
    for v in out.values():
        v["frac"] = v["achieved"] / v["peak"]
    return out


def far_field(r1, n, plan, mode):
    """Stand-alone far-field stages (every stage on one stream): spreading,
    transforms + scaling, interpolation; algorithmic HBM bytes: spreading
    reads positions and charges (32 B per source) and writes the grid once
    (8 B per cell); interpolation reads positions (24 B), reads and writes
    the potential (16 B) and reads the complex grid once (16 B per cell);
    flops: w^d multiply-adds per point each way."""
    sm = r1["stages_ms"]
    g = plan["fourier_grid"]
    cells = 1
    for m in g:
        cells *= m
    w = plan["nufft_w"]
    out = {}
    for name, key, by in (("k_spread_coop", "t_spread_ms", 32.0 * n + 8.0 * cells),
                          ("k_interp_t", "t_interp_ms", 40.0 * n + 16.0 * cells)):
        t = sm.get(key, 0.0) * 1e-3
        out[name] = {"bound": "hbm", "launch_ms": sm.get(key, 0.0), "launches": 1,
                     "bytes_per_launch": by,
                     "achieved": by / t / 1e9 if t > 0 else 0.0, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "tflops": 2.0 * n * w ** 3 / t / 1e12 if t > 0 else 0.0}
        out[name]["frac"] = out[name]["achieved"] / PEAK_HBM_GBS
    out["fft_and_scaling_ms"] = sm.get("t_fft_ms", 0.0)
    out["fourier_grid"] = g
    out["note"] = ("one-stream run of the same plan (no overlap with the near field); "
                   "the spreading and interpolation are bound by LDS atomics and the "
                   "w^d stencil arithmetic, not by HBM")
    out["precision"] = mode
    return out


def roofline(r, mode, plan):
    """The bench's `roofline` object: the kernel with the largest time per call."""
    allk = roofline_all(r, mode, plan)
    dom = max(allk, key=lambda k: allk[k]["launch_ms"] * allk[k]["launches"])
    d = dict(allk[dom])
    d["kernel"] = dom
    d["traffic"] = load_traffic(mode, dom, plan["kappa"], plan["n_s"])
    d["arith"] = "fp32" if mode == "mixed" else "fp64"
    d["kernels"] = {k: {kk: allk[k][kk] for kk in ("achieved", "frac", "launch_ms", "launches")}
                    for k in allk}
    return d


def copy_calib():
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}))


def child(args):
    """Time one arithmetic mode on the GPU and print its results as JSON."""
    import numpy as np
    import torch
    from paper_2606_28608_amd import pdmk, workloads as W

    n = int(args.n)
    L, src, q = W.shell3d(n, seed=3)
    dev = torch.device("cuda:0")
    S = torch.tensor(src, dtype=torch.float64, device=dev)
    Q = torch.tensor(q, dtype=torch.float64, device=dev)
    gold = None
    if not args.no_check and n == 10_000_000:
        path = os.path.join(ROOT, "tests", "golden", "shell3d_n1e7_seed3.txt")
        if os.path.exists(path):
            data = np.loadtxt(path)
            gold = (data[:, 0].astype(np.int64), data[:, 1])
    over, tuning = {}, None
    if args.kappa > 0 and args.n_s > 0:
        over = {"kappa": args.kappa, "n_s": args.n_s}
    elif not args.no_tune:
        # runtime planning of (kappa, n_s) on this input, before the timed region
        t0 = time.perf_counter()
        progress("%s: planning (kappa, n_s) on the input" % args.precision)
        k, ns, table = pdmk.tune(L, S, Q, eps=args.eps, precision=args.precision, trials=1)
        over = {"kappa": k, "n_s": ns}
        tuning = {"seconds": round(time.perf_counter() - t0, 2),
                  "ms_per_candidate": {"kappa=%g,n_s=%d" % c: round(t, 2) for c, t in table.items()}}
    r = run_mode(pdmk, L, S, Q, n, args.eps, args.precision, args.steps, args.warmup, gold, over)
    r["tuning"] = tuning
    g = r.pop("plan")

    def plan_of(g):
        return {"kappa": g.kappa, "n_s": g.n_s, "porder": g.porder, "npw": g.npw,
                "nufft_w": g.nufft_w, "fourier_grid": list(g.fgrid)}

    r["plan"] = plan_of(g)
    r["roofline"] = roofline(r, args.precision, r["plan"])
    if not args.no_extra:
        def brief(x, eps):
            d = {k: x[k] for k in ("value", "ms_per_step", "median_ms", "e_rel_sampled")}
            d["plan"] = plan_of(x.pop("plan"))
            d["parity_ok"] = x["e_rel_sampled"] is None or x["e_rel_sampled"] <= eps
            d["n_images"] = x["stats"]["n_images"]
            d["stages_ms"] = x["stages_ms"]
            return d
        extra = {}
        # the second C3 tolerance, with its own planned (kappa, n_s)
        k3, ns3, _ = pdmk.tune(L, S, Q, eps=1e-3, precision=args.precision, trials=1)
        extra["eps_1e-3"] = brief(run_mode(pdmk, L, S, Q, n, 1e-3, args.precision, 3, 1, gold,
                                           {"kappa": k3, "n_s": ns3}), 1e-3)
        # the default plan, with its image halo (N'/N ~ 1.45 at kappa = 3)
        extra["default_plan"] = brief(run_mode(pdmk, L, S, Q, n, args.eps, args.precision, 3, 1,
                                               gold, {}), args.eps)
        # every stage on one stream: stand-alone stage times
        one = run_mode(pdmk, L, S, Q, n, args.eps, args.precision, 3, 1, gold,
                       dict(over, one_stream=True))
        r["far_field"] = far_field(one, n, r["plan"], args.precision)
        extra["one_stream"] = brief(one, args.eps)
        # quasi-periodic conditions (Section 4.1) with the same plan
        extra["bloch"] = run_bloch(pdmk, L, S, Q, n, args.eps, args.precision, 3, 1, over)
        # the cube-cell construction (virtual images) against physical images
        del S, Q
        torch.cuda.empty_cache()
        extra["cube"] = run_cube(pdmk, n, args.eps, args.precision, 3)
        r["extra"] = extra
        for k in ("k_spread_coop", "k_interp_t"):
            r["roofline"]["kernels"][k] = {kk: r["far_field"][k][kk]
                                           for kk in ("achieved", "frac", "launch_ms", "launches")}
    print(json.dumps(r))


def child_batch(args):
    """Batched evaluation of many small cells (random triclinic cells, log-uniform
    sizes 500..5e4, even systems uniform, odd clustered; +-1 charges): one call
    evaluates every system.  Prints the timing as JSON."""
    import numpy as np
    import torch
    from paper_2606_28608_amd import pdmk, workloads as W
    systems = W.batch_cells(n_sys=args.batch_systems, seed=5)
    offs = np.cumsum([0] + [len(s[2]) for s in systems]).astype(np.int64)
    src = torch.tensor(np.vstack([s[1] for s in systems]), device="cuda:0")
    q = torch.tensor(np.concatenate([s[2] for s in systems]), device="cuda:0")
    Ls = np.stack([s[0] for s in systems])
    t0 = time.perf_counter()
    B = pdmk.Batch(Ls, eps=args.eps, precision=args.precision, workers=args.batch_workers)
    t_plan = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.eval(offs, src, q)
    cold = time.perf_counter() - t0
    for _ in range(max(0, args.warmup - 1)):
        B.eval(offs, src, q)
    per = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        B.eval(offs, src, q)
        per.append(time.perf_counter() - t1)
    n = int(offs[-1])
    ms = 1e3 * sum(per) / len(per)
    res = {"systems": len(systems), "particles": n, "ms_per_call": ms,
           "value": n / (ms * 1e-3), "cold_first_call_ms": 1e3 * cold,
           "plan_create_s": t_plan, "precision": args.precision,
           "workers": args.batch_workers}
    if not args.no_batch_tune:
        # batch autotuner: (kappa, n_s) per size class, then the same timing
        progress("batch %s: autotuning the size classes" % args.precision)
        t0 = time.perf_counter()
        k, ns = B.tune(offs, src, q, trials=3)
        res["tune_s"] = time.perf_counter() - t0
        B.eval(offs, src, q)
        per = []
        for _ in range(args.steps):
            t1 = time.perf_counter()
            B.eval(offs, src, q)
            per.append(time.perf_counter() - t1)
        ms_t = 1e3 * sum(per) / len(per)
        res.update({"untuned_ms_per_call": ms, "ms_per_call": ms_t, "value": n / (ms_t * 1e-3),
                    "tuned_plans": {"%g,%d" % (r[0], r[1]): int(c) for r, c in
                                    zip(*np.unique(np.stack([k, ns.astype(np.float64)], 1),
                                                   axis=0, return_counts=True))}})
    # kept trees of every cell: new charges enqueued over the worker streams
    # (no tree build, no host read), eager and as one replayed graph
    progress("batch %s: kept trees, execute and graph replay" % args.precision)
    B.bind(offs, src, q)
    rng = np.random.default_rng(7)
    qn = np.concatenate([rng.permutation(s[2]) for s in systems])   # neutral per cell
    q2 = torch.tensor(qn, device="cuda:0")
    out = torch.empty_like(q2)
    for _ in range(2):
        B.execute(q2, out=out)
    B.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.execute(q2, out=out)
    torch.cuda.synchronize()
    ms_x = 1e3 * (time.perf_counter() - t0) / args.steps
    B.status()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.execute(q2, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    t0 = time.perf_counter()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        B.execute(q2, out=out)
    t_cap = time.perf_counter() - t0
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    ms_g = 1e3 * (time.perf_counter() - t0) / args.steps
    res["kept_trees"] = {"execute_ms_per_call": ms_x, "execute_value": n / (ms_x * 1e-3),
                         "graph_ms_per_call": ms_g, "graph_value": n / (ms_g * 1e-3),
                         "capture_s": t_cap,
                         "what": "new charges on every cell's kept tree (pdmk_batch_execute)"}
    print(json.dumps(res))


# The paper's own per-step times t_PDMK (seconds, one CPU thread, FP64,
# N = 1e7) for each cell and eps = 1e-3, 1e-6, 1e-9, 1e-12 (tab:2d,
# tab:rect3d, tab:tri3d).  Context for the GPU times, not a target.
PAPER_T_PDMK = {
    "2d-A1": (11.45, 14.47, 21.51, 31.07), "2d-A10": (8.37, 12.05, 18.84, 26.00),
    "2d-A100": (8.37, 11.76, 19.62, 27.68),
    "rect-iso": (15.27, 51.77, 130.37, 285.13), "rect-rod": (14.84, 62.36, 152.06, 368.90),
    "rect-slab": (21.11, 76.54, 172.28, 345.15),
    "tri-iso": (23.27, 63.77, 183.64, 404.83), "tri-rod": (17.25, 74.22, 163.96, 489.45),
    "tri-slab": (27.23, 95.68, 197.27, 431.24),
}
PAPER_EPS = (1e-3, 1e-6, 1e-9, 1e-12)


def child_paper(args):
    """The paper's nine cells with their wavy distributions at N = 1e7, FP64,
    every eps of its tables: per-step time and stage split, E_rel on the
    stored oracle values when present.  The plan keeps the cell's default
    kappa (the paper's tuning table) and takes n_s from the runtime planner
    over 1, 2, 3 and 4 times the table's leaf capacity (the table was tuned
    for a CPU); the default plan's time from the planner's trial is reported
    beside it."""
    import numpy as np
    import torch
    from paper_2606_28608_amd import pdmk, workloads as W
    n = int(args.paper_n)
    dev = torch.device("cuda:0")
    rows = []
    cells = [c for c in args.paper_cells.split(",") if c] or list(W.PAPER_SYSTEMS)
    epss = [float(e) for e in args.paper_eps.split(",") if e] or list(PAPER_EPS)
    for name in cells:
        progress("paper cell %s: generating N=%d" % (name, n))
        L, src, q = W.paper_system(name, n)
        S = torch.tensor(src, dtype=torch.float64, device=dev)
        Q = torch.tensor(q, dtype=torch.float64, device=dev)
        del src, q
        gold = None
        path = os.path.join(ROOT, "tests", "golden", "paper_%s_n1e7_seed8.txt" % name)
        if n == 10_000_000 and os.path.exists(path):
            data = np.loadtxt(path)
            gold = (data[:, 0].astype(np.int64), data[:, 1])
        for eps in epss:
            j = PAPER_EPS.index(eps) if eps in PAPER_EPS else None
            progress("paper cell %s eps=%g: planning n_s" % (name, eps))
            g0 = pdmk.geometry(L, eps=eps)
            cand = [(g0.kappa, int(g0.n_s * f)) for f in (1, 2, 3, 4)]
            bk, bn, table = pdmk.tune(L, S, Q, eps=eps, candidates=cand, trials=1)
            default_ms = table[(float(g0.kappa), int(g0.n_s))]
            progress("paper cell %s eps=%g: n_s %d" % (name, eps, bn))
            plan = pdmk.Plan(L, eps=eps, kappa=bk, n_s=bn)
            pot = plan.eval(S, Q)   # cold call (tables, workspace)
            pot = plan.eval(S, Q)
            torch.cuda.synchronize()
            per, stats = [], []
            t0 = time.perf_counter()
            for _ in range(args.paper_steps):
                t1 = time.perf_counter()
                pot = plan.eval(S, Q)
                per.append(1e3 * (time.perf_counter() - t1))
                stats.append(plan.stats())
            dt = (time.perf_counter() - t0) / args.paper_steps
            err = None
            if gold is not None:
                got = pot.cpu().numpy()[gold[0]]
                err = float(np.linalg.norm(got - gold[1]) / np.linalg.norm(gold[1]))
            avg = {k: round(sum(x[k] for x in stats) / len(stats), 3)
                   for k in ("t_build_ms", "t_near_ms", "t_far_ms", "t_total_ms")}
            g = plan.geometry()
            t_paper = PAPER_T_PDMK[name][j] if j is not None and n == 10_000_000 else None
            rows.append({"cell": name, "eps": eps, "ms_per_step": round(1e3 * dt, 3),
                         "median_ms": round(statistics.median(per), 3),
                         "particles_per_s": n / dt, "e_rel_sampled": err,
                         "parity_ok": err is None or err <= eps, "stages_ms": avg,
                         "kappa": g.kappa, "n_s": g.n_s, "fourier_grid": list(g.fgrid),
                         "default_plan": {"n_s": int(g0.n_s), "ms_per_step": round(default_ms, 3),
                                          "from": "the planner's trial"},
                         "n_images": stats[-1]["n_images"], "n_levels": stats[-1]["n_levels"],
                         "paper_t_pdmk_s": t_paper,
                         "paper_over_gpu": t_paper / dt if t_paper else None})
            del plan, pot
        del S, Q
        torch.cuda.empty_cache()
    print(json.dumps({"paper_tables": rows, "n": n, "precision": "fp64",
                      "plans": "default kappa, n_s from the runtime planner (1-4x the default)",
                      "steps": args.paper_steps}))


def run_child(args, mode, batch=False):
    cmd = [sys.executable, os.path.abspath(__file__), "--child-batch" if batch else "--child",
           "--precision", mode, "--steps", str(args.batch_steps if batch else args.steps),
           "--warmup", str(args.warmup), "--n", str(args.n), "--eps", str(args.eps),
           "--batch-systems", str(args.batch_systems), "--batch-workers", str(args.batch_workers)]
    if args.no_batch_tune:
        cmd.append("--no-batch-tune")
    if args.no_check:
        cmd.append("--no-check")
    if args.no_tune:
        cmd.append("--no-tune")
    if args.no_extra:
        cmd.append("--no-extra")
    if args.kappa > 0 and args.n_s > 0:
        cmd += ["--kappa", str(args.kappa), "--n-s", str(args.n_s)]
    progress("child %s%s" % (mode, " batch" if batch else ""))
    p = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
    if p.returncode != 0:
        print("bench.py: %s%s run failed with status %d"
              % (mode, " batch" if batch else "", p.returncode), file=sys.stderr)
        sys.exit(p.returncode if p.returncode > 0 else 1)
    return json.loads(p.stdout.strip().splitlines()[-1])


def cpu_baseline(args, n):
    """The Ewald oracle as it stands, on this host's cores (OpenMP threads).

    Sampled mode on the benchmark's own system: the structure factor S(m)
    runs over all N sources once, then each sampled target costs a
    real-space sum over all sources and images plus a reciprocal sum, the
    targets spread over the threads.  A run with one target per thread and
    one with nine per thread give the S(m) time and the time of one round of
    targets (per target: a round / threads); the full-N figure is
    extrapolated from them (labelled as such).  Full runs (every source a target, splitting
    parameter balanced by the oracle's cost model) on uniform +-1 systems at
    the sizes of --cpu-full give measured full-N rates."""
    import numpy as np
    from oracle import ewald as E
    from paper_2606_28608_amd import workloads as W
    progress("cpu baseline: oracle on %d threads" % E.threads())
    L, src, q = W.shell3d(n, seed=3)
    k = args.cpu_sample if args.cpu_sample > 0 else E.threads()
    idx = np.random.default_rng(7).choice(n, 9 * k, replace=False)
    t0 = time.perf_counter()
    E.ewald_sampled(L, src, q, idx[:k], alpha=args.cpu_alpha)
    t_one = time.perf_counter() - t0
    progress("cpu baseline: %d targets in %.1f s" % (k, t_one))
    t0 = time.perf_counter()
    E.ewald_sampled(L, src, q, idx, alpha=args.cpu_alpha)
    t_k = time.perf_counter() - t0
    progress("cpu baseline: %d targets in %.1f s" % (len(idx), t_k))
    rnd = max(t_k - t_one, 0.0) / 8.0
    per_target = rnd / k
    t_s = max(t_one - rnd, 0.0)
    full_est = t_s + n * per_target
    out = {"value": len(idx) / t_k, "unit": "particles/s", "cores": E.threads(),
           "kind": "oracle",
           "sample": "Ewald potential at %d sampled sources of the same N=%d shell system, "
                     "splitting alpha=%g (structure factor over all N sources, real-space sum "
                     "over all N sources and their images); %.1f s"
                     % (len(idx), n, args.cpu_alpha, t_k),
           "structure_factor_s": t_s, "per_target_s": per_target,
           "extrapolated_full_n": {"seconds": full_est, "particles_per_s": n / full_est,
                                   "label": "EXTRAPOLATED: S(m) time + N x per-target time "
                                            "at this alpha, not measured"}}
    full = []
    sizes = [int(float(x)) for x in args.cpu_full.split(",") if x.strip()]
    for m in sizes:
        rng = np.random.default_rng(11)
        u = rng.random((m, 3))
        Lu = W.TRICLINIC3D_L
        sm = u @ Lu.T
        qm = np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
        progress("cpu baseline: full oracle run at N=%d" % m)
        t0 = time.perf_counter()
        E.ewald(Lu, sm, qm)
        tm = time.perf_counter() - t0
        progress("cpu baseline: N=%d in %.1f s" % (m, tm))
        full.append({"n": m, "seconds": tm, "particles_per_s": m / tm,
                     "workload": "uniform, triclinic a1=(1,0,0) a2=(0.4,1.2,0) a3=(0.3,0.5,2), "
                                 "+-1 charges, every source a target"})
    if full:
        out["full_runs"] = full
        if len(full) >= 2:
            a = math.log(full[-1]["seconds"] / full[-2]["seconds"]) / \
                math.log(full[-1]["n"] / full[-2]["n"])
            out["full_runs_fit"] = {"exponent": a, "label": "EXTRAPOLATED from the last two "
                                    "full runs: t ~ N^exponent",
                                    "seconds_at_1e6": full[-1]["seconds"] *
                                    (1e6 / full[-1]["n"]) ** a}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calib()
        return
    if args.child:
        child(args)
        return
    if args.child_batch:
        child_batch(args)
        return
    if args.child_paper:
        child_paper(args)
        return
    if args.paper_tables:
        cmd = [sys.executable, os.path.abspath(__file__), "--child-paper",
               "--paper-steps", str(args.paper_steps), "--paper-cells", args.paper_cells,
               "--paper-eps", args.paper_eps, "--paper-n", str(args.paper_n)]
        p = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
        if p.returncode != 0:
            print("bench.py: paper-table run failed with status %d" % p.returncode,
                  file=sys.stderr)
            sys.exit(p.returncode if p.returncode > 0 else 1)
        print(p.stdout.strip().splitlines()[-1])
        return
    # Each arithmetic mode runs in a child process of its own, one after the
    # other, so that the two measurements share no device state.  This
    # process never touches the GPU.
    modes = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    res = {m: run_child(args, m) for m in modes}
    head = modes[0]
    r = res[head]
    n = int(args.n)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, n)

    def summary(x):
        d = {k: x[k] for k in ("value", "ms_per_step", "median_ms", "step_ms",
                               "cold_first_call_ms", "e_rel_sampled", "stages_ms",
                               "roofline", "tuning")}
        d["kappa"], d["n_s"] = x["plan"]["kappa"], x["plan"]["n_s"]
        return d

    pl = r["plan"]
    out = {
        "metric": "particles/sec, 3D triclinic N=1e7 at eps=1e-6: mixed-precision vs FP64 on 1 GPU",
        "value": r["value"], "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "shell3d: triclinic a1=(1,0,0) a2=(0.5,4,0) a3=(0.3,0.7,17), "
                               "N=%d thin shell r=0.3 w=1e-3, +-1 charges, eps=%g, "
                               "targets = sources" % (n, args.eps),
                   "precision": head, "kappa": pl["kappa"], "n_s": pl["n_s"],
                   "porder": pl["porder"], "npw": pl["npw"], "nufft_w": pl["nufft_w"],
                   "fourier_grid": pl["fourier_grid"],
                   "kappa_n_s_from": "runtime planner (pdmk_plan_tune) on this input, "
                                     "before the timed steps" if r.get("tuning") else "defaults"},
        "tuning": r.get("tuning"),
        "median_ms": r["median_ms"], "step_ms": r["step_ms"],
        "cold_first_call_ms": r["cold_first_call_ms"],
        "e_rel_sampled": r["e_rel_sampled"],
        "stages_ms": r["stages_ms"],
        "counts": {k: r["stats"][k] for k in ("n_images", "n_levels", "n_boxes", "n_leaves",
                                             "n_nonleaf", "n_direct_pairs", "n_staged_pairs",
                                             "n_support_pairs", "n_pw_pairs", "n_pwout_boxes",
                                             "n_pwin_boxes", "workspace_bytes")},
        "roofline": r["roofline"],
        "cpu_baseline": cpu,
    }
    # no value for a result that misses the tolerance on the stored oracle values
    ok = r["e_rel_sampled"] is None or r["e_rel_sampled"] <= args.eps
    out["parity_ok"] = ok
    if not ok:
        out["value"] = None
    if "far_field" in r:
        out["far_field"] = r["far_field"]
    if "extra" in r:
        out["extra"] = {head: r["extra"]}
    for m in modes[1:]:
        out[m] = summary(res[m])
        out[m]["parity_ok"] = res[m]["e_rel_sampled"] is None or \
            res[m]["e_rel_sampled"] <= args.eps
        if "extra" in res[m]:
            out.setdefault("extra", {})[m] = res[m]["extra"]
            out[m]["far_field"] = res[m].get("far_field")
    if not args.no_batch:
        out["batch"] = {"workload": "%d random triclinic cells (edges 1, U[1,8], U[1,8], angles "
                                    "U[60,120] deg), N per cell log-uniform in [500, 5e4], even "
                                    "cells uniform, odd clustered, +-1 charges, eps=%g"
                                    % (args.batch_systems, args.eps),
                        "unit": "particles/s"}
        for m in modes:
            out["batch"][m] = run_child(args, m, batch=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
