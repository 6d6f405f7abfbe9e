"""Benchmark of the separable bispectrum projection on one MI355X.

One step = one whole projection (Gauss-Legendre rule, P_l table, j_l and the
k contraction, the l contraction, the triple-product quadrature and the
gather of Gamma) over seeded synthetic inputs already resident in HBM.
Prints ONE JSON line (rank 0).  The default workload is the Planck-like
case: lmax = 2500, Nk = 2000, Nr = 400, Nmu = 3752, 30 + 30 one-dimensional
modes, symmetric 4960 x 4960 Gamma.

Fields beyond the driver contract:
  roofline      the dominant kernel (the triple-product quadrature) measured
                with HIP events on the library's stream over the timed steps;
                achieved = algorithmic FLOPs per launch / mean launch time.
  cpu_baseline  the oracle (plain FP64 C, OpenMP) timed on this host on a
                bounded sample of the same workload, extrapolated to the
                whole projection by its exact per-unit costs.
  paths         per-precision seconds per projection, errors vs the FP64 path.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6}
HBM_GBS = 8000.0


def unique_moments(U: int) -> int:
    """Entries T[i <= j <= k] of the symmetric third-moment tensor."""
    return U * (U + 1) * (U + 2) // 6


def algorithmic_flops(cfg) -> dict:
    """FLOPs the method has to do (an FMA counts 2)."""
    L, U = cfg.L, cfg.n1 * cfg.n1
    fb = 2.0 * cfg.n1 * cfg.nk * cfg.nr * L
    fc = 2.0 * U * cfg.nr * L * cfg.nmu
    fd = 2.0 * unique_moments(U) * cfg.nr * cfg.nmu
    return {"beta": fb, "S": fc, "triple": fd, "total": fb + fc + fd}


def cpu_baseline(inp, max_seconds: float = 25.0) -> dict:
    """Time the oracle on a bounded sample and extrapolate.

    Sample: the oracle's own stages on a slice of nr_s radial points (the
    oracle's cost is linear in Nr): beta for every primordial mode, S for a
    few (a, p) pairs and Gamma for a block of entries.  Each measured per-unit
    cost is multiplied by the workload's unit count.
    """
    from oracle import oracle as O
    from paper_1503_08809_amd import synth
    c = inp.cfg
    nr_s = max(2, min(c.nr, 16))
    sub = synth.Inputs(c, inp.k, inp.wk, inp.r[:nr_s].copy(), inp.wr[:nr_s].copy(), inp.cl,
                       inp.delta, inp.qk, inp.ql, inp.tri_a, inp.tri_p)
    import dataclasses
    sub_cfg = dataclasses.replace(c, nr=nr_s)
    sub.cfg = sub_cfg
    t0 = time.perf_counter()
    mu, wmu = O.gauss_legendre(c.nmu)
    t_gl = time.perf_counter() - t0
    t0 = time.perf_counter()
    bet = O.beta(sub)                                   # every primordial mode
    t_beta = (time.perf_counter() - t0) * (c.nr / nr_s)
    pairs = [(a, p) for a in range(min(c.n1, 3)) for p in range(min(c.n1, 3))]
    t0 = time.perf_counter()
    S = O.S_pairs(sub, mu, bet, pairs)
    t_s = (time.perf_counter() - t0) / len(pairs) * (c.n1 * c.n1) * (c.nr / nr_s)
    ne = 1 << 16
    rng = np.random.default_rng(0)
    sidx = rng.integers(0, len(pairs), size=(ne, 9)).astype(np.int32)
    t0 = time.perf_counter()
    O.gamma_from_S(sub, wmu, S, sidx)
    t_g1 = time.perf_counter() - t0
    n_entries = inp.tri_a.shape[0] * inp.tri_p.shape[0]
    t_d = t_g1 / ne * n_entries * (c.nr / nr_s)
    total = t_gl + t_beta + t_s + t_d
    return {
        "value": total, "unit": "s (extrapolated)", "cores": O.num_threads(), "kind": "oracle",
        "sample": (f"oracle stages on {nr_s} of {c.nr} r points: beta for all modes, "
                   f"S for {len(pairs)} of {c.n1 * c.n1} (a,p) pairs, {ne} of {n_entries} "
                   "Gamma entries; per-unit costs x unit counts (cost is linear in each)"),
        "stages_s": {"gl": t_gl, "beta": t_beta, "S": t_s, "gamma": t_d},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3, help="workload 1..5")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU r-sharding is a design, not built)", file=sys.stderr)
        return 2

    import torch
    from paper_1503_08809_amd import modalproj as mp
    from paper_1503_08809_amd import synth

    cfg = synth.CONFIGS[args.config]
    t0 = time.perf_counter()
    inp = synth.make_inputs(cfg)
    print(f"[bench] inputs for {cfg.name} in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    ctx = mp.Context(0)
    pr = mp.projection_from_inputs(ctx, inp)
    out = ctx.empty(inp.tri_a.shape[0], inp.tri_p.shape[0])
    flops = algorithmic_flops(cfg)

    def run_path(prec: str, steps: int, warmup: int):
        ctx.enable_timing(False)
        for _ in range(warmup):
            pr.gamma(prec, out=out)
        torch.cuda.synchronize()
        ctx.enable_timing(True)
        stage_sum = {}
        t_start = time.perf_counter()
        for s in range(steps):
            pr.gamma(prec, out=out)
            st = ctx.stage_times()          # waits for the stream
            for kname, v in st.items():
                stage_sum[kname] = stage_sum.get(kname, 0.0) + v
            print(f"[bench] {prec} step {s + 1}/{steps} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        ctx.enable_timing(False)
        return elapsed / steps, {k: v / steps for k, v in stage_sum.items()}

    paths = {}
    sec64, st64 = run_path("fp64", args.steps if args.precision == "fp64" else 1,
                           args.warmup if args.precision == "fp64" else 0)
    g64 = out.clone()
    paths["fp64"] = {"s_per_projection": sec64, "stage_ms": st64}
    main_prec = args.precision
    if main_prec == "mixed":
        secm, stm = run_path("mixed", args.steps, args.warmup)
        err = float((out - g64).abs().max() / g64.abs().max())
        paths["mixed"] = {"s_per_projection": secm, "stage_ms": stm,
                          "normwise_err_vs_fp64": err, "speedup_vs_fp64": sec64 / secm}
    sec, stages = paths[main_prec]["s_per_projection"], paths[main_prec]["stage_ms"]

    triple_ms = stages["triple"]
    achieved = flops["triple"] / (triple_ms * 1e-3) / 1e12
    if main_prec == "fp64":
        peak, dt = PEAK_TFLOPS["fp64"], "f64"
    else:
        peak, dt = PEAK_TFLOPS["bf16"] / 3.0, "bf16x3+f32acc+f64"
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": None, "kernel": "k_triple",
            "flops_per_launch": flops["triple"], "mean_launch_ms": triple_ms}

    line = {
        "metric": "Gamma projection time (s) at lmax=2500 and MFMA TFLOP/s fraction",
        "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": cfg.name, "lmax": cfg.lmax, "nk": cfg.nk, "nr": cfg.nr,
                   "nmu": cfg.nmu, "n1": cfg.n1, "kind": cfg.kind, "precision": main_prec,
                   "gamma_shape": list(out.shape)},
        "algorithmic_tflop": flops["total"] / 1e12,
        "achieved_tflops_total": flops["total"] / sec / 1e12,
        "roofline": roof,
        "paths": paths,
    }
    if not args.no_cpu:
        cb = cpu_baseline(inp)
        cb["gpu_speedup"] = cb["value"] / sec
        line["cpu_baseline"] = cb
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line))
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
