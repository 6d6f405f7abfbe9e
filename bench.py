"""Benchmark of the separable bispectrum projection and its adjoint on one MI355X.

One step = one forward projection Gamma (Gauss-Legendre rule, P_l table, j_l
and the k contraction, the l contraction, the triple-product quadrature, the
gather of Gamma) followed by its adjoint for the loss L = Sum (Gamma * W)^2
with W a seeded N(0,1) matrix: dL/dq_p(k) and dL/dDelta_l(k) (j_l tables
regenerated, not stored).  Inputs are seeded synthetic tables already
resident in HBM.  Prints ONE JSON line.  The default workload is the
Planck-like case: lmax = 2500, Nk = 2000, Nr = 400, Nmu = 3752, 30 + 30
one-dimensional modes, symmetric 4960 x 4960 Gamma, in the mixed precision;
the FP64 path runs beside it (one untimed and three timed steps by default)
for the speed-up and the errors.

Fields beyond the driver contract:
  roofline      the dominant kernel of the timed path (the adjoint of the
                triple-product step), measured with HIP events on the
                library's stream over the timed steps; achieved = algorithmic
                FLOPs per launch / mean launch time, against the published
                dense peak of the kernel's matrix-core type.  The split-BF16
                kernels issue three BF16 products per algorithmic term, so
                their matrix pipes are busy 3 x frac of the time
                ("mfma_pipe_frac").
  roofline_forward  the same for the forward triple-product kernel.
  cpu_baseline  the oracle (plain FP64 C, OpenMP) timed on this host on a
                bounded sample of the same workload, extrapolated by its
                exact per-unit costs.
  paths         per-precision seconds per step (mean over the timed steps,
                and their median), forward and adjoint separately,
                per-stage milliseconds, errors vs the FP64 path.  The FP64
                path runs --fp64-warmup untimed and --fp64-steps timed steps.

Other modes (their own JSON line, not the benchmark line):
  --modal3d     times Eq. (3D) (modal_gamma_3d, exact symbol) on the
                workload: seconds per call, algorithmic TFLOP/s against the
                FP64 peak, the normwise error against Eq. (2D) in FP64, and
                the error on the stored oracle rows when there are some.
  --cpu-full    times the whole oracle (every stage, every Gamma entry, and
                the adjoint unless --forward-only) on this host: the small
                workloads only.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Γ projection time (s) and MFMA TFLOP/s fraction, mixed vs FP64, at stated rel err"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6}


def unique_moments(U: int) -> int:
    """Entries T[i <= j <= k] of the symmetric third-moment tensor."""
    return U * (U + 1) * (U + 2) // 6


def algorithmic_flops(cfg) -> dict:
    """FLOPs the method has to do (an FMA counts 2), per stage.  Step d counts
    the outer-product form of Eq. (2D): one product term per output entry and
    z for N_out = Ta x N1^3 entries (all a-triples of the list against the
    ordered p-triples; Ta x Tp for the ordered lists), whatever the kernel
    computes instead (the unique moments T[i <= j <= k], about 9 % fewer at
    N1 = 30)."""
    L, U, Z = cfg.L, cfg.n1 * cfg.n1, cfg.nr * cfg.nmu
    n1 = cfg.n1
    ta = n1 ** 3 if cfg.kind == "ordered" else n1 * (n1 + 1) * (n1 + 2) // 6
    f = {
        "beta": 2.0 * cfg.n1 * cfg.nk * cfg.nr * L,
        "S": 2.0 * U * cfg.nr * L * cfg.nmu,
        "triple": 2.0 * ta * n1 ** 3 * Z,
        # adjoint: every row u against every pair v <= w, per z
        "adj_triple": 2.0 * U * (U * (U + 1) // 2) * Z,
        "adj_S": 2.0 * U * cfg.nr * L * cfg.nmu,
        "adj_beta": 2.0 * cfg.n1 * cfg.nk * cfg.nr * L + 4.0 * cfg.n1 * cfg.nk * L,
    }
    f["forward"] = f["beta"] + f["S"] + f["triple"]
    f["adjoint"] = f["adj_triple"] + f["adj_S"] + f["adj_beta"]
    f["total"] = f["forward"] + f["adjoint"]
    return f


KERNEL_SOURCES = {"k_adj_fac": "k_adjoint_fac.hip", "k_triple_bt": "k_triple_mx.hip",
                  "k_adj_fac64": "k_adjoint_fac64.hip", "k_triple_f64": "k_triple.hip"}


def code_fingerprint(path: str) -> str:
    """sha256[:16] of a source file's code: comments and white space removed,
    so that an edit of comments alone keeps a measurement valid and any edit
    of the code voids it."""
    import hashlib
    import re
    text = open(path, encoding="utf-8").read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256("".join(text.split()).encode()).hexdigest()[:16]


def measured_traffic(kernel: str, tag: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary profiles/<tag>_hbm_traffic.txt (FETCH_SIZE and WRITE_SIZE scaled
    by the copy-kernel calibration recorded there), or None when there is no
    such record or the kernel's code has changed since it was measured."""
    path = os.path.join(ROOT, "profiles", f"{tag}_hbm_traffic.txt")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    src = os.path.join(ROOT, "paper_1503_08809_amd", "csrc", KERNEL_SOURCES[kernel])
    sha = code_fingerprint(src)
    ff = wf = None
    for line in open(path):
        f = line.split()
        if f[:1] == ["calibration"]:
            ff, wf = float(f[2]), float(f[4])
        elif f[:2] == ["traffic", kernel] and ff is not None:
            if f[5] != sha:
                return None
            return (float(f[2]) * ff + float(f[3]) * wf) * 1024.0
    return None


def host_cpu() -> dict:
    """The host's CPU model and logical core count."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def cpu_full(inp, adjoint: bool) -> dict:
    """The whole oracle on this host: Gamma in full (every stage, every
    entry) and, with the adjoint, dL/dq and dL/dDelta for dL/dGamma = 2
    Gamma W^2 (the benchmark's loss).  Small workloads only."""
    from oracle import oracle as O
    from paper_1503_08809_amd import synth
    c = inp.cfg
    t0 = time.perf_counter()
    # the oracle's Gamma in full, its rows in blocks (a progress line after each)
    mu, wmu = O.gauss_legendre(c.nmu)
    S, _ = O.full_S(inp, mu)
    S = S.reshape(-1, c.nr, c.nmu)
    npm = inp.qk.shape[0]
    ta, tp = inp.tri_a, inp.tri_p
    g = np.empty((ta.shape[0], tp.shape[0]))
    nblk = 16
    for bi, rows in enumerate(np.array_split(np.arange(ta.shape[0]), nblk)):
        sidx = (ta[rows][:, None, :, None] * npm + tp[None, :, None, :]).reshape(-1, 9)
        g[rows] = O.gamma_from_S(inp, wmu, S, sidx).reshape(rows.size, tp.shape[0])
        print(f"[bench] oracle Gamma rows block {bi + 1}/{nblk}: {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    t = {"gamma": time.perf_counter() - t0}
    if adjoint:
        W = synth.loss_weights(c, g.shape[0], g.shape[1])
        t0 = time.perf_counter()
        O.gamma_full_backward(inp, 2.0 * g * W * W)
        t["adjoint"] = time.perf_counter() - t0
    out = {"value": sum(t.values()), "unit": "s", "cores": O.num_threads(), "kind": "oracle",
           "sample": "the whole workload (not sampled)", "stages_s": t}
    out.update(host_cpu())
    return out


def cpu_baseline(inp, adjoint: bool = True) -> dict:
    """Time the oracle on a bounded sample and extrapolate.

    Sample: the oracle's own stages on a slice of nr_s radial points (every
    stage's cost is linear in Nr): beta for every primordial mode, S for 9
    (a, p) pairs and Gamma for 2^16 entries; with the adjoint, the same three
    adjoint stages on the same sample.  Each measured per-unit cost is
    multiplied by the workload's unit count.
    """
    from oracle import oracle as O
    from paper_1503_08809_amd import synth
    c = inp.cfg
    nr_s = max(2, min(c.nr, 16))
    sub = synth.Inputs(c, inp.k, inp.wk, inp.r[:nr_s].copy(), inp.wr[:nr_s].copy(), inp.cl,
                       inp.delta, inp.qk, inp.ql, inp.tri_a, inp.tri_p)
    sub.cfg = dataclasses.replace(c, nr=nr_s)
    rscale = c.nr / nr_s
    U = c.n1 * c.n1
    t = {}
    t0 = time.perf_counter()
    mu, wmu = O.gauss_legendre(c.nmu)
    t["gl"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    bet = O.beta(sub)                                   # every primordial mode
    t["beta"] = (time.perf_counter() - t0) * rscale
    print("[bench] oracle sample stage beta done", file=sys.stderr, flush=True)
    pairs = [(a, p) for a in range(min(c.n1, 3)) for p in range(min(c.n1, 3))]
    t0 = time.perf_counter()
    S = O.S_pairs(sub, mu, bet, pairs)
    t["S"] = (time.perf_counter() - t0) / len(pairs) * U * rscale
    print("[bench] oracle sample stage S done", file=sys.stderr, flush=True)
    ne = 1 << 16
    rng = np.random.default_rng(0)
    sidx = rng.integers(0, len(pairs), size=(ne, 9)).astype(np.int32)
    n_entries = inp.tri_a.shape[0] * inp.tri_p.shape[0]
    t0 = time.perf_counter()
    O.gamma_from_S(sub, wmu, S, sidx)
    t["gamma"] = (time.perf_counter() - t0) / ne * n_entries * rscale
    print("[bench] oracle sample stage gamma done", file=sys.stderr, flush=True)
    sample = (f"oracle stages on {nr_s} of {c.nr} r points: beta for all modes, "
              f"S for {len(pairs)} of {U} (a,p) pairs, {ne} of {n_entries} Gamma entries")
    if adjoint:
        g = rng.standard_normal(ne)
        t0 = time.perf_counter()
        Shat = O.gamma_adjoint_S(sub, wmu, S, sidx, g)
        t["adj_gamma"] = (time.perf_counter() - t0) / ne * n_entries * rscale
        print("[bench] oracle sample stage adj_gamma done", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        bhat = O.S_adjoint(sub, mu, Shat, np.array(pairs, dtype=np.int32), c.n1)
        t["adj_S"] = (time.perf_counter() - t0) / len(pairs) * U * rscale
        print("[bench] oracle sample stage adj_S done", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        O.beta_adjoint(sub, bhat)
        t["adj_beta"] = (time.perf_counter() - t0) * rscale
        sample += "; the three adjoint stages on the same sample"
    sample += "; per-unit costs x unit counts (cost is linear in each)"
    out = {"value": sum(t.values()), "unit": "s (extrapolated)", "cores": O.num_threads(),
           "kind": "oracle", "sample": sample, "stages_s": t}
    out.update(host_cpu())
    return out


def modal3d_flops(cfg) -> float:
    """Algorithmic FLOPs of Eq. (3D) as contracted here (an FMA counts 2):
    stage 1 over the (l1, l2, l3) triples that meet the triangle and parity
    conditions, for every r and row u; stage 2 one triangle of the symmetric
    B_r per (l1, r); stage 3 the unique moments u1 <= u2 <= u3 per (l1, r)."""
    ls = np.arange(cfg.lmin, cfg.lmax + 1)
    L, U, nr = cfg.L, cfg.n1 * cfg.n1, cfg.nr
    ntri = 0
    for l1 in ls:
        lo = np.abs(l1 - ls)
        hi = np.minimum(l1 + ls, cfg.lmax)
        first = np.maximum(lo, cfg.lmin)
        first = first + ((l1 + ls + first) & 1)            # l3 of the parity of l1 + l2
        ntri += int(np.maximum(0, (hi - first) // 2 + 1).sum())
    return 2.0 * nr * U * ntri + float(L) * L * nr * U * (U + 1) + 2.0 * L * nr * unique_moments(U)


def run_modal3d(cfg, inp, reps: int) -> dict:
    """Eq. (3D) timed on the workload, checked against Eq. (2D) (FP64 path)
    and against the stored oracle rows."""
    import gzip
    import torch
    from paper_1503_08809_amd import modalproj as mp
    ctx = mp.Context(0)
    pr = mp.projection_from_inputs(ctx, inp)
    g2 = pr.gamma("fp64")
    times = []
    for i in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g3 = pr.gamma_3d("exact")
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"[bench] Eq. (3D) call {i + 1}/{reps}: {times[-1]:.2f} s", file=sys.stderr, flush=True)
    sec = float(np.mean(times))
    fl = modal3d_flops(cfg)
    out = {"mode": "modal3d", "workload": cfg.name, "s_per_call": sec, "median_s": float(np.median(times)),
           "calls": reps, "algorithmic_tflop": fl / 1e12, "achieved_tflops": fl / sec / 1e12,
           "frac_fp64_peak": fl / sec / 1e12 / PEAK_TFLOPS["fp64"],
           "normwise_err_vs_eq2d_fp64": float((g3 - g2).abs().max() / g2.abs().max())}
    path = os.path.join(ROOT, "tests", "golden", f"oracle_rows_{cfg.name}.txt.gz")
    if os.path.exists(path):
        with gzip.open(path, "rt") as f:
            a = np.loadtxt(f, comments="#", ndmin=2)
        rows, cols = a[:, 0].astype(np.int64), a[:, 1].astype(np.int64)
        g = g3.cpu().numpy()[rows, cols]
        out["stored_rows_entries"] = int(rows.size)
        out["stored_rows_err_over_scale"] = float((np.abs(g - a[:, 2]) / a[:, 3]).max())
        out["stored_rows_normwise_err"] = float(np.abs(g - a[:, 2]).max() / float(g2.abs().max()))
    ctx.close()
    return out


def measure_ceilings() -> dict:
    """What the libraries reach on this GPU, next to the datasheet peaks: a
    plain square GEMM per dtype (torch.matmul, 2-D, contiguous operands) and a
    device-to-device copy, timed with events over repeated launches."""
    import torch
    dev = torch.device("cuda", 0)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / 1e3 / reps

    out = {}
    for name, dt, n, reps in (("bf16", torch.bfloat16, 16384, 20), ("fp32", torch.float32, 8192, 10),
                              ("fp64", torch.float64, 8192, 5)):
        x = torch.randn(n, n, device=dev, dtype=torch.float32).to(dt)
        y = torch.randn(n, n, device=dev, dtype=torch.float32).to(dt)
        sec = timed(lambda: torch.matmul(x, y), reps)
        out[f"gemm_{name}_tflops"] = 2.0 * n ** 3 / sec / 1e12
        out[f"gemm_{name}_size"] = n
        del x, y
    n = 1 << 29                                               # 4 GiB of doubles
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    sec = timed(lambda: dst.copy_(src), 10)
    out["copy_gbs"] = 2.0 * n * 8 / sec / 1e9                 # bytes read + written
    out["copy_bytes"] = n * 8
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3,
                    help="workload: 1 lmax64_ordered_n8, 2 lmax500_ordered_n16, 3 lmax2500_symmetric_n30, "
                         "4 lmax1000_symmetric_n20, 5 lmax4000_symmetric_n40")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--forward-only", action="store_true", help="time Gamma without the adjoint")
    ap.add_argument("--no-fp64-ref", action="store_true",
                    help="skip the FP64 reference step (profiling runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--ceilings", action="store_true",
                    help="measure library GEMM and copy ceilings on this GPU, print them, exit")
    ap.add_argument("--fp64-steps", type=int, default=3, help="timed steps of the FP64 reference path")
    ap.add_argument("--fp64-warmup", type=int, default=1, help="untimed steps of the FP64 reference path")
    ap.add_argument("--fp64-adjoint-chunks", type=int, default=1, metavar="N",
                    help="run the FP64 adjoint as N calls on consecutive r-chunks of the grid, summed (for a "
                         "fixed dL/dGamma the gradient is a sum over r); each call then finishes in 1/N of the "
                         "time, and steps a-c are recomputed per chunk")
    ap.add_argument("--modal3d", type=int, default=0, metavar="CALLS",
                    help="time Eq. (3D) (modal_gamma_3d) over this many calls on the workload, print, exit")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the whole oracle on this host (small workloads), print, exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU r-sharding is a design, not built)", file=sys.stderr)
        return 2
    if args.ceilings:
        print(json.dumps(measure_ceilings()))
        return 0

    import torch
    from paper_1503_08809_amd import modalproj as mp
    from paper_1503_08809_amd import synth

    cfg = synth.CONFIGS[args.config]
    t0 = time.perf_counter()
    inp = synth.make_inputs(cfg)
    print(f"[bench] inputs for {cfg.name} in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    if args.cpu_full:
        if cfg.lmax > 500:
            print("bench.py: --cpu-full runs the whole oracle; use it on lmax <= 500", file=sys.stderr)
            return 2
        res = cpu_full(inp, not args.forward_only)
        res.update({"mode": "cpu_full", "workload": cfg.name})
        print(json.dumps(res))
        return 0
    if args.modal3d:
        print(json.dumps(run_modal3d(cfg, inp, args.modal3d)))
        return 0
    ctx = mp.Context(0)
    # the inputs never change: the adjoint takes the forward's tables (steps
    # a-c) instead of recomputing them, as an autograd backward would
    ctx.set_forward_reuse(True)
    pr = mp.projection_from_inputs(ctx, inp)
    out = ctx.empty(inp.tri_a.shape[0], inp.tri_p.shape[0])
    W = ctx.to_dev(synth.loss_weights(cfg, inp.tri_a.shape[0], inp.tri_p.shape[0]))
    W2 = 2.0 * W * W
    flops = algorithmic_flops(cfg)
    adjoint = not args.forward_only

    if args.copy_calibration > 0:
        n = args.copy_calibration << 17                     # doubles
        src = torch.ones(n, dtype=torch.float64, device=ctx.torch_device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {n * 8} bytes read, {n * 8} bytes written",
              file=sys.stderr, flush=True)
        del src, dst

    # the FP64 adjoint in r-chunks: projections on consecutive slices of the
    # r grid with the same per-node weights
    chunks = []
    if args.fp64_adjoint_chunks > 1:
        for idx in np.array_split(np.arange(cfg.nr), args.fp64_adjoint_chunks):
            chunks.append(mp.projection_from_inputs(ctx, inp, r=inp.r[idx].copy(), wr=inp.wr[idx].copy()))

    def backward(prec: str, dG, timed: bool):
        if prec != "fp64" or not chunks:
            g = pr.gamma_backward(dG, prec)
            return g, (ctx.stage_times() if timed else None)
        dq = dd = None
        st = {}
        for ci, prc in enumerate(chunks):
            tq = time.perf_counter()
            a, b = prc.gamma_backward(dG, prec)
            sc = ctx.stage_times()                          # waits for the stream
            dq, dd = (a, b) if dq is None else (dq + a, dd + b)
            for kname, v in sc.items():
                st[kname] = st.get(kname, 0.0) + v
            print(f"[bench] fp64 adjoint chunk {ci + 1}/{len(chunks)} ({prc.r.numel()} r): "
                  f"{time.perf_counter() - tq:.3f} s", file=sys.stderr, flush=True)
        return (dq, dd), (st if timed else None)

    def one_step(prec: str, timed: bool):
        ta = time.perf_counter()
        pr.gamma(prec, out=out)
        sf = ctx.stage_times() if timed else None          # waits for the stream
        if not timed:
            torch.cuda.synchronize()
        tb = time.perf_counter()
        print(f"[bench] {prec} forward {tb - ta:.3f} s", file=sys.stderr, flush=True)
        grads, sb = None, None
        if adjoint:
            grads, sb = backward(prec, out * W2, timed)
            if not timed:
                torch.cuda.synchronize()
        tc = time.perf_counter()
        return tb - ta, tc - tb, sf, sb, grads

    def run_path(prec: str, steps: int, warmup: int):
        ctx.enable_timing(False)
        for _ in range(warmup):
            one_step(prec, False)
        torch.cuda.synchronize()
        ctx.enable_timing(True)
        acc = {"fwd": 0.0, "adj": 0.0}
        stf, stb = {}, {}
        grads = None
        per_step = []
        t_start = time.perf_counter()
        for s in range(steps):
            tf, tb, sf, sb, grads = one_step(prec, True)
            acc["fwd"] += tf
            acc["adj"] += tb
            per_step.append(tf + tb)
            for src, dst in ((sf, stf), (sb, stb)):
                for kname, v in (src or {}).items():
                    if v:
                        dst[kname] = dst.get(kname, 0.0) + v
            print(f"[bench] {prec} step {s + 1}/{steps}: forward {tf:.3f} s, adjoint {tb:.3f} s",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        ctx.enable_timing(False)
        res = {"s_per_step": elapsed / steps, "median_s_per_step": float(np.median(per_step)),
               "steps": steps, "warmup": warmup, "forward_s": acc["fwd"] / steps,
               "adjoint_s": acc["adj"] / steps,
               "stage_ms_forward": {k: v / steps for k, v in stf.items()},
               "stage_ms_adjoint": {k: v / steps for k, v in stb.items()}}
        return res, grads

    def nerr(a, b):
        return float((a - b).abs().max() / b.abs().max())

    def elem_large(a, b):
        # elementwise relative error over the entries with |b| >= 1e-3 max|b|
        big = b.abs() >= 1e-3 * b.abs().max()
        return float(((a - b).abs()[big] / b.abs()[big]).max())

    def pct_rmse(a, b):
        # the percentage RMSE of the unit-normalised Gamma (performance section)
        return float(100.0 * ((a / a.norm() - b / b.norm()) ** 2).mean().sqrt())

    paths = {}
    main_prec = args.precision
    ref = None
    if main_prec == "fp64" or not args.no_fp64_ref:
        fp_steps = args.steps if main_prec == "fp64" else max(1, args.fp64_steps)
        fp_warm = args.warmup if main_prec == "fp64" else max(0, args.fp64_warmup)
        paths["fp64"], g64 = run_path("fp64", fp_steps, fp_warm)
        ref = (out.clone(), g64)
    if main_prec == "mixed":
        paths["mixed"], gm = run_path("mixed", args.steps, args.warmup)
        if ref is not None:
            m = paths["mixed"]
            m["gamma_normwise_err_vs_fp64"] = nerr(out, ref[0])
            m["gamma_elementwise_large_err_vs_fp64"] = elem_large(out, ref[0])
            m["gamma_pct_rmse_vs_fp64"] = pct_rmse(out, ref[0])
            if adjoint:
                m["dq_normwise_err_vs_fp64"] = nerr(gm[0], ref[1][0])
                m["ddelta_normwise_err_vs_fp64"] = nerr(gm[1], ref[1][1])
            f64 = paths["fp64"]
            m["speedup_vs_fp64"] = f64["s_per_step"] / m["s_per_step"]
            m["forward_speedup_vs_fp64"] = f64["forward_s"] / m["forward_s"]
            if adjoint:
                m["adjoint_speedup_vs_fp64"] = f64["adjoint_s"] / m["adjoint_s"]
    main = paths[main_prec]
    sec = main["s_per_step"]

    if main_prec == "fp64":
        peak, dt, pipe = PEAK_TFLOPS["fp64"], "f64", 1.0
    else:
        peak, dt, pipe = PEAK_TFLOPS["bf16"], "bf16x3+f32acc+f64", 3.0

    tag = f"{main_prec}_lmax{cfg.lmax}"

    def roof(kernel: str, stage: str, ms: float) -> dict:
        achieved = flops[stage] / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "mfma_pipe_frac": pipe * achieved / peak,
                "traffic": measured_traffic(kernel, tag), "traffic_unit": "bytes per launch",
                "kernel": kernel, "flops_per_launch": flops[stage], "mean_launch_ms": ms}

    kfwd = "k_triple_bt" if main_prec == "mixed" else "k_triple_f64"
    kadj = "k_adj_fac" if main_prec == "mixed" else "k_adj_fac64"
    r_fwd = roof(kfwd, "triple", main["stage_ms_forward"]["triple"])
    r_adj = roof(kadj, "adj_triple", main["stage_ms_adjoint"]["adj_triple"]) if adjoint else None
    dominant = r_adj if adjoint and r_adj["mean_launch_ms"] > r_fwd["mean_launch_ms"] else r_fwd

    line = {
        "metric": METRIC,
        "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": dt, "data": "synthetic",
        "config": {"workload": cfg.name + ("_forward" if not adjoint else "_forward_adjoint"),
                   "lmax": cfg.lmax, "nk": cfg.nk, "nr": cfg.nr, "nmu": cfg.nmu, "n1": cfg.n1,
                   "kind": cfg.kind, "precision": main_prec, "gamma_shape": list(out.shape),
                   "loss": "sum((Gamma * W)^2), W seeded N(0,1)" if adjoint else None},
        "algorithmic_tflop": (flops["total"] if adjoint else flops["forward"]) / 1e12,
        "achieved_tflops_total": (flops["total"] if adjoint else flops["forward"]) / sec / 1e12,
        "roofline": dominant,
        "roofline_forward": r_fwd,
        "paths": paths,
    }
    if not args.no_cpu:
        cb = cpu_baseline(inp, adjoint)
        cb["gpu_speedup"] = cb["value"] / sec
        line["cpu_baseline"] = cb
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line))
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
