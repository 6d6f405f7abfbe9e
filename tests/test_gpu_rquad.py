"""Accuracy of the r rules in Gamma against the number of r nodes (the
integrator study of the performance section, Fig. integrator-error, on
synthetic inputs).

Workload: lmax = 500, Nk = 1000, 8 modes per dimension (120 x 120 symmetric
Gamma), FP64 path, r on the fixed interval r* +- 4 sigma (r* = 14000,
sigma = 300) with nested grids of n nodes, so that every n integrates the
same interval:
  uniform:  r* + sigma (-4 + 8 j / (n - 1));
  quantile: r* + sigma Phi^-1(p_lo + (p_hi - p_lo) j / (n - 1)), clustered on
            r* like the workloads' grids, with intervals in the tails that
            shrink only slowly with n.
The reference is the Hermite rule at n = 6401 on the same family.  Error:
percentage RMSE of the unit-normalised Gamma,
100 sqrt(mean((G / |G|_F - G_ref / |G_ref|_F)^2)).

Bars, from the orders of the rules: on the uniform grid the trapezium's
error falls 4x per halving (second order) and the Hermite rule's about 8x
(third order) until the FP64 floor (~1e-13 %); on the quantile grid the
trapezium still falls 4x per halving and the Hermite rule stays below it,
but stalls near 1e-9 %, the share of Gamma in the sparse tails.
"""
import time

import numpy as np
import pytest
from scipy.special import ndtr, ndtri

from paper_1503_08809_amd import synth

pytestmark = pytest.mark.gpu

SIGMA = 300.0
COUNTS = (51, 101, 201, 401, 801)
REF_N = 6401


def nodes(grid, n):
    if grid == "uniform":
        return synth.R_STAR + SIGMA * np.linspace(-4.0, 4.0, n)
    p = ndtr(-4.0) + (ndtr(4.0) - ndtr(-4.0)) * np.linspace(0.0, 1.0, n)
    return synth.R_STAR + SIGMA * ndtri(p)


def pct_rmse(g, ref):
    a = g / np.linalg.norm(g)
    b = ref / np.linalg.norm(ref)
    return 100.0 * float(np.sqrt(np.mean((a - b) ** 2)))


@pytest.fixture(scope="module")
def study():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_08809_amd import modalproj as mp
    cfg = synth.small_config(lmax=500, nk=1000, nr=2, n1=8, kind="symmetric", kmin=1e-5,
                             kmax=0.1, k_damp=0.02, l_damp=400.0, seed_index=94)
    inp = synth.make_inputs(cfg)
    ctx = mp.Context(0)

    def gamma(grid, rule, n):
        r = nodes(grid, n)
        pr = mp.projection_from_inputs(ctx, inp, r=r, wr=mp.r_weights(rule, r))
        pr.gamma("fp64")
        torch.cuda.synchronize()
        t = time.perf_counter()
        g = pr.gamma("fp64")
        torch.cuda.synchronize()
        return g.cpu().numpy(), time.perf_counter() - t

    out = {}
    for grid in ("uniform", "quantile"):
        ref, _ = gamma(grid, "hermite", REF_N)
        for rule in ("trapezoid", "hermite"):
            for n in COUNTS:
                g, dt = gamma(grid, rule, n)
                out[grid, rule, n] = pct_rmse(g, ref)
                print(f"{grid:8s} {rule:9s} n = {n:4d}: {out[grid, rule, n]:.3e} % RMSE, "
                      f"{dt * 1e3:.1f} ms", flush=True)
    ctx.close()
    return out


def _ratios(study, grid, rule, counts):
    e = [study[grid, rule, n] for n in counts]
    return [a / b for a, b in zip(e, e[1:])]


def test_uniform_grid_orders(study):
    rt = _ratios(study, "uniform", "trapezoid", (101, 201, 401))
    rh = _ratios(study, "uniform", "hermite", (101, 201, 401))
    assert all(3.5 < x < 4.5 for x in rt), rt
    assert all(x > 6.0 for x in rh), rh
    assert all(study["uniform", "hermite", n] <= study["uniform", "trapezoid", n] for n in COUNTS[1:])
    assert study["uniform", "hermite", 401] <= 1e-12


def test_quantile_grid(study):
    rt = _ratios(study, "quantile", "trapezoid", (51, 101, 201, 401))
    assert all(3.5 < x < 4.5 for x in rt), rt
    assert all(study["quantile", "hermite", n] < study["quantile", "trapezoid", n] for n in COUNTS)
    assert max(study["quantile", "hermite", n] for n in COUNTS) <= 1e-7
