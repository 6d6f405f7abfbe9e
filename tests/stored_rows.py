"""Stored oracle rows of Gamma at the large workloads, and the elementwise
check against them.

tests/golden/make_oracle_samples.py writes, from the oracle alone, whole
rows of Gamma (every column of six a-triples) with each entry's magnitude
scale, c Sum_r wr r^2 Sum_mu wmu Sum_terms |S S S|.  A result agrees with a
stored entry to relative tolerance tol when |result - value| <= tol * scale:
the scale bounds what any summation order, or a relative perturbation of
each product term, can move the entry by, so the check is well posed for
entries that cancel to almost nothing and for the largest ones alike.
"""
import gzip
import os
import re

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# FP64 path: two FP64 evaluations that differ in summation order and in the
# rounding of the j_l / P_l recurrences (a few 1e-13 relative at l = 4000).
FP64_TOL = 1e-9
# mixed path: split-BF16 products lose about 3 * 2^-18 of each term
MIXED_TOL = 1e-4


def path(name: str) -> str:
    return os.path.join(GOLDEN, f"oracle_rows_{name}.txt.gz")


def load(name: str):
    """(rows, cols, values, scales) of the stored rows of a workload."""
    with gzip.open(path(name), "rt") as f:
        a = np.loadtxt(f, comments="#", ndmin=2)
    return a[:, 0].astype(np.int64), a[:, 1].astype(np.int64), a[:, 2], a[:, 3]


def worst(vals, ref, scale) -> float:
    """Largest |vals - ref| / scale over the stored entries."""
    return float((np.abs(np.asarray(vals) - ref) / scale).max())


def check(g, name: str, tol: float, label: str = "") -> float:
    """Every stored entry of workload `name` against the matrix g."""
    rows, cols, ref, scale = load(name)
    assert np.all(scale > 0)
    w = worst(g[rows, cols], ref, scale)
    print(f"{label or name}: {rows.size} stored entries, worst |G - ref| / scale = {w:.2e}")
    assert w <= tol, (label or name, w)
    return w


def load_grad(name: str):
    """The stored oracle gradient of L = Sum (Gamma * W)^2 at a workload:
    (dL/dq [np][nk] in full, {l: dL/dDelta_l(k) row}, L), written by
    tests/golden/make_oracle_samples.py grad."""
    p = os.path.join(GOLDEN, f"oracle_grad_{name}.txt.gz")
    q, d, L = {}, {}, None
    with gzip.open(p, "rt") as f:
        for line in f:
            if line.startswith("#"):
                m = re.search(r"; L = ([-+0-9.eE]+)", line)
                if m:
                    L = float(m.group(1))
                continue
            kind, i, k, v = line.split()
            (q if kind == "q" else d).setdefault(int(i), {})[int(k)] = float(v)
    nq, nk = max(q) + 1, max(q[0]) + 1
    dq = np.array([[q[i][k] for k in range(nk)] for i in range(nq)])
    rows = {l: np.array([d[l][k] for k in range(nk)]) for l in sorted(d)}
    return dq, rows, L
