"""Write oracle values of whole Gamma rows at the large workloads.

Gamma at lmax = 500, 1000, 2500 and 4000 takes the oracle minutes to hours
to compute, too long for a GPU test run, so whole rows of it are computed
here, once, by the oracle alone (oracle/ and the seeded input generator;
nothing from the HIP path) and stored as gzipped text, one line per entry:

    row col value scale

value is Gamma[row, col] and scale is the oracle's magnitude scale of that
entry, c Sum_r wr r^2 Sum_mu wmu Sum_terms |S S S| (Eq. (2D) taken over the
absolute values of its product terms): an elementwise check compares
|Gamma - value| with a tolerance times scale, which is well posed for
entries that cancel to nearly zero as well as for the largest ones.

Rows: every column (every p-triple) of six a-triples chosen by structure,
the lowest modes (0,0,0), (0,0,1), a triple of three distinct low modes,
one seeded row, three distinct high modes (N1-3, N1-2, N1-1) and the
highest (N1-1, N1-1, N1-1); for the ordered lists the distinct low triple
is (2, 1, 0), whose order differs from the sorted one.

    python tests/golden/make_oracle_samples.py [workload name ...]
    python tests/golden/make_oracle_samples.py grad     (the lmax = 1000 gradient)
"""
import gzip
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_1503_08809_amd import synth               # noqa: E402

WORKLOADS = ["lmax500_ordered_n16", "lmax1000_symmetric_n20", "lmax2500_symmetric_n30",
             "lmax4000_symmetric_n40"]
SEED_OFFSET = 11


def path_for(name: str) -> str:
    return os.path.join(HERE, f"oracle_rows_{name}.txt.gz")


def row_of(tri: np.ndarray, t) -> int:
    hit = np.nonzero((tri == np.asarray(t, dtype=tri.dtype)).all(axis=1))[0]
    if hit.size != 1:
        raise ValueError(f"triple {t} not in the mode list")
    return int(hit[0])


def chosen_rows(cfg, tri: np.ndarray):
    n = cfg.n1
    low3 = (2, 1, 0) if cfg.kind == "ordered" else (0, 1, 2)
    fixed = [row_of(tri, t) for t in [(0, 0, 0), (0, 0, 1), low3, (n - 3, n - 2, n - 1),
                                      (n - 1, n - 1, n - 1)]]
    rng = np.random.Generator(np.random.PCG64(cfg.pick_seed + SEED_OFFSET))
    while True:
        seeded = int(rng.integers(0, tri.shape[0]))
        if seeded not in fixed:
            break
    return sorted(fixed + [seeded])


def main(names):
    for name in names:
        t0 = time.time()
        cfg = synth.workload(name)
        inp = synth.make_inputs(cfg)
        ta, tp = inp.tri_a.shape[0], inp.tri_p.shape[0]
        rows_sel = chosen_rows(cfg, inp.tri_a)
        rows = np.repeat(np.asarray(rows_sel, dtype=np.int64), tp)
        cols = np.tile(np.arange(tp, dtype=np.int64), len(rows_sel))
        vals, scale = O.gamma_entries(inp, rows, cols, return_scale=True)
        with gzip.open(path_for(name), "wt") as f:
            f.write(f"# oracle Gamma rows, workload {cfg.name} (Gamma {ta} x {tp}),\n")
            f.write(f"# rows {rows_sel} (a-triples {[tuple(int(v) for v in inp.tri_a[r]) for r in rows_sel]}),"
                    f" every column\n")
            f.write("# written by tests/golden/make_oracle_samples.py from the oracle only\n")
            f.write("# row col value scale (scale = c Sum_r wr r^2 Sum_mu wmu Sum_terms |S S S|)\n")
            for r, c, v, s in zip(rows, cols, vals, scale):
                f.write(f"{r} {c} {v:.17g} {s:.17g}\n")
        print(f"wrote {path_for(name)} ({rows.size} entries, {time.time() - t0:.0f} s)", flush=True)


# ---- the gradient at lmax = 1000 ------------------------------------------
# The loss of the forward + adjoint workload, L = Sum (Gamma * W)^2 with W the
# seeded N(0,1) matrix of synth.loss_weights: the oracle's full Gamma, then
# its adjoint for dL/dGamma = 2 Gamma W^2.  Stored: all of dL/dq [np][nk] and
# the rows dL/dDelta_l(k) for l in GRAD_L (every k), "kind index k value".
GRAD_WORKLOAD = "lmax1000_symmetric_n20"
GRAD_L = [2, 3, 4, 10, 50, 100, 200, 333, 500, 501, 640, 777, 900, 950, 990, 998, 999, 1000]


def grad_path(name: str) -> str:
    return os.path.join(HERE, f"oracle_grad_{name}.txt.gz")


def main_grad(name: str = GRAD_WORKLOAD):
    t0 = time.time()
    cfg = synth.workload(name)
    inp = synth.make_inputs(cfg)
    g = O.gamma_full(inp)
    print(f"oracle Gamma {g.shape} in {time.time() - t0:.0f} s", flush=True)
    W = synth.loss_weights(cfg, g.shape[0], g.shape[1])
    dq, dd = O.gamma_full_backward(inp, 2.0 * g * W * W)
    with gzip.open(grad_path(name), "wt") as f:
        f.write(f"# oracle gradient of L = Sum (Gamma * W)^2 (W = synth.loss_weights), workload {cfg.name}\n")
        f.write(f"# all of dL/dq [{dq.shape[0]}][{dq.shape[1]}] ('q p k value'), and dL/dDelta_l(k) for l in "
                f"{GRAD_L} ('d l k value'); L = {float(((g * W) ** 2).sum()):.17g}\n")
        f.write("# written by tests/golden/make_oracle_samples.py from the oracle only\n")
        for p in range(dq.shape[0]):
            for k in range(dq.shape[1]):
                f.write(f"q {p} {k} {dq[p, k]:.17g}\n")
        for l in GRAD_L:
            for k in range(dd.shape[1]):
                f.write(f"d {l} {k} {dd[l - cfg.lmin, k]:.17g}\n")
    print(f"wrote {grad_path(name)} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args == ["grad"]:
        main_grad()
    else:
        main(args or WORKLOADS)
