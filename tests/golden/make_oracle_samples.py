"""Write oracle values of sampled Gamma entries at the large workloads.

Gamma entries at lmax = 1000, 2500 and 4000 take the oracle seconds to minutes to
compute, too long for a GPU test run, so they are computed here, once, by
the oracle alone (oracle/ and the seeded input generator; nothing from the
HIP path) and stored as text: one line per entry, "row col value" with the
value printed to 17 significant digits.

    python tests/golden/make_oracle_samples.py [workload name ...]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_1503_08809_amd import synth               # noqa: E402

COUNT = {"lmax2500_symmetric_n30": 8, "lmax1000_symmetric_n20": 8, "lmax4000_symmetric_n40": 6}
SEED_OFFSET = 11
# Besides the seeded entries (almost all small against the largest |Gamma|),
# entries of the lowest modes, chosen by structure alone: the lowest sorted
# triples carry the most power, so these sit near the top of |Gamma| and pin
# the large entries elementwise.
STRUCTURAL = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 2)]


def path_for(name: str) -> str:
    return os.path.join(HERE, f"oracle_gamma_{name}.txt")


def main(names):
    for name in names:
        cfg = synth.workload(name)
        inp = synth.make_inputs(cfg)
        shape = (inp.tri_a.shape[0], inp.tri_p.shape[0])
        idx = synth.pick_entries(cfg, shape, COUNT[name], seed_offset=SEED_OFFSET)
        rows, cols = np.unravel_index(idx, shape)
        rows = np.concatenate([rows, [r for r, _ in STRUCTURAL]]).astype(np.int64)
        cols = np.concatenate([cols, [c for _, c in STRUCTURAL]]).astype(np.int64)
        vals = O.gamma_entries(inp, rows, cols)
        with open(path_for(name), "w") as f:
            f.write(f"# oracle Gamma entries, workload {cfg.name} (Gamma {shape[0]} x {shape[1]}),\n")
            f.write(f"# {COUNT[name]} seeded entries (synth.pick_entries, seed offset {SEED_OFFSET}), then the "
                    f"low-mode entries {STRUCTURAL};\n")
            f.write("# written by tests/golden/make_oracle_samples.py from the oracle only\n")
            f.write("# row col value\n")
            for r, c, v in zip(rows, cols, vals):
                f.write(f"{r} {c} {v:.17g}\n")
        print("wrote", path_for(name), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(COUNT))
