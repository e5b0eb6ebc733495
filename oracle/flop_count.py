"""Writes profiles/flops_per_cell.json: the algorithmic FP64 flops per interior
cell that roofline fractions use, counted by the oracle's op-counting scalar
(oracle_flops_per_cell: add, sub, mul, div, sqrt, cbrt, exp, pow one each;
constants folded; only the operations the outputs depend on).

TEST AND MEASUREMENT INFRASTRUCTURE: run by hand after a change to the
oracle's arithmetic (``python -m oracle.flop_count``); a CPU test checks that
the stored numbers are still the oracle's.  The count does not depend on the
data as long as no input value is degenerate, so a 4^3 box of a puncture with
a small seeded perturbation on every field stands in for each workload."""
from __future__ import annotations

import json
import os

import numpy as np

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "profiles", "flops_per_cell.json")

# the parameter sets the benchmark reports (names as in the bench line)
CASES = {
    "full_theory": {},
    "full_theory_shift_advection": {"shift_advec": 1.0},
    "decoupled": {"decoupled": 1.0},
    "sixth_order": {"fd_order": 6.0},
}


def generic_state(n=4, dx=0.25, seed=5):
    from paper_2309_06225_amd import inputs as I
    u = I.single_puncture(n, dx)
    rng = np.random.default_rng(seed)
    u = u + 1e-3 * rng.standard_normal(u.shape)
    return I.wrap_ghosts(u)


def counts() -> dict:
    from paper_2309_06225_amd import inputs as I
    u = generic_state()
    out = {}
    for name, over in CASES.items():
        c = O.flops_per_cell(I.params_vector(I.default_params(**over)), u, 0.25)
        out[name] = {k: float(v) for k, v in c.items()}
    return out


def main():
    O.build(force=False)
    data = {"convention": "oracle op-counting scalar: add, sub, mul, div, sqrt, cbrt, exp, pow = 1; "
                          "constants folded; additions of 0 and products with 0 or +-1 free; dead values not counted",
            "per_cell": counts()}
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    print(json.dumps(data, indent=1))


if __name__ == "__main__":
    main()
