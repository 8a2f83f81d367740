"""Write stored expected values of all 46 one-dimensional sectors of the
32-site square J1-J2 model (J2/J1 = 0.5, Sz = 0; 150,281,582 states, 22
sectors complex) from the fast CPU oracle alone (oracle/fast.c, pinned
against the brute-force oracle in tests/test_oracle_fast.py).

    OMP_NUM_THREADS=8 python tests/golden/make_golden_sectors32.py --steps 12

Output: tests/golden/square32_sectors.json, rewritten after every sector.
Per sector: dimension and basis checksums, and the first Lanczos
coefficients from the start vector the batched run uses (seed 2002 for
sector 0, Gamma.A1.even; 4001 + k for sector k otherwise), with the lowest
Ritz value after that many steps.  One H.x over all 46 sectors costs
minutes on 8 cores, so the runs are short.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from workloads import lattices as L  # noqa: E402
from workloads import vectors as V  # noqa: E402


def fast_for(inst):
    """Fewest sublattices the sector's group keeps stable."""
    for ns in (2, 4, 8, 16, 32):
        try:
            return O.Fast(inst, ns), ns
        except ValueError:
            pass
    raise ValueError("no stable sublattice decomposition")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, required=True)
    args = ap.parse_args()
    t0 = time.time()
    insts = L.square32_sectors()
    out = {
        "about": "32-site square J1-J2 (J2/J1 = 0.5), torus (4,4),(-4,4), Sz = 0, all 46 one-dimensional "
                 "sectors in the order of workloads.lattices.square32_sectors(); every value from the fast "
                 "CPU oracle (tests/golden/make_golden_sectors32.py)",
        "lanczos_steps": args.steps,
        "sectors": [],
    }
    path = os.path.join(HERE, "square32_sectors.json")
    for k, inst in enumerate(insts):
        F, ns = fast_for(inst)
        reps, stabs = F.basis()
        D = len(reps)
        assert D == O.character_formula_dim(inst)
        cplx = inst.is_complex
        seed = 2002 if k == 0 else 4001 + k
        v0 = V.start_vector(D, seed, cplx)
        a, b = O.lanczos(lambda v: F.apply(reps, stabs, v), v0, args.steps, hermitian_complex=cplx)
        out["sectors"].append({
            "index": k,
            "sector": inst.sector,
            "complex": bool(cplx),
            "n_sub": ns,
            "dim": int(D),
            "reps_sum_mod_2_64": int(np.sum(reps, dtype=np.uint64)),
            "reps_xor": int(np.bitwise_xor.reduce(reps)),
            "stab_sum": int(stabs.astype(np.int64).sum()),
            "lanczos_seed": seed,
            "alpha": [float(t) for t in a],
            "beta": [float(t) for t in b],
            "ritz0": float(O.tmatrix_eigs(a, b)[0]),
        })
        out["seconds"] = round(time.time() - t0, 1)
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(path + ".tmp", path)
        print(f"[{time.time() - t0:8.1f} s] sector {k} {inst.sector} dim {D} n_sub {ns}", flush=True)
        F.close()


if __name__ == "__main__":
    main()
