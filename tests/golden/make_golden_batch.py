"""Write the stored expected values of the smallest complex sector of the
32-site square batch (all one-dimensional sectors of the J1-J2 model,
J2/J1 = 0.5, Sz = 0) from the oracle alone: brute-force orbits, push-form
matrix, plain complex Lanczos.

    OMP_NUM_THREADS=8 python tests/golden/make_golden_batch.py

Output: tests/golden/square32_batch_complex.json.  The sector is number 10
of workloads.lattices.square32_sectors() (momentum (0, 1/4), little-group
irrep 1, flip even; 4,689,460 states, complex characters); its start vector
is the batch's, seed 4001 + 10.  Takes about half an hour on 8 cores.
"""
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

SECTOR = 10


def main():
    t0 = time.time()
    inst = L.square32_sectors()[SECTOR]
    assert inst.is_complex
    reps, stabs = O.enumerate_basis(inst)
    D = len(reps)
    print("basis", D, round(time.time() - t0, 1), "s", flush=True)
    H = O.coo_matrix(inst, reps, stabs)
    print("matrix nnz", H.nnz, round(time.time() - t0, 1), "s", flush=True)
    n_iter = 100
    seed = 4001 + SECTOR
    v0 = V.start_vector(D, seed, True)
    a, b = O.lanczos(lambda v: H @ v, v0, n_iter, hermitian_complex=True)
    e100 = float(O.tmatrix_eigs(a, b)[0])
    print("E0 after 100", repr(e100), round(time.time() - t0, 1), "s", flush=True)
    out = {
        "about": "32-site square J1-J2 (J2/J1 = 0.5), torus (4,4),(-4,4), Sz = 0, sector "
                 f"{inst.sector} (number {SECTOR} of the 46 one-dimensional sectors, complex characters); "
                 "every value from the oracle (tests/golden/make_golden_batch.py)",
        "sector_index": SECTOR,
        "sector": inst.sector,
        "dim": int(D),
        "reps_sum_mod_2_64": int(np.sum(reps, dtype=np.uint64)),
        "reps_xor": int(np.bitwise_xor.reduce(reps)),
        "stab_sum": int(stabs.astype(np.int64).sum()),
        "nnz": int(H.nnz),
        "lanczos_seed": seed,
        "lanczos_steps": n_iter,
        "alpha_first10": [float(t) for t in a[:10]],
        "beta_first10": [float(t) for t in b[:10]],
        "E0_after_100": e100,
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "square32_batch_complex.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
