"""Write the stored expected values of the 32-site square sector from the
oracle alone (brute-force orbits, push-form matrix, plain Lanczos).

    OMP_NUM_THREADS=8 python tests/golden/make_golden.py

Output: tests/golden/square32_gamma_a1_even.json.  Takes about a quarter of
an hour on 8 cores (enumeration of C(32,16) configurations, then the matrix).
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


def main():
    t0 = time.time()
    inst = L.square32()
    reps, stabs = O.enumerate_basis(inst)
    D = len(reps)
    print("basis", D, round(time.time() - t0, 1), "s", flush=True)
    H = O.coo_matrix(inst, reps, stabs)
    print("matrix nnz", H.nnz, round(time.time() - t0, 1), "s", flush=True)
    n_iter = 100
    v0 = V.start_vector(D, 2002)
    a, b = O.lanczos(lambda v: H @ v, v0, n_iter)
    e100 = float(O.tmatrix_eigs(a, b)[0])
    a3, b3 = O.lanczos(lambda v: H @ v, v0, 300)
    e300 = float(O.tmatrix_eigs(a3, b3)[0])
    x = V.state_vector(reps, 4242)
    y = H @ x
    out = {
        "about": "32-site square J1-J2 (J2/J1 = 0.5), torus (4,4),(-4,4), Sz = 0, T32 x| C4v x Z2, "
                 "Gamma.A1.even; every value from the oracle (tests/golden/make_golden.py)",
        "dim": int(D),
        "reps_sum_mod_2_64": int(np.sum(reps, dtype=np.uint64)),
        "reps_xor": int(np.bitwise_xor.reduce(reps)),
        "stab_sum": int(stabs.astype(np.int64).sum()),
        "nnz": int(H.nnz),
        "lanczos_seed": 2002,
        "lanczos_steps": n_iter,
        "alpha_first10": [float(t) for t in a[:10]],
        "beta_first10": [float(t) for t in b[:10]],
        "E0_after_100": e100,
        "E0_after_300": e300,
        "hv_state_vector_seed": 4242,
        "hv_sum": float(y.sum()),
        "hv_norm2": float(np.dot(y, y)),
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "square32_gamma_a1_even.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
