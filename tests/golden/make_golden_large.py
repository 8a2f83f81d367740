"""Write stored expected values of the 36-site triangular K sector and the
40-site square Gamma.A.even sector from the fast CPU oracle alone
(oracle/fast.c: the thesis's sublattice-coding method on the host, pinned
against the brute-force oracle in tests/test_oracle_fast.py).

    OMP_NUM_THREADS=8 python tests/golden/make_golden_large.py tri36 --steps 12
    OMP_NUM_THREADS=8 python tests/golden/make_golden_large.py square40 --steps 3

Output: tests/golden/triangular36_K.json, tests/golden/square40_gamma_a_even.json.
Stored per sector:
  - dimension and checksums of the basis;
  - one whole-vector H.x with x(s) = state_vector(s, 4242): sum, squared
    norm, <x, Hx>, and y on every row whose index is a multiple of the stride;
  - the first Lanczos coefficients from start_vector(dim, seed) and the
    lowest Ritz value after that many steps.
Each H.x costs minutes at 36 sites and about 20 minutes at 40 sites on 8
cores, so the Lanczos runs are short.
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

SECTORS = {
    "tri36": (L.tri36_K, 4, 3002, 1 << 16, "triangular36_K.json",
              "36-site triangular J1-J2-Jchi (J2 = 0.1, Jchi = 0.2), K point, Sz = 0, complex"),
    "square40": (L.square40, 4, 5002, 1 << 20, "square40_gamma_a_even.json",
                 "40-site square J1-J2 (J2/J1 = 0.5), Gamma.A.even, Sz = 0"),
}


def _c(z):
    z = complex(z)
    return [z.real, z.imag]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("sector", choices=sorted(SECTORS))
    ap.add_argument("--steps", type=int, required=True)
    args = ap.parse_args()
    make, n_sub, seed, stride, fname, about = SECTORS[args.sector]
    t0 = time.time()

    def say(*a):
        print(f"[{time.time() - t0:8.1f} s]", *a, flush=True)

    inst = make()
    F = O.Fast(inst, n_sub)
    reps, stabs = F.basis()
    D = len(reps)
    say("basis", D)
    assert D == O.character_formula_dim(inst)
    cplx = inst.is_complex
    out = {
        "about": about + "; every value from the fast CPU oracle (tests/golden/make_golden_large.py)",
        "n_sub": n_sub,
        "dim": int(D),
        "reps_sum_mod_2_64": int(np.sum(reps, dtype=np.uint64)),
        "reps_xor": int(np.bitwise_xor.reduce(reps)),
        "stab_sum": int(stabs.astype(np.int64).sum()),
    }
    x = V.state_vector(reps, 4242, cplx)
    y = F.apply(reps, stabs, x)
    say("H.x done")
    idx = np.arange(0, D, stride)
    out.update({
        "hv_state_vector_seed": 4242,
        "hv_sum": _c(y.sum()),
        "hv_norm2": float(np.vdot(y, y).real),
        "hv_xHx": float(np.vdot(x, y).real),
        "hv_stride": stride,
        "hv_rows": [_c(t) for t in y[idx]] if cplx else [float(t) for t in y[idx]],
    })
    del x, y
    calls = [0]

    def mv(v):
        calls[0] += 1
        r = F.apply(reps, stabs, v)
        say("Lanczos H.v", calls[0])
        return r

    v0 = V.start_vector(D, seed, cplx)
    a, b = O.lanczos(mv, v0, args.steps, hermitian_complex=cplx)
    out.update({
        "lanczos_seed": seed,
        "lanczos_steps": len(a),
        "alpha": [float(t) for t in a],
        "beta": [float(t) for t in b],
        "ritz0": float(O.tmatrix_eigs(a, b)[0]),
        "seconds": round(time.time() - t0, 1),
    })
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
    say("wrote", fname)


if __name__ == "__main__":
    main()
