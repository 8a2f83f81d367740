#!/usr/bin/env python3
"""Benchmark: H.v elements/s and seconds per Lanczos step on one MI355X.

Workload (default): 40-site square-lattice J1-J2 Heisenberg model (J2/J1 =
0.5) on the torus (6,2),(-2,6), Sz = 0, symmetry group T(40) x| C4 x Z2
(|G| = 320), sector Gamma.A.even, dimension 430,909,650.  FP64 vectors; the
Lanczos start vector is seeded N(0,1) (PCG64, seed 5002) in canonical basis
order.  A "step" is one Lanczos iteration: the graph-replayed H.v with the
fused w <- Hv - beta w epilogue, the alpha/beta reductions, the axpy and the
rotate/scale.  Basis construction and learned-index training are set-up and
are reported separately.

Prints one JSON line (see keys below).  Only one GPU is used; --gpus > 1
exits with a message.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks used for the roofline
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="square40", choices=["square40", "square32", "triangular36", "chain16"])
    ap.add_argument("--lookup", default="both", choices=["plain", "learned", "both"])
    ap.add_argument("--apply-reps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this size first (calibrates HBM byte counters)")
    return ap.parse_args()


def workload(name):
    from workloads import lattices as L
    if name == "square40":
        return L.square40(), ("square40 J1-J2 (J2/J1=0.5) torus (6,2),(-2,6), Sz=0, T40 x| C4 x Z2, Gamma.A.even",
                              5002)
    if name == "square32":
        return L.square32(), ("square32 J1-J2 (J2/J1=0.5) torus (4,4),(-4,4), Sz=0, T32 x| C4v x Z2, Gamma.A1.even",
                              2002)
    if name == "triangular36":
        return L.tri36_K(), ("triangular36 J1-J2-Jchi (0.1, 0.2) 6x6, Sz=0, T36 x| C3 x Z2, K.A.even", 3002)
    return L.chain16(), ("chain16 Heisenberg, Sz=0, T16, k=0", 1002)


def cpu_baseline(inst, budget_s):
    """The oracle (brute-force orbits, plain definition) on a bounded sample
    of rows of the same sector, timed on the host cores."""
    from oracle import oracle as O
    from workloads import vectors as V
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    # calibrate on a small sample, then run a sample sized to the budget
    n = 256
    st = V.random_sector_states(inst.n_sites, inst.n_up, n, 77)
    rep, g, stab, triv = O.rep_many(inst, st)
    rows = np.unique(rep[triv])
    t0 = time.perf_counter()
    O.row_entries(inst, rows)
    t_cal = max(time.perf_counter() - t0, 1e-3)
    n_rows = int(max(32, min(200000, len(rows) * budget_s / t_cal)))
    st = V.random_sector_states(inst.n_sites, inst.n_up, int(n_rows * 1.3) + 8, 78)
    rep, g, stab, triv = O.rep_many(inst, st)
    rows = np.unique(rep[triv])[:n_rows]
    t0 = time.perf_counter()
    rp, tgt, coef, ok, ne = O.row_entries(inst, rows)
    t = time.perf_counter() - t0
    elements = int(ne.sum())
    return {"value": elements / t, "unit": "elements/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(rows)} oracle-sampled sector rows of the same sector ({elements} elements, "
                      f"brute-force orbits, pull form), {t:.1f} s on {cores} host threads",
            "rows_per_s": len(rows) / t}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one MI355X; --gpus {args.gpus} is not supported in this build "
              f"(the multi-GPU design is described in DESIGN.md but not implemented).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2210_03511_amd import symed as S
    from workloads import vectors as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    inst, (desc, seed) = workload(args.config)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    basis = S.Basis.build(inst)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = basis.info()
    D = info["dim"]
    cplx = bool(info["is_complex"])
    modes = []
    train = None
    if args.lookup in ("plain", "both"):
        modes.append(0)
    if args.lookup in ("learned", "both") and hasattr(S.lib(), "ed_index_train"):
        t0 = time.perf_counter()
        train = basis.train_index()
        train["wall_seconds"] = time.perf_counter() - t0
        modes.append(1)
        info = basis.info()

    v0 = V.start_vector(D, seed, cplx)
    v0t = torch.from_numpy(v0).cuda()
    del v0
    y = torch.empty_like(v0t)

    # H.v timing per lookup mode (HIP events on the launch stream)
    stream = torch.cuda.current_stream()
    apply_t = {}
    for m in modes:
        basis.apply_H(v0t, y, mode=m)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.apply_reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            basis.apply_H(v0t, y, mode=m)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        apply_t[m] = float(np.mean(ts))
    del y

    # Lanczos steps: warmup, then exactly K timed steps per mode
    step_t = {}
    energies = {}
    for m in modes:
        if args.warmup > 0:
            basis.lanczos(v0t, args.warmup, mode=m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a, b, n, broken = basis.lanczos(v0t, args.steps, mode=m)
        torch.cuda.synchronize()
        step_t[m] = (time.perf_counter() - t0) / max(n, 1)
        energies[m] = float(S.eigenvalues(a, b, 1)[0])

    best = min(modes, key=lambda m: step_t[m])
    n_el = info["n_elements"]
    n_off = info["n_offdiag"]
    vb = 16 if cplx else 8
    # algorithmic bytes of one H.v launch: per row rep (8) + stabilizer code
    # (2) + x_i + y_i; per off-diagonal element x_j + rep_j
    alg_bytes = D * (8 + 2 + 2 * vb) + n_off * (vb + 8)
    t_apply = apply_t[best]
    achieved = alg_bytes / t_apply / 1e9
    out = {
        "metric": "H.v elements/s & s per Lanczos step, 40-site square: learned vs plain lookup",
        "value": n_el / step_t[best],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_t[best] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if cplx else "f64",
        "data": "synthetic (seeded N(0,1) start vector; deterministic lattice)",
        "config": {"workload": desc, "dim": D, "n_elements_per_Hv": n_el, "lookup": "learned" if best == 1 else "plain",
                   "n_sub_rep": info["n_sub_rep"], "n_sub_act": info["n_sub_act"],
                   "prefix_bits": info["prefix_bits"], "parallelism": "single GPU"},
        "elements_per_s_Hv": {("learned" if m == 1 else "plain"): n_el / apply_t[m] for m in modes},
        "s_per_step": {("learned" if m == 1 else "plain"): step_t[m] for m in modes},
        "rows_per_s_Hv": D / t_apply,
        "lanczos_E0_after_steps": {("learned" if m == 1 else "plain"): energies[m] for m in modes},
        "setup": {"basis_build_s": t_build, "table_bytes": info["table_bytes"],
                  "limits_bytes": info["limits_bytes"], "device_bytes": info["bytes_device"]},
        "search_window_keys": {"plain_mean": info["limits_mean_window"], "plain_max": info["limits_max_window"],
                               "learned_mean": train["mean_window"] if train else None,
                               "learned_max": train["max_err"] if train else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_apply", "alg_bytes_per_launch": alg_bytes, "avg_launch_s": t_apply},
    }
    if train is not None:
        out["learned_index"] = train
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
