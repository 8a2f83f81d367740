"""Tower-of-states sweeps and order diagnostics (host orchestration only).

The thesis reads magnetic order off the low-energy spectrum: the lowest
level of every total spin S, labelled by momentum and point-group irrep,
must carry the irreps and multiplicities that the symmetry analysis of the
ordered state predicts (appendix on the tower of states; for the square
lattice Neel antiferromagnet the lowest level of even S lies in Gamma.A1 and
of odd S in M.A1).

This module only strings library calls together; every H.v, Lanczos step,
Ritz vector and expectation value runs in the HIP kernels behind the C ABI.

* ``sector_lowest`` - lowest Lanczos eigenvalue of each sector;
* ``lowest_by_spin`` - for S = 0, 1, ... the sectors at Sz = S, sorted by
  their lowest level.  For a Hamiltonian whose lowest level rises with S
  (Lieb-Mattis, bipartite antiferromagnets) the lowest level at Sz = S has
  total spin exactly S, so the head of each list is the S-th level of the
  tower;
* ``total_spin`` - S from <S^2> = 3N/4 + 2 sum_{i<j} <S_i . S_j> of a state,
  through the expectation-value kernel with the all-pairs operator (which
  every site permutation and the spin flip leave invariant);
* ``structure_factor`` - S(q), the Fourier sum of the spin correlations (its
  value at the ordering vector measures the order: M = (pi, pi) for the
  Neel state), through the same kernel.
"""
from __future__ import annotations

import math

import numpy as np

from . import symed


def _start(dim, is_complex, seed):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    dt = torch.complex128 if is_complex else torch.float64
    return torch.randn(dim, dtype=dt, device="cuda", generator=g)


def sector_lowest(instances, n_iter=100, mode=0, seed=1, k=1):
    """[(E_0, ..., E_{k-1}), instance] for every non-empty sector: Lanczos
    from a seeded normal start vector, lowest k eigenvalues of T.  mode 0
    (plain lookup) or 2 (hashed table, built per sector)."""
    out = []
    for inst in instances:
        b = symed.Basis.build(inst)
        try:
            if b.dim == 0:
                continue
            if mode == 2:
                b.build_hash()
            v0 = _start(b.dim, b.is_complex, seed)
            a, beta, n, _ = b.lanczos(v0, min(n_iter, b.dim), mode=mode)
            ev = symed.eigenvalues(a[:n], beta[:n], min(k, n))
            out.append((tuple(float(e) for e in ev), inst))
        finally:
            b.free()
    return out


def lowest_by_spin(make_sectors, spins, n_iter=100, mode=0, seed=1):
    """{S: [(E0, instance), ...] sorted by E0} over the sectors
    ``make_sectors(S)`` at Sz = S."""
    table = {}
    for S in spins:
        rows = [(e[0], inst) for e, inst in sector_lowest(make_sectors(S), n_iter, mode, seed)]
        rows.sort(key=lambda r: r[0])
        table[S] = rows
    return table


def all_pairs(n_sites):
    """Bonds (i, j), i < j, of every pair of sites, coupling 1."""
    ij = np.array([(i, j) for i in range(n_sites) for j in range(i + 1, n_sites)], np.int32)
    return ij, np.ones(len(ij))


def total_spin(basis, psi, mode=0):
    """(S, S(S+1)) of a normalized state from <S^2>."""
    n = basis.info()["n_sites"]
    bonds, J = all_pairs(n)
    ss = 0.75 * n + 2.0 * basis.expectation(psi, bonds, J, mode=mode).real
    return 0.5 * (math.sqrt(1.0 + 4.0 * max(ss, 0.0)) - 1.0), ss


def structure_factor(basis, psi, coords, qs, mode=0):
    """Spin structure factor S(q) = (1/N) sum_{i,j} exp(i q.(r_i - r_j))
    <S_i . S_j> of a normalized state, averaged over the momenta ``qs``:
    3/4 + (2/N) sum_{i<j} <cos(2 pi q.(r_i - r_j))>_qs <S_i . S_j>, one call of
    the expectation kernel.  ``coords``: lattice coordinates of the sites;
    ``qs``: q in the matching reciprocal units, and with it every momentum
    the basis's point group maps it to (its star), so that the operator is
    invariant.  For a state of full point symmetry every q of a star gives
    the same S(q)."""
    r = np.asarray(coords, float)
    n = len(r)
    bonds, _ = all_pairs(n)
    d = r[bonds[:, 0]] - r[bonds[:, 1]]
    Q = np.array([[float(c) for c in q] for q in qs], float)
    J = (2.0 / n) * np.cos(2.0 * np.pi * (d @ Q.T)).mean(axis=1)
    return 0.75 + basis.expectation(psi, bonds, J, mode=mode).real


def _main(argv=None):
    import argparse
    import time

    from workloads import lattices as L

    ap = argparse.ArgumentParser(description="Tower-of-states sweep of the square Heisenberg (J1-J2) model: the "
                                             "lowest level of every one-dimensional sector at Sz = S.")
    ap.add_argument("--sites", type=int, default=32, choices=[16, 32])
    ap.add_argument("--J2", type=float, default=0.0)
    ap.add_argument("--spins", type=int, nargs="+", default=[0, 1, 2, 3])
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--mode", type=int, default=0, choices=[0, 2])
    ap.add_argument("--show", type=int, default=3, help="sectors listed per S")
    a = ap.parse_args(argv)
    make = L.square32_sectors if a.sites == 32 else L.square16_sectors
    for S in a.spins:
        t0 = time.perf_counter()
        rows = lowest_by_spin(lambda s: make(J2=a.J2, n_up=a.sites // 2 + s), [S], a.steps, a.mode)[S]
        dt = time.perf_counter() - t0
        print(f"S={S}: {len(rows)} sectors, {dt:.1f} s", flush=True)
        for e, inst in rows[: a.show]:
            print(f"    {e:.10f}  {inst.name}", flush=True)


if __name__ == "__main__":
    _main()
