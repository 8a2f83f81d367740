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
* ``sector_levels`` / ``spin_levels`` - the lowest few levels of every
  sector at Sz = S, and of them those of total spin exactly S: every level
  of spin S' > S also lies at Sz = S + 1, so a level at Sz = S below the
  lowest level of all sectors at Sz = S + 1 has spin S (this holds on any
  lattice, frustrated or not);
* ``total_spin`` - S from <S^2> = 3N/4 + 2 sum_{i<j} <S_i . S_j> of a state,
  through the expectation-value kernel with the all-pairs operator (which
  every site permutation and the spin flip leave invariant);
* ``structure_factor`` - S(q), the Fourier sum of the spin correlations (its
  value at the ordering vector measures the order: M = (pi, pi) for the
  Neel state), through the same kernel;
* ``chirality_correlation`` / ``nematic`` - the thesis's order parameters
  that tell tetrahedral from stripy order on the triangular lattice (chapter
  on the J1-J2-Jchi model): the summed scalar-chirality correlation
  X = sum_t <chi_0 chi_t> and the connected bond-bond sum
  N = sum_{b || b0} <(S.S)_b0 (S.S)_b>_c, each from products
  <A psi, B psi> of two symmetric operators applied by the library.
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


def good_ritz(alpha, beta, k, tol=1e-12):
    """Lowest k distinct eigenvalues of the Lanczos T-matrix with the
    spurious ones removed (Cullum and Willoughby's test, 1985).  Without
    reorthogonalization T acquires, besides repeated copies of converged
    eigenvalues, simple eigenvalues that belong to no eigenvalue of H; each
    of those is also an eigenvalue of T with its first row and column
    deleted, to rounding, because the start vector has no weight on it.  A
    cluster of T eigenvalues equal to 1e-8 (relative) counts once; a simple
    one closer than ``tol`` (relative to the largest |eigenvalue|) to an
    eigenvalue of the reduced matrix is dropped.

    A genuine level lies about D u^2 from the nearest eigenvalue of the
    reduced matrix, u being the start vector's weight on it and D of the
    order of the spectral width: about 1e-7 for a random start vector in a
    10^8-state sector, and now and then orders of magnitude less, while
    the spurious values sit at rounding distance.  Hence ``tol`` is at
    rounding scale, and the lowest value is always kept: T's eigenvalues
    never fall below the sector's lowest level (beyond rounding), so the
    lowest one is that level or its approximation from above, never a
    spurious value."""
    a = np.ascontiguousarray(alpha, np.float64)
    b = np.ascontiguousarray(beta, np.float64)
    n = len(a)
    lam = symed.eigenvalues(a, b, n)
    scale = max(1.0, float(np.max(np.abs(lam))))
    mu = symed.eigenvalues(a[1:], b[1:], n - 1) if n > 1 else np.zeros(0)
    out = []
    i = 0
    while i < n and len(out) < k:
        j = i + 1
        while j < n and lam[j] - lam[i] <= 1e-8 * scale:
            j += 1
        if i == 0 or j - i > 1 or len(mu) == 0 or np.min(np.abs(mu - lam[i])) > tol * scale:
            out.append(float(lam[i]))
        i = j
    return out


def sector_levels(instances, n_iter=100, k=3, mode=0, seed=1, label=None, check=10, log=None):
    """For every non-empty sector: (label, [lowest k Ritz values], drift,
    dim).  Lanczos runs min(n_iter, dim) steps from a seeded normal start
    vector without reorthogonalization; ``good_ritz`` merges the copies of
    converged levels and drops the spurious ones (one Krylov space sees each
    eigenvalue once, so a sector's own degeneracies are never resolved
    anyway).  ``drift``: largest change of the k values over the last
    ``check`` steps, a convergence measure (0 when the run spans the whole
    Krylov space: all dim steps, or a breakdown).  ``label(inst)``
    names the sector (default: its name); ``log`` receives one line per
    sector."""
    import time
    out = []
    for inst in instances:
        t0 = time.perf_counter()
        b = symed.Basis.build(inst)
        try:
            if b.dim == 0:
                continue
            if mode == 2:
                b.build_hash()
            v0 = _start(b.dim, b.is_complex, seed)
            a, beta, n, broken = b.lanczos(v0, min(n_iter, b.dim), mode=mode)
            del v0
            lv = good_ritz(a[:n], beta[:n], k)
            drift = 0.0
            # a run that spans the whole Krylov space (n = dim, or breakdown) is exact
            if n > check + k and n < b.dim and not broken:
                prev = good_ritz(a[:n - check], beta[:n - check], len(lv))
                drift = max(abs(x - y) for x, y in zip(lv, prev)) if len(prev) == len(lv) else float("inf")
            name = label(inst) if label else inst.name
            out.append((name, lv, drift, b.dim))
            if log:
                log(f"  {name:<22s} dim {b.dim:>11d}  {n:3d} steps  {time.perf_counter() - t0:6.1f} s  "
                    f"drift {drift:.1e}  " + " ".join(f"{e:.8f}" for e in lv))
        finally:
            b.free()
    return out


def spin_levels(at_s, at_s1, safety=1.0):
    """Levels of total spin exactly S, sorted: [(E, label)] from
    ``sector_levels`` output at Sz = S (``at_s``) that lie below the lowest
    level of every sector at Sz = S + 1 (``at_s1``); also that cut.  A Ritz
    value lies above the level it approximates, so each sector's value at
    Sz = S + 1 is first lowered by ``safety`` times its drift: a level of
    higher spin whose copy at Sz = S + 1 is less converged stays above the
    cut."""
    cut = min(lv[0] - safety * drift for _, lv, drift, _ in at_s1)
    return sorted((e, name) for name, lv, _, _ in at_s for e in lv if e < cut), cut


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


def _op_args(op):
    return dict(bonds=op.get("bonds"), bond_J=op.get("bond_J"), tris=op.get("tris"), tri_Jchi=op.get("tri_Jchi"))


def product_expectation(basis, psi, A, B, mode=0):
    """<psi|A B|psi> = <A psi, B psi> for Hermitian operators A and B, each
    a dict of the ``expectation`` arguments (bonds, bond_J, tris,
    tri_Jchi), both invariant under the basis's group.  The products and
    the inner product run in the library (ed_apply_op)."""
    import torch
    a = torch.empty_like(psi)
    if A is B:
        return basis.apply_op(psi, a, z=a, mode=mode, **_op_args(A))      # |A psi|^2
    basis.apply_op(psi, a, mode=mode, **_op_args(A))
    b = torch.empty_like(psi)
    return basis.apply_op(psi, b, z=a, mode=mode, **_op_args(B))


def chirality_correlation(basis, psi, up, down, c6=True, mode=0):
    """X = sum_t <chi_t0 chi_t> over all elementary triangles t (up and
    down, counter-clockwise; t0 an up triangle) of a translation-invariant
    normalized state.  Translations make it (1/N) <X_up X_all>, X_up and
    X_all the chirality sums over the up and over all triangles.  With the
    60-degree rotation in the group (``c6``), which swaps up and down
    triangles, <X_up X_all> = <X_all X_all> / 2 = |X_all psi|^2 / 2, and
    X_up need not be invariant; otherwise X_up must be."""
    up = np.asarray(up, np.int32)
    down = np.asarray(down, np.int32)
    n = len(up)
    all_ = dict(tris=np.concatenate([up, down]), tri_Jchi=np.ones(len(up) + len(down)))
    if c6:
        return product_expectation(basis, psi, all_, all_, mode).real / (2 * n)
    return product_expectation(basis, psi, dict(tris=up, tri_Jchi=np.ones(n)), all_, mode).real / n


def nematic(basis, psi, bonds, mode=0):
    """N = sum_b <(S.S)_b0 (S.S)_b>_c over the bonds b parallel to b0, of a
    translation-invariant normalized state: (<B^2> - <B>^2) / N with B the
    sum of the N bonds ``bonds`` of one direction.  B must be invariant
    under the basis's group: build the sector with the point-group elements
    that keep that direction (a state of higher symmetry lies in the
    trivial irrep of the smaller group)."""
    bonds = np.asarray(bonds, np.int32)
    Bop = dict(bonds=bonds, bond_J=np.ones(len(bonds)))
    e = basis.expectation(psi, mode=mode, **_op_args(Bop)).real
    b2 = product_expectation(basis, psi, Bop, Bop, mode).real
    return (b2 - e * e) / len(bonds)


def _main(argv=None):
    import argparse
    import time

    from workloads import lattices as L

    ap = argparse.ArgumentParser(description="Tower-of-states sweep: the low levels of every one-dimensional "
                                             "sector at Sz = S, square J1-J2 (16, 32 sites), triangular J1-J2 "
                                             "(12, 36 sites, C6v) or kagome J1-J2 (12 sites, C6v).")
    ap.add_argument("--lattice", default="square", choices=["square", "triangular", "kagome"])
    ap.add_argument("--sites", type=int, default=32, choices=[12, 16, 32, 36])
    ap.add_argument("--J2", type=float, default=0.0)
    ap.add_argument("--spins", type=int, nargs="+", default=[0, 1, 2, 3])
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--levels", type=int, default=1, help="levels per sector (more than 1: spin-resolved table)")
    ap.add_argument("--next-steps", type=int, default=0, help="steps per sector at Sz = S + 1 (spin-resolved)")
    ap.add_argument("--mode", type=int, default=0, choices=[0, 2])
    ap.add_argument("--show", type=int, default=3, help="sectors listed per S")
    ap.add_argument("--with-e", action="store_true",
                    help="spin-resolved sweep: add the sectors of the 2-D irreps (E, E1, E2)")
    ap.add_argument("--order", action="store_true",
                    help="triangular order parameters X and N of the Gamma ground state (with --Jchi)")
    ap.add_argument("--Jchi", type=float, default=0.0)
    a = ap.parse_args(argv)
    if a.order:
        if a.lattice != "triangular" or a.sites not in (12, 36):
            ap.error("--order needs --lattice triangular and --sites 12 or 36")
        _order_main(a, L)
        return
    makers = {("square", 32): L.square32_sectors, ("square", 16): L.square16_sectors,
              ("triangular", 12): L.triangular12_sectors, ("triangular", 36): L.triangular36_sectors,
              ("kagome", 12): lambda J2=0.0, n_up=None: L.kagome_sectors(L.KAG12_L, L.KAG12_CHAIN, J2=J2,
                                                                         n_up=n_up)}
    if (a.lattice, a.sites) not in makers:
        ap.error(f"no {a.sites}-site {a.lattice} cluster; available: "
                 + ", ".join(f"{lat} {n}" for lat, n in makers))
    make = makers[(a.lattice, a.sites)]
    if a.with_e and a.lattice == "kagome":
        ap.error("--with-e: no sectors of 2-D irreps for the kagome lattice")
    if a.with_e:
        geo = {("square", 32): (L.SQ32_L, L.SQ32_CHAIN), ("square", 16): (L.SQ16_L, L.SQ16_CHAIN),
               ("triangular", 12): (L.TRI12_L, L.TRI12_CHAIN),
               ("triangular", 36): (L.TRI36_L, L.TRI36_CHAIN)}[(a.lattice, a.sites)]
        base = make

        def make(J2, n_up):
            return base(J2=J2, n_up=n_up) + L.two_dim_sectors(a.lattice, geo[0], geo[1], J2=J2, n_up=n_up)

    def say(s):
        print(s, flush=True)

    if a.levels > 1:
        # spin-resolved: k levels per sector at Sz = S, lowest levels at Sz = S + 1
        for S in a.spins:
            t0 = time.perf_counter()
            say(f"Sz={S}: {a.levels} levels per sector, {a.steps} steps")
            at_s = sector_levels(make(J2=a.J2, n_up=a.sites // 2 + S), a.steps, a.levels, a.mode,
                                 label=L.sector_label, log=say)
            say(f"Sz={S + 1}: lowest level per sector, {a.next_steps or a.steps} steps")
            at_s1 = sector_levels(make(J2=a.J2, n_up=a.sites // 2 + S + 1), a.next_steps or a.steps, 1, a.mode,
                                  label=L.sector_label, log=say)
            rows, cut = spin_levels(at_s, at_s1)
            say(f"S={S}: {len(rows)} levels of spin {S} below {cut:.8f} (lowest at Sz={S + 1}), "
                f"{time.perf_counter() - t0:.1f} s")
            for e, name in rows:
                say(f"    {e:.8f}  {name}")
        return
    for S in a.spins:
        t0 = time.perf_counter()
        rows = lowest_by_spin(lambda s: make(J2=a.J2, n_up=a.sites // 2 + s), [S], a.steps, a.mode)[S]
        dt = time.perf_counter() - t0
        print(f"S={S}: {len(rows)} sectors, {dt:.1f} s", flush=True)
        for e, inst in rows[: a.show]:
            print(f"    {e:.10f}  {inst.name}", flush=True)


def _order_main(a, L):
    """X (sector of C6: chirality needs Jchi != 0, a complex sector) and N
    (sector of the point-group elements that keep a1's direction) of the
    Gamma ground state of the triangular J1-J2-Jchi model."""
    import time

    import torch
    Lt, ch = {12: (L.TRI12_L, L.TRI12_CHAIN), 36: (L.TRI36_L, L.TRI36_CHAIN)}[a.sites]

    def ground(inst):
        t0 = time.perf_counter()
        b = symed.Basis.build(inst)
        if a.mode == 2:
            b.build_hash()
        e0, psi = b.ground_state(_start(b.dim, b.is_complex, 1), min(a.steps, b.dim), mode=a.mode)
        return b, e0, psi, time.perf_counter() - t0

    if a.Jchi != 0.0:
        inst = L.triangular_j1j2chi(Lt[0], Lt[1], 1.0, a.J2, a.Jchi, L.Q0, irrep="A", flip=1, sublat_chain=ch)
        b, e0, psi, dt = ground(inst)
        up, down = L.triangles(inst)
        t0 = time.perf_counter()
        x = chirality_correlation(b, psi, up, down, c6=True, mode=a.mode)
        print(f"X: Gamma C6 sector, dim {b.dim}, E0 {e0:.10f} ({dt:.1f} s), X = {x:.8f} "
              f"({time.perf_counter() - t0:.1f} s)", flush=True)
        del psi
        b.free()
    gens = [L.TRI_C2] + ([L.TRI_MY] if a.Jchi == 0.0 else [])
    inst = L.triangular_j1j2chi(Lt[0], Lt[1], 1.0, a.J2, a.Jchi, L.Q0, irrep="A", flip=1, sublat_chain=ch,
                                pg_gens=gens)
    b, e0, psi, dt = ground(inst)
    t0 = time.perf_counter()
    nem = nematic(b, psi, L.bonds_along(inst, (1, 0)), mode=a.mode)
    print(f"N: Gamma sector of {len(inst.meta['little'])} point-group elements, dim {b.dim}, E0 {e0:.10f} "
          f"({dt:.1f} s), N = {nem:.8f} ({time.perf_counter() - t0:.1f} s)", flush=True)
    # S(q) over the whole C6v star of q (a union of orbits of the sector's group)
    pg6v = L.triangular_lattice(Lt[0], Lt[1], ch, mirrors=True).pg
    pos = L.site_coords(inst)
    h, t = L.Fraction(1, 2), L.Fraction(1, 3)
    for name, q in (("Gamma", L.Q0), ("K", (t, 2 * t)), ("M", (h, L.Fraction(0)))):
        star = L.momentum_star(inst, q, pg6v)
        print(f"   S({name}) = {structure_factor(b, psi, pos, star, mode=a.mode):.8f} (star of {len(star)})",
              flush=True)
    del psi
    b.free()
    torch.cuda.synchronize()


if __name__ == "__main__":
    _main()
