"""Tower-of-states sweeps through the C ABI.

* 16 sites: the lowest level of every one-dimensional sector at Sz = 0..3,
  from the HIP Lanczos, equals the oracle's dense lowest eigenvalue, and the
  lowest level of each S carries the irrep of the Neel tower-of-states table.
* 32 sites (the thesis's cluster of that table): the same sweep over all
  one-dimensional sectors at Sz = 0..3 puts the lowest level of each S in
  the table's irrep, each level of spin S reappears at Sz < S (an SU(2)
  multiplet), and the Ritz vectors of these levels have <S^2> = S(S+1) from
  the expectation-value kernel with the all-pairs operator.
* 12-site triangular (C6v): the lowest four levels of every sector at
  Sz = 0..3 (Lanczos, spurious Ritz values removed by the Cullum-Willoughby
  test) equal the oracle's dense spectra, and the spin-resolved levels
  built from them hold the 120-degree tower table's irreps and
  multiplicities for S = 0, 1, 2; the sectors of the 2-D irreps (E1, E2 at
  Gamma, E at K) give the oracle's levels too; with chirality (J2 = 0.2,
  Jchi = 0.5, point group C6) the spin-resolved levels hold the tetrahedral
  tower table for S = 0..3.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from workloads import lattices as L

pytestmark = pytest.mark.gpu

_ALL = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))
GOLD = _ALL["tos_neel_square"]
GOLD120 = _ALL["tos_120_triangular"]
GOLDTET = _ALL["tos_tetrahedral_triangular"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def T():
    _torch()
    from paper_2210_03511_amd import symed, tower
    symed.lib()
    return tower


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _label(inst):
    q = tuple(float(c) for c in inst.meta["q"])
    name = {(0.0, 0.0): "Gamma", (0.5, 0.5): "M"}.get(q, str(q))
    return f"{name}.A1" if inst.meta["irrep"] == 0 else f"{name}.ir{inst.meta['irrep']}"


def test_tower_square16_equals_oracle_and_neel_table(T):
    table = T.lowest_by_spin(lambda S: L.square16_sectors(J2=0.0, n_up=8 + S), GOLD["S"], n_iter=120)
    for S in GOLD["S"]:
        rows = table[S]
        _say("square16 S", S, [(round(e, 6), _label(i)) for e, i in rows[:3]])
        for e, inst in rows:
            reps, stabs = O.enumerate_basis(inst)
            exact = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())[0]
            assert abs(e - exact) <= 1e-10 * abs(exact), inst.name
        expect = [k for k, m in GOLD["multiplicity"].items() if m[GOLD["S"].index(S)] == 1]
        assert [_label(rows[0][1])] == expect
    lows = [table[S][0][0] for S in GOLD["S"]]
    assert all(a < b for a, b in zip(lows, lows[1:]))


def test_tower_square32_neel_table(T):
    spins = GOLD["S"]
    table = T.lowest_by_spin(lambda S: L.square32_sectors(J2=0.0, n_up=16 + S), spins, n_iter=60)
    lows = []
    for S in spins:
        rows = table[S]
        _say("square32 S", S, [(round(e, 8), _label(i)) for e, i in rows[:3]])
        expect = [k for k, m in GOLD["multiplicity"].items() if m[spins.index(S)] == 1]
        assert [_label(rows[0][1])] == expect
        assert rows[1][0] > rows[0][0] + 1e-3
        lows.append(rows[0][0])
        if S > 0:
            # the spin-S level is also a level of every Sz < S, in the same irrep
            prev = [(e, _label(i)) for e, i in table[S - 1]]
            assert any(abs(e - rows[0][0]) < 1e-7 and lab == _label(rows[0][1]) for e, lab in prev)
    assert all(a < b for a, b in zip(lows, lows[1:]))


def test_tower_triangular12_equals_oracle_and_120_table(T):
    k = 4
    at, labels = {}, {}
    for sz in range(4):
        secs = L.triangular12_sectors(J2=0.0, n_up=6 + sz)
        at[sz] = T.sector_levels(secs, n_iter=200, k=k)
        for inst in secs:
            labels[inst.name] = L.sector_label(inst)
            reps, stabs = O.enumerate_basis(inst)
            if not len(reps):
                continue
            w = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())
            exact = [e for i, e in enumerate(w) if i == 0 or e - w[i - 1] > 1e-8][:k]
            got = next(lv for name, lv, _, _ in at[sz] if name == inst.name)
            # the lowest level converges fully; the higher ones of the
            # tiniest sectors (n_iter = dim) keep a rounding error near 1e-8
            assert len(got) == len(exact) and abs(got[0] - exact[0]) < 1e-10, inst.name
            assert np.allclose(got, exact, rtol=0, atol=1e-7), inst.name
    for S in GOLD120["S"][:3]:
        rows, cut = T.spin_levels(at[S], at[S + 1])
        rows = [(e, labels[name]) for e, name in rows]
        m = {lab: c[GOLD120["S"].index(S)] for lab, c in GOLD120["multiplicity"].items()}
        n = sum(m.values())
        _say("triangular12 S", S, "cut", round(cut, 6), [(round(e, 6), lab) for e, lab in rows[:n + 1]])
        assert sorted(lab for _, lab in rows[:n]) == sorted(lab for lab, c in m.items() for _ in range(c))
        # a gap above the tower: the next spin-S level, or the cut if no other
        # level lies below it
        nxt = rows[n][0] if len(rows) > n else cut
        assert nxt > rows[n - 1][0] + 0.1


def test_tower_triangular12_tetrahedral_table(T):
    k = 4
    at, labels = {}, {}
    for sz in range(5):
        secs = L.triangular_chiral_sectors(L.TRI12_L, L.TRI12_CHAIN, J2=0.2, Jchi=0.5, n_up=6 + sz)
        at[sz] = T.sector_levels(secs, n_iter=200, k=k)
        for inst in secs:
            labels[inst.name] = L.sector_label(inst)
            reps, stabs = O.enumerate_basis(inst)
            if not len(reps):
                continue
            w = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())
            exact = [e for i, e in enumerate(w) if i == 0 or e - w[i - 1] > 1e-8][:k]
            got = next(lv for name, lv, _, _ in at[sz] if name == inst.name)
            assert len(got) == len(exact) and abs(got[0] - exact[0]) < 1e-10, inst.name
            assert np.allclose(got, exact, rtol=0, atol=1e-7), inst.name
    for S in GOLDTET["S"]:
        rows, cut = T.spin_levels(at[S], at[S + 1])
        rows = [(e, labels[name]) for e, name in rows]
        m = {lab: c[GOLDTET["S"].index(S)] for lab, c in GOLDTET["multiplicity"].items()}
        n = sum(m.values())
        _say("tetrahedral12 S", S, "cut", round(cut, 6), [(round(e, 6), lab) for e, lab in rows[:n + 1]])
        assert sorted(lab for _, lab in rows[:n]) == sorted(lab for lab, c in m.items() for _ in range(c))
        nxt = rows[n][0] if len(rows) > n else cut
        assert nxt > rows[n - 1][0] + 0.2


def test_two_dim_irrep_sectors_equal_oracle(T):
    k = 4
    for sz in (0, 1):
        secs = L.two_dim_sectors("triangular", L.TRI12_L, L.TRI12_CHAIN, J2=0.1, n_up=6 + sz)
        got = T.sector_levels(secs, n_iter=200, k=k, label=L.sector_label)
        assert [g[0] for g in got] == [L.sector_label(i) for i in secs if len(O.enumerate_basis(i)[0])]
        for (name, lv, _, _), inst in zip(got, [i for i in secs if len(O.enumerate_basis(i)[0])]):
            reps, stabs = O.enumerate_basis(inst)
            w = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())
            exact = [e for i, e in enumerate(w) if i == 0 or e - w[i - 1] > 1e-8][:k]
            _say("triangular12 Sz", sz, name, [round(e, 8) for e in lv])
            assert len(lv) == len(exact) and abs(lv[0] - exact[0]) < 1e-10, inst.name
            assert np.allclose(lv, exact, rtol=0, atol=1e-7), inst.name


def test_tower_square32_levels_and_total_spin(T):
    from paper_2210_03511_amd import symed
    torch = _torch()
    M = (L.F(1, 2), L.F(1, 2))
    e_prev = -np.inf
    for S in GOLD["S"]:
        q = L.Q0 if S % 2 == 0 else M
        inst = L.square_j1j2(L.SQ32_L[0], L.SQ32_L[1], 1.0, 0.0, q, irrep="A1", flip=1 if S == 0 else None,
                             sublat_chain=L.SQ32_CHAIN, n_up=16 + S)
        b = symed.Basis.build(inst)
        g = torch.Generator(device="cuda")
        g.manual_seed(100 + S)
        v0 = torch.randn(b.dim, dtype=torch.float64, device="cuda", generator=g)
        e0, psi = b.ground_state(v0, 90)
        s_val, ss = T.total_spin(b, psi)
        _say("square32", _label(inst), "Sz", S, "dim", b.dim, "E0", e0, "S(S+1)", ss)
        assert ss == pytest.approx(S * (S + 1), abs=1e-6)
        assert round(s_val) == S
        assert e0 > e_prev
        e_prev = e0
        del psi, v0
        b.free()


def _ground(symed, torch, inst, n_iter, seed):
    b = symed.Basis.build(inst)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    dt = torch.complex128 if inst.is_complex else torch.float64
    v0 = torch.randn(b.dim, dtype=dt, device="cuda", generator=g)
    e0, psi = b.ground_state(v0, min(n_iter, b.dim))
    return b, e0, psi


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_structure_factor_square16_equals_oracle(T, J2):
    """S(q) of the 16-site ground state (Gamma.A1.even) through the
    expectation kernel against the oracle's correlations of the dense
    full-Sz-sector ground state, at M, at the star of X and at Gamma."""
    from paper_2210_03511_amd import symed
    torch = _torch()
    inst = L.square_j1j2(L.SQ16_L[0], L.SQ16_L[1], 1.0, J2, L.Q0, sublat_chain=L.SQ16_CHAIN)
    b, e0, psi = _ground(symed, torch, inst, 120, 7)
    states, H = O.unsym_sector_matrix(inst)
    w, v = np.linalg.eigh(H.toarray())
    assert w[1] > w[0] + 1e-6 and abs(e0 - w[0]) < 1e-10
    C = O.spin_correlations(inst, states, v[:, 0])
    pos = L.site_coords(inst)
    for q in [L.Q0, (L.F(1, 2), L.F(1, 2)), (L.F(1, 2), L.F(0)), (L.F(1, 4), L.F(0))]:
        star = L.momentum_star(inst, q)
        exact = np.mean([O.structure_factor(C, pos, qq) for qq in star])
        got = T.structure_factor(b, psi, pos, star)
        _say("square16 J2", J2, "q", [str(c) for c in q], "star", len(star), "S", got, "oracle", exact)
        assert abs(got - exact) < 1e-8      # Ritz-vector accuracy
    b.free()


def test_structure_factor_square32_frustration(T):
    """Neel correlations at 32 sites: S(M) is largest at J2 = 0 and is
    suppressed by the frustrating J2 = 0.5; the singlet has S(Gamma) = 0."""
    from paper_2210_03511_amd import symed
    torch = _torch()
    M = (L.F(1, 2), L.F(1, 2))
    sm = {}
    for J2 in (0.0, 0.5):
        inst = L.square32(J2=J2)
        b, e0, psi = _ground(symed, torch, inst, 120, 11)
        pos = L.site_coords(inst)
        sm[J2] = T.structure_factor(b, psi, pos, L.momentum_star(inst, M))
        s0 = T.structure_factor(b, psi, pos, [L.Q0])
        _say("square32 J2", J2, "E0", e0, "S(M)", sm[J2], "S(Gamma)", s0)
        assert abs(s0) < 1e-6
        b.free()
    assert sm[0.0] > sm[0.5] > 0.75


def test_tower_kagome12_sector_levels_equal_oracle(T):
    """Every one-dimensional sector of the 12-site kagome J1-J2-J3 model at
    Sz = 0 and 1: the sweep's lowest level equals the oracle's dense
    spectrum.  (Higher levels are not compared: these sectors hold 8-100
    states, the sweep stops at dim steps without reorthogonalization, and a
    pair of levels 0.008 apart in the 24-state Sz = 1 Gamma.A1 sector is
    then not always resolved.)  The spin-0 levels below the Sz = 1 cut are
    levels of the dense Sz = 0 spectra."""
    at, dense = {}, {}
    for sz in (0, 1):
        secs = L.kagome_sectors(L.KAG12_L, L.KAG12_CHAIN, J2=0.2, J3=0.1, n_up=6 + sz)
        at[sz] = T.sector_levels(secs, n_iter=200, k=3)
        for inst in secs:
            reps, stabs = O.enumerate_basis(inst)
            if not len(reps):
                continue
            w = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())
            dense[inst.name] = w
            got = next(lv for name, lv, _, _ in at[sz] if name == inst.name)
            assert abs(got[0] - w[0]) < 1e-10, inst.name
    rows, cut = T.spin_levels(at[0], at[1])
    _say("kagome12 S 0 cut", round(cut, 6), [(round(e, 6), n) for e, n in rows[:4]])
    assert len(rows) >= 1 and all(e < cut for e, _ in rows)
    assert all(np.min(np.abs(dense[n] - e)) < 1e-8 for e, n in rows[:2])
