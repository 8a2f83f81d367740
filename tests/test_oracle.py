"""Pins of the CPU oracle against facts the thesis and the mathematics fix.

Every check here is independent of the oracle's own formulas: worked
examples printed in the thesis, closed forms, a Kronecker-product
construction from spin matrices, the character formula, projector-built
symmetric vectors and finite differences.
"""
import numpy as np
import pytest
import scipy.sparse

from oracle import oracle as O
from workloads import lattices as L

import json
import os

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


def _state(bits):
    """'uudu' -> integer, first site = most significant bit, up = 1."""
    v = 0
    for c in bits:
        v = (v << 1) | (1 if c == "u" else 0)
    return v


# --- encoding and the exchange example ("Representing Hilbert spaces") ------

def test_integer_encoding_example():
    g = GOLD["encoding"]
    assert _state(g["state"]) == g["value"]


def test_exchange_example_kron_and_terms():
    g = GOLD["exchange"]
    a, b = (k - 1 for k in g["pair_one_based"])
    inst = L.Instance("pair", g["n_sites"], np.array([[a, b]], np.int32), np.array([1.0]),
                      np.zeros((0, 3), np.int32), np.zeros(0), 3, np.arange(4, dtype=np.int32)[None],
                      np.zeros(1, np.uint8), np.ones(1, complex), [1])
    H = O.kron_hamiltonian(inst).toarray()
    assert H[g["to"], g["from"]] == pytest.approx(g["amplitude"])
    assert H[g["from"], g["to"]] == pytest.approx(g["amplitude"])
    rp, tgt, coef, ok, ne = O.row_entries(inst, np.array([g["from"]], np.uint64))
    entries = {int(t): c for t, c in zip(tgt, coef)}
    assert entries[g["to"]] == pytest.approx(g["amplitude"])
    # Ising piece: the pair is up, down -> -1/4
    assert entries[g["from"]] == pytest.approx(-0.25)
    assert ne[0] == 2


def test_two_site_singlet_triplet():
    # S.S = -3/4 (singlet), +1/4 (triplet)
    inst = L.Instance("dimer", 2, np.array([[0, 1]], np.int32), np.array([1.0]), np.zeros((0, 3), np.int32),
                      np.zeros(0), 1, np.arange(2, dtype=np.int32)[None], np.zeros(1, np.uint8),
                      np.ones(1, complex), [1])
    ev = np.linalg.eigvalsh(O.kron_hamiltonian(inst).toarray())
    assert np.allclose(ev, [-0.75, 0.25, 0.25, 0.25])
    _, Hs = O.unsym_sector_matrix(inst)
    assert np.allclose(np.linalg.eigvalsh(Hs.toarray()), [-0.75, 0.25])


def test_triangle_ising_counts():
    # J sum sigma_i sigma_j on a triangle (sigma = +-1): 6 states at -J, 2 at 3J
    inst = L.Instance("tri", 3, np.array([[0, 1], [1, 2], [2, 0]], np.int32), np.ones(3),
                      np.zeros((0, 3), np.int32), np.zeros(0), 0, np.arange(3, dtype=np.int32)[None],
                      np.zeros(1, np.uint8), np.ones(1, complex), [1])
    diag = []
    for s in range(8):
        rp, tgt, coef, ok, ne = O.row_entries(inst, np.array([s], np.uint64))
        d = [c for t, c in zip(tgt, coef) if int(t) == s]
        diag.append(4 * d[0].real if d else 0.0)  # S^z S^z = sigma sigma / 4
    assert sorted(np.round(diag, 12)) == [-1] * 6 + [3] * 2


def test_four_site_ring_ground_state():
    # E0 = -2J for the periodic 4-site Heisenberg ring (k = 0)
    inst = L.chain(4)
    reps, stabs = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps, stabs).toarray()
    assert np.linalg.eigvalsh(H)[0] == pytest.approx(-2.0, abs=1e-13)
    full = np.linalg.eigvalsh(O.kron_hamiltonian(inst).toarray())
    assert full[0] == pytest.approx(-2.0, abs=1e-13)


# --- sublattice-coding worked examples (section "Sublattice coding") --------

def test_two_sublattice_example_representative():
    g = GOLD["two_sublattice"]
    inst = L.chain(g["n_sites"], sublat=(2,))
    assert inst.meta["positions"] == g["chain_positions_by_label"]
    s = _state(g["state"])
    rep, gm, st, tv = O.rep_many(inst, np.array([s], np.uint64))
    assert int(rep[0]) == _state(g["representative_state"]) == g["representative"]
    assert int(gm[0]) == g["g"]
    assert O.act(inst, g["g"], s) == g["representative"]


def test_three_sublattice_example_representative():
    g = GOLD["three_sublattice"]
    inst = L.chain(g["n_sites"], sublat=(3,))
    assert inst.meta["positions"] == g["chain_positions_by_label"]
    s = _state(g["state"])
    rep, gm, st, tv = O.rep_many(inst, np.array([s], np.uint64))
    assert int(rep[0]) == _state(g["representative_state"]) == g["representative"]
    assert int(gm[0]) == g["g"]
    # the other candidate printed in the example is larger
    oc = g["other_candidate"]
    assert O.act(inst, oc["g"], s) == _state(oc["state"]) > g["representative"]


# --- enumeration vs the character formula -----------------------------------

@pytest.mark.parametrize("inst", L.small_instances(), ids=lambda i: f"{i.name}-{i.sector}")
def test_dimension_equals_character_formula(inst):
    reps, stabs = O.enumerate_basis(inst)
    assert len(reps) == O.character_formula_dim(inst)
    assert np.all(np.diff(reps.astype(np.float64)) > 0)
    # stabilizer sizes divide the group order
    assert np.all(inst.n_elem % stabs == 0)


def test_enumeration_trivial_group_is_sz_sector():
    inst = L.chain(10, n_up=4)
    from dataclasses import replace
    triv = replace(inst, perms=np.arange(10, dtype=np.int32)[None], flips=np.zeros(1, np.uint8),
                   chi=np.ones(1, complex))
    reps, _ = O.enumerate_basis(triv)
    assert np.array_equal(reps, O.sz_states(10, 4))


def test_named_sector_dimensions():
    # character formula at the benchmark sizes (exact integers)
    assert O.character_formula_dim(L.chain16()) == 810
    assert O.character_formula_dim(L.square32()) == 1184480
    assert O.character_formula_dim(L.tri36_K()) == 42018826
    assert O.character_formula_dim(L.square40()) == 430909650
    dims = [O.character_formula_dim(s) for s in L.square32_sectors()]
    assert len(dims) == 46 and sum(dims) == 150281582


# --- Hamiltonian: unsymmetrized terms vs spin matrices ----------------------

@pytest.mark.parametrize("inst", [i for i in L.small_instances() if i.n_sites <= 12],
                         ids=lambda i: f"{i.name}-{i.sector}")
def test_sector_terms_match_kronecker(inst):
    states, Hs = O.unsym_sector_matrix(inst)
    Hk = O.kron_hamiltonian(inst)
    idx = states.astype(np.int64)
    ref = Hk[idx][:, idx].toarray()
    assert np.max(np.abs(Hs.toarray() - ref)) < 1e-13


# --- symmetrized matrix vs projector-built symmetric vectors ----------------

@pytest.mark.parametrize("inst", [i for i in L.small_instances() if i.n_sites <= 16],
                         ids=lambda i: f"{i.name}-{i.sector}")
def test_symmetrized_matrix_equals_projection(inst):
    reps, stabs = O.enumerate_basis(inst)
    Hsym = O.coo_matrix(inst, reps, stabs).toarray()
    states, Hs = O.unsym_sector_matrix(inst)
    B = O.projector_basis(inst, reps, states)
    ref = B.conj().T @ (Hs @ B)
    assert np.max(np.abs(Hsym - ref)) < 1e-12
    # hermitian, and projected basis orthonormal
    assert np.max(np.abs(Hsym - Hsym.conj().T)) < 1e-12
    assert np.max(np.abs(B.conj().T @ B - np.eye(len(reps)))) < 1e-12


@pytest.mark.parametrize("inst", [i for i in L.small_instances() if i.n_sites <= 16],
                         ids=lambda i: f"{i.name}-{i.sector}")
def test_push_equals_pull(inst):
    reps, stabs = O.enumerate_basis(inst)
    Hsym = O.coo_matrix(inst, reps, stabs)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(len(reps)) + (1j * rng.standard_normal(len(reps)) if inst.is_complex else 0)
    lut = {int(s): x[i] for i, s in enumerate(reps)}
    y_pull, ok, _ = O.rows_apply(inst, reps, lambda t: np.array([lut[int(v)] for v in t]))
    assert ok.all()
    assert np.max(np.abs(Hsym @ x - y_pull)) < 1e-13


def test_union_of_sector_spectra_is_full_spectrum():
    # abelian group (translations x flip): sector spectra partition the Sz=0 spectrum
    n = 10
    allev = []
    for k in range(n):
        for fl in (1, -1):
            inst = L.chain(n, k=k, flip=fl, sublat=(2,))
            reps, stabs = O.enumerate_basis(inst)
            if len(reps):
                allev.extend(np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray()))
    _, Hs = O.unsym_sector_matrix(L.chain(n))
    full = np.linalg.eigvalsh(Hs.toarray())
    assert len(allev) == len(full)
    assert np.max(np.abs(np.sort(allev) - full)) < 1e-12


def test_su2_multiplets_and_flip_parity():
    # Sz=1 levels are a subset of Sz=0 levels; flip parity of |S,0> is (-1)^(S+N/2)
    n = 12
    i0 = L.chain(n, k=0, n_up=6, sublat=(2,))
    i1 = L.chain(n, k=0, n_up=7, sublat=(2,))
    e0 = np.linalg.eigvalsh(O.coo_matrix(i0, *O.enumerate_basis(i0)).toarray())
    e1 = np.linalg.eigvalsh(O.coo_matrix(i1, *O.enumerate_basis(i1)).toarray())
    for e in e1:
        assert np.min(np.abs(e0 - e)) < 1e-10
    # singlet ground state (S=0) lives in flip parity (-1)^(N/2) = +1 for N=12
    ev = {}
    for fl in (1, -1):
        inst = L.chain(n, k=0, flip=fl, sublat=(2,))
        ev[fl] = np.linalg.eigvalsh(O.coo_matrix(inst, *O.enumerate_basis(inst)).toarray())[0]
    assert ev[1] < ev[-1]
    assert ev[1] == pytest.approx(e0[0], abs=1e-12)


# --- Lanczos ------------------------------------------------------------------

@pytest.mark.parametrize("inst", [L.chain16(), L.small_instances()[13], L.small_instances()[15]],
                         ids=lambda i: f"{i.name}-{i.sector}")
def test_lanczos_lowest_eigenvalue(inst):
    reps, stabs = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps, stabs)
    rng = np.random.default_rng(11)
    v0 = rng.standard_normal(len(reps))
    if inst.is_complex:
        v0 = v0 + 1j * rng.standard_normal(len(reps))
    a, b = O.lanczos(lambda v: H @ v, v0, 120, hermitian_complex=inst.is_complex)
    e = O.tmatrix_eigs(a, b)[0]
    exact = np.linalg.eigvalsh(H.toarray())[0]
    assert abs(e - exact) <= 1e-10 * abs(exact)


def test_lanczos_breakdown_on_tiny_sector():
    inst = L.chain(4)
    reps, stabs = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps, stabs).toarray()
    a, b = O.lanczos(lambda v: H @ v, np.array([1.0, 0.3]), 10)
    assert len(a) == 2 and b[-1] < 1e-12
    assert np.allclose(np.sort(O.tmatrix_eigs(a, b)), [-2.0, 1.0])


def test_chain16_ground_state_value():
    # k = 0 sector of the 16-site Heisenberg ring: Lanczos vs full diagonalization
    inst = L.chain16()
    reps, stabs = O.enumerate_basis(inst)
    assert len(reps) == 810
    H = O.coo_matrix(inst, reps, stabs).toarray()
    e0 = np.linalg.eigvalsh(H)[0]
    # the full Sz=0 spectrum contains the same level
    _, Hs = O.unsym_sector_matrix(inst)
    full0 = scipy.sparse.linalg.eigsh(Hs, k=1, which="SA")[0][0]
    assert e0 == pytest.approx(full0, abs=1e-10)


# --- tower of states ------------------------------------------------------------

def _tos_label(inst):
    q = tuple(inst.meta["q"])
    name = {(0, 0): "Gamma", (0.5, 0.5): "M"}.get((float(q[0]), float(q[1])), str(q))
    return f"{name}.A1" if inst.meta["irrep"] == 0 else f"{name}.ir{inst.meta['irrep']}"


def test_tower_of_states_square16_neel_table():
    """The lowest level of each total spin S of the 4 x 4 Heisenberg
    antiferromagnet carries the irrep the thesis's Neel tower-of-states table
    assigns to it (Gamma.A1 for even S, M.A1 for odd S).  The lowest level at
    Sz = S is the lowest of spin S because E_min(Sz) rises with Sz; the
    minimum over the one-dimensional sectors equals the full Sz-sector
    minimum, so no two-dimensional irrep holds a lower level."""
    g = GOLD["tos_neel_square"]
    emin = []
    for S in g["S"]:
        rows = []
        for inst in L.square16_sectors(J2=0.0, n_up=8 + S):
            reps, stabs = O.enumerate_basis(inst)
            if len(reps):
                rows.append((np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())[0], inst))
        rows.sort(key=lambda r: r[0])
        e0, inst0 = rows[0]
        expect = [k for k, m in g["multiplicity"].items() if m[g["S"].index(S)] == 1]
        assert [_tos_label(inst0)] == expect
        assert rows[1][0] > e0 + 1e-6                      # the lowest level is not degenerate across sectors
        _, Hs = O.unsym_sector_matrix(inst0)               # same model and Sz, trivial group
        full0 = scipy.sparse.linalg.eigsh(Hs, k=1, which="SA")[0][0]
        assert e0 == pytest.approx(full0, abs=1e-9)
        emin.append(e0)
    assert all(a < b for a, b in zip(emin, emin[1:]))


def _minus(a, b, tol=1e-8):
    """Multiset difference of two eigenvalue lists: the levels of a left after
    one matching level (within tol) is taken out for every level of b."""
    left = sorted(a)
    for x in b:
        k = int(np.argmin(np.abs(np.array(left) - x)))
        assert abs(left[k] - x) < tol
        left.pop(k)
    return left


def test_tower_of_states_triangular12_120_table():
    """The 12-site triangular Heisenberg antiferromagnet (C6v cluster with
    the K points): its lowest levels of total spin S = 0, 1, 2 carry exactly
    the irreps and multiplicities of the thesis's 120-degree tower table
    (S = 3 needs a sublattice spin of at least 3, i.e. 18 sites or more), a
    clear gap separates them from the next spin-S level, and the
    unsymmetrized Sz spectra hold the same levels with K.A1 twice (K and K')
    and nothing in between, so no two-dimensional irrep intrudes.  A level
    at Sz = S has spin S when the same sector at Sz = S + 1 lacks it."""
    g = GOLD["tos_120_triangular"]
    n, top = 12, 3
    spec, full = {}, {}
    for sz in range(top + 1):
        for inst in L.triangular12_sectors(J2=0.0, n_up=n // 2 + sz):
            reps, stabs = O.enumerate_basis(inst)
            if len(reps):
                w = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())
                spec.setdefault((sz, L.sector_label(inst)), []).extend(w)
        full[sz] = np.linalg.eigvalsh(O.unsym_sector_matrix(inst)[1].toarray())
    for S in range(top):
        levels = sorted((e, lab) for (sz, lab), w in spec.items() if sz == S
                        for e in _minus(w, spec.get((S + 1, lab), [])))
        m = {k: v[g["S"].index(S)] for k, v in g["multiplicity"].items()}
        tower = levels[:sum(m.values())]
        assert sorted(lab for _, lab in tower) == sorted(k for k, c in m.items() for _ in range(c))
        assert levels[len(tower)][0] > tower[-1][0] + 0.1
        expanded = sorted(e for e, lab in tower for _ in range(2 if lab.startswith("K.") else 1))
        spin_s = _minus(full[S], full[S + 1])
        assert np.allclose(spin_s[:len(expanded)], expanded, atol=1e-9)
        assert spin_s[len(expanded)] > expanded[-1] + 0.1


# --- learned-index network reference -----------------------------------------

def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(3)
    F, H = 6, 32
    params = [rng.standard_normal((H, F)) * 0.5, rng.standard_normal(H) * 0.1,
              rng.standard_normal((H, H)) * 0.3, rng.standard_normal(H) * 0.1,
              rng.standard_normal((1, H)) * 0.3, rng.standard_normal(1) * 0.1]
    X = rng.random((50, F))
    t = rng.random(50)
    loss, grads = O.mlp_loss_grad(params, X, t)
    h = 1e-6
    for p, g in zip(params, grads):
        flat = p.reshape(-1)
        gflat = g.reshape(-1)
        for k in rng.choice(flat.size, size=min(8, flat.size), replace=False):
            old = flat[k]
            flat[k] = old + h
            lp, _ = O.mlp_loss_grad(params, X, t)
            flat[k] = old - h
            lm, _ = O.mlp_loss_grad(params, X, t)
            flat[k] = old
            assert (lp - lm) / (2 * h) == pytest.approx(gflat[k], rel=1e-5, abs=1e-9)


# --- ground-state correlations ------------------------------------------------

def _op_instance(inst, bonds, bond_J, tris=None, tri_J=None):
    from dataclasses import replace
    return replace(inst, bonds=np.asarray(bonds, np.int32), bond_J=np.asarray(bond_J, float),
                   tris=np.zeros((0, 3), np.int32) if tris is None else np.asarray(tris, np.int32),
                   tri_Jchi=np.zeros(0) if tri_J is None else np.asarray(tri_J, float))


def test_ring4_correlations_closed_form():
    # singlet ground state of the 4-site ring: <S0.S1> = -1/2 (E0 = -2 over
    # four bonds); total spin 0 gives sum_j <S0.Sj> = 0, so <S0.S2> = +1/4
    inst = L.chain(4)
    reps, stabs = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps, stabs).toarray()
    w, v = np.linalg.eigh(H)
    psi = v[:, 0]
    c = {}
    for r in (1, 2):
        b, J = L.chain_distance_bonds(inst, r)
        Hr = O.coo_matrix(_op_instance(inst, b, J), reps, stabs).toarray()
        c[r] = float(psi @ Hr @ psi)
    assert c[1] == pytest.approx(-0.5, abs=1e-13)
    assert c[2] == pytest.approx(0.25, abs=1e-13)
    assert 0.75 + 2 * c[1] + c[2] == pytest.approx(0.0, abs=1e-13)


# --- structure factor -----------------------------------------------------------

def _ground_state_full(inst):
    states, H = O.unsym_sector_matrix(inst)
    w, v = np.linalg.eigh(H.toarray())
    return states, v[:, 0], w


def test_structure_factor_ring4_closed_form():
    # 4-site Heisenberg ring: singlet ground state with <S0.S1> = -1/2 and
    # <S0.S2> = 1/4, so S(0) = 0, S(pi/2) = S(3 pi/2) = 1/2, S(pi) = 2
    inst = L.chain(4, sublat=(2,))
    states, psi, w = _ground_state_full(inst)
    assert w[0] == pytest.approx(-2.0, abs=1e-12) and w[1] > w[0] + 1e-6
    C = O.spin_correlations(inst, states, psi)
    pos = L.site_coords(inst)
    from fractions import Fraction as F
    expect = {0: 0.0, 1: 0.5, 2: 2.0, 3: 0.5}
    for m, sq in expect.items():
        assert O.structure_factor(C, pos, (F(m, 4),)) == pytest.approx(sq, abs=1e-12)


def test_structure_factor_sum_rule_and_singlet_square16():
    # sum over all momenta of S(q) is 3N/4 for any state; a singlet has S(0) = 0
    inst = L.square_j1j2(L.SQ16_L[0], L.SQ16_L[1], 1.0, 0.0, L.Q0, sublat_chain=L.SQ16_CHAIN)
    states, H = O.unsym_sector_matrix(inst)
    w, v = scipy.sparse.linalg.eigsh(H, k=1, which="SA")
    psi = v[:, 0] / np.linalg.norm(v[:, 0])
    C = O.spin_correlations(inst, states, psi)
    # the correlations reproduce the energy: E = sum_b J_b C[i_b, j_b]
    assert sum(J * C[i, j] for (i, j), J in zip(inst.bonds.tolist(), inst.bond_J)) == pytest.approx(w[0], abs=1e-10)
    pos = L.site_coords(inst)
    lat = inst.meta["lattice"]
    total = sum(O.structure_factor(C, pos, q) for q in lat.momenta())
    assert total == pytest.approx(0.75 * inst.n_sites, abs=1e-10)
    assert O.structure_factor(C, pos, L.Q0) == pytest.approx(0.0, abs=1e-10)
    # Neel correlations peak at M = (pi, pi)
    sM = O.structure_factor(C, pos, (L.F(1, 2), L.F(1, 2)))
    assert all(sM >= O.structure_factor(C, pos, q) for q in lat.momenta())


@pytest.mark.parametrize("J2,peak", [(0.0, "K"), (0.3, "M")])
def test_structure_factor_triangular12_peaks(J2, peak):
    """Lattice coordinates on the triangular lattice (a1, a2 at 60 degrees):
    in the Gamma.A1 state of the 12-site cluster the sum rule gives 3N/4,
    S(q) is the same over each star, and it peaks at K with 120-degree
    correlations (J2 = 0) and at M on the stripy side (J2 = 0.3), as the
    thesis states for these orders."""
    inst = L.triangular_j1j2chi(L.TRI12_L[0], L.TRI12_L[1], 1.0, J2, 0.0, L.Q0, irrep="A1", flip=1,
                                sublat_chain=L.TRI12_CHAIN)
    states, psi = O.sector_state(inst)
    C = O.spin_correlations(inst, states, psi)
    pos = L.site_coords(inst)
    S = {q: O.structure_factor(C, pos, q) for q in inst.meta["lattice"].momenta()}
    assert sum(S.values()) == pytest.approx(0.75 * inst.n_sites, abs=1e-10)
    stars = {"K": L.momentum_star(inst, (L.F(1, 3), L.F(2, 3))), "M": L.momentum_star(inst, (L.F(1, 2), L.F(0)))}
    assert [len(stars["K"]), len(stars["M"])] == [2, 3]
    for star in stars.values():
        assert np.allclose([S[q] for q in star], S[star[0]], atol=1e-10)
    top = max(S.values())
    assert S[stars[peak][0]] == pytest.approx(top, abs=1e-12)
    assert all(S[q] < top - 0.5 for q in S if q not in stars[peak])


# --- order-parameter correlations (triangular J1-J2-Jchi chapter) --------------

def _triangle_instance(n_up):
    return L.Instance("triangle", 3, np.zeros((0, 2), np.int32), np.zeros(0), np.array([[0, 1, 2]], np.int32),
                      np.ones(1), n_up, np.arange(3, dtype=np.int32)[None], np.zeros(1, np.uint8),
                      np.ones(1, complex), [1])


def test_triangle_chirality_spectrum_and_correlation():
    """Three spins 1/2: S_0.(S_1 x S_2) is +-sqrt(3)/4 on the two spin-1/2
    doublets of definite chirality and 0 on the spin-3/2 quartet, so a
    chiral eigenstate has <chi chi> = 3/16."""
    S = O._spin_matrices(3)
    X = O.chirality_operator(S, 0, 1, 2).toarray()
    assert np.max(np.abs(X - X.conj().T)) < 1e-15
    r = np.sqrt(3.0) / 4
    assert np.allclose(np.linalg.eigvalsh(X), [-r, -r, 0, 0, 0, 0, r, r], atol=1e-14)
    inst = _triangle_instance(2)
    states, _ = O.unsym_sector_matrix(inst)
    w, v = np.linalg.eigh(X[np.ix_(states.astype(np.int64), states.astype(np.int64))])
    assert w[-1] == pytest.approx(r, abs=1e-14)
    c = O.chirality_correlation(inst, states, v[:, -1], (0, 1, 2), [(0, 1, 2)])
    assert c == pytest.approx(3.0 / 16, abs=1e-14)


def test_bond_correlation_ring4_closed_forms():
    """4-site ring ground state: the bond sum over the ring is H itself, so
    for an eigenstate sum_b <(S.S)_b0 (S.S)_b>_c = <b0 H> - <b0><H> = 0; and
    (S_0.S_1)^2 = 3/16 - (S_0.S_1)/2 for spins 1/2 gives 7/16 at
    <S_0.S_1> = -1/2."""
    inst = L.chain(4)
    states, H = O.unsym_sector_matrix(inst)
    w, v = np.linalg.eigh(H.toarray())
    psi = v[:, 0]
    b0 = tuple(inst.bonds[0])
    assert O.bond_correlation(inst, states, psi, b0, inst.bonds) == pytest.approx(0.0, abs=1e-13)
    sq = O.bond_correlation(inst, states, psi, b0, [b0], connected=False)
    assert sq == pytest.approx(7.0 / 16, abs=1e-13)
    assert O.bond_correlation(inst, states, psi, b0, inst.bonds, connected=False) == pytest.approx(1.0, abs=1e-13)


def test_resolvent_ring4_single_pole():
    """O = H on the 4-site ring ground state: O psi = E0 psi, so the
    resolvent has the single pole E0 with weight E0^2: 4 / (z + 2)."""
    inst = L.chain(4)
    reps, stabs = O.enumerate_basis(inst)
    w, v = np.linalg.eigh(O.coo_matrix(inst, reps, stabs).toarray())
    z = np.array([0.3 + 0.1j, -1.0 + 0.05j, 2.0 + 1.0j, -2.0 + 0.01j])
    G = O.sector_resolvent(inst, v[:, 0], inst, z)
    assert np.allclose(G, 4.0 / (z + 2.0), rtol=1e-13, atol=1e-13)
    # the pairs (0, 2) and (1, 3) each form spin 1 in that state, so
    # S_0.S_2 = S_1.S_3 = 1/4 on it: O = (S_0.S_2 + S_1.S_3)/2 (the distance-2
    # bonds at weight 1/4, each pair twice) has the single pole E0, weight 1/16
    b2, J2 = L.chain_distance_bonds(inst, 2)
    G2 = O.sector_resolvent(inst, v[:, 0], _op_instance(inst, b2, J2), z)
    assert np.allclose(G2, (1.0 / 16) / (z + 2.0), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("k", [0, 1])
def test_sector_state_is_symmetric_eigenvector(k):
    """The k-th sector eigenvector written out in the Sz configurations is an
    eigenvector of the unsymmetrized H with the same energy, and every group
    element g maps it to chi(g) times itself: with the projector
    sum_g conj(chi(g)) g, h P = chi(h) P.  Here for a complex sector (K
    point, chirality on), where a wrong conjugation shows."""
    inst = L.small_instances()[15]
    assert inst.is_complex
    reps, stabs = O.enumerate_basis(inst)
    w = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())
    states, psi = O.sector_state(inst, k)
    _, Hs = O.unsym_sector_matrix(inst)
    assert np.linalg.norm(Hs @ psi - w[k] * psi) < 1e-11
    pos = {int(s): i for i, s in enumerate(states)}
    for g in range(inst.n_elem):
        img = O.apply_group_numpy(inst, g, states)
        moved = np.zeros_like(psi)
        moved[[pos[int(t)] for t in img]] = psi
        assert np.linalg.norm(moved - inst.chi[g] * psi) < 1e-11


def _spectrum(insts):
    out = []
    for inst in insts:
        reps, stabs = O.enumerate_basis(inst)
        if len(reps):
            out.extend(np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray()))
    return np.sort(out)


@pytest.mark.parametrize("kind,sz", [("triangular", 0), ("triangular", 1), ("square", 0), ("square", 1)])
def test_two_dim_irreps_complete_the_spectrum(kind, sz):
    """At every momentum whose little group is C_nv (n >= 3), the levels of
    the one-dimensional sectors plus those of the rotation-subgroup sectors
    of the two-dimensional irreps, each counted twice, are exactly the
    spectrum of the same momentum with translations only (12-site
    triangular: Gamma (E1, E2) and K (E); 16-site square: Gamma and M)."""
    if kind == "triangular":
        Lt, ch, J2, n = L.TRI12_L, L.TRI12_CHAIN, 0.1, 12
        one = L.triangular_sectors(Lt, ch, J2=J2, n_up=n // 2 + sz)

        def trans_only(q, fl):
            return L.triangular_j1j2chi(Lt[0], Lt[1], 1.0, J2, 0.0, q, irrep="A", flip=fl, sublat_chain=ch,
                                        pg_gens=[], n_up=n // 2 + sz)
    else:
        Lt, ch, J2, n = L.SQ16_L, L.SQ16_CHAIN, 0.3, 16
        one = L.square_sectors(Lt, ch, J2=J2, n_up=n // 2 + sz)

        def trans_only(q, fl):
            return L.square_j1j2(Lt[0], Lt[1], 1.0, J2, q, irrep="A1", flip=fl, sublat_chain=ch, pg_gens=[],
                                 n_up=n // 2 + sz)
    two = L.two_dim_sectors(kind, Lt, ch, J2=J2, n_up=n // 2 + sz)
    flips = (1, -1) if sz == 0 else (None,)
    qs = sorted({tuple(i.meta["q"]) for i in two})
    assert len(qs) == 2
    for q in qs:
        got = np.sort(np.concatenate([_spectrum([i for i in one if tuple(i.meta["q"]) == q]),
                                      np.repeat(_spectrum([i for i in two if tuple(i.meta["q"]) == q]), 2)]))
        ref = _spectrum([trans_only(q, fl) for fl in flips])
        assert len(got) == len(ref) and np.allclose(got, ref, atol=1e-10), (kind, sz, q)
        assert any(len(O.enumerate_basis(i)[0]) for i in two if tuple(i.meta["q"]) == q)


def test_tower_of_states_triangular12_tetrahedral_table():
    """The 12-site triangular J1-J2-Jchi model at J2 = 0.2, Jchi = 0.5 (point
    group C6): the lowest levels of total spin S = 0..3 carry exactly the
    irreps and multiplicities of the thesis's tetrahedral tower table, with
    a gap above 0.2 to the next spin-S level.  Spin S = levels at Sz = S
    that the same sector lacks at Sz = S + 1."""
    g = GOLD["tos_tetrahedral_triangular"]
    n = 12
    spec = {}
    for sz in range(5):
        for inst in L.triangular_chiral_sectors(L.TRI12_L, L.TRI12_CHAIN, J2=0.2, Jchi=0.5, n_up=n // 2 + sz):
            reps, stabs = O.enumerate_basis(inst)
            if len(reps):
                w = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())
                spec.setdefault((sz, L.sector_label(inst)), []).extend(w)
    for S in g["S"]:
        levels = sorted((e, lab) for (sz, lab), w in spec.items() if sz == S
                        for e in _minus(w, spec.get((S + 1, lab), [])))
        m = {k: v[g["S"].index(S)] for k, v in g["multiplicity"].items()}
        n_tower = sum(m.values())
        assert sorted(lab for _, lab in levels[:n_tower]) == sorted(k for k, c in m.items() for _ in range(c)), S
        assert levels[n_tower][0] > levels[n_tower - 1][0] + 0.2


def test_bond_and_chirality_correlations_eigenstate_identities():
    """12-site triangular lattice.  With J2 = 0, H is the sum of the bonds of
    all three directions, so in an eigenstate sum_b <(S.S)_b0 (S.S)_b>_c over
    all bonds b vanishes.  With H = X_all (every triangle's chirality, point
    group C6), an eigenstate of eigenvalue x has sum_t <chi_0 chi_t> =
    <chi_0 X_all> = x <chi_0> = x^2 / 2N (the 2N triangles are equivalent
    under translations and C6)."""
    inst = L.triangular_j1j2chi(L.TRI12_L[0], L.TRI12_L[1], 1.0, 0.0, 0.0, L.Q0, irrep="A1", flip=1,
                                sublat_chain=L.TRI12_CHAIN)
    states, psi = O.sector_state(inst)
    b0 = tuple(L.bonds_along(inst, (1, 0))[0])
    assert abs(O.bond_correlation(inst, states, psi, b0, inst.bonds)) < 1e-10
    # a sub-sum alone is not zero: the check is not trivially satisfied
    assert abs(O.bond_correlation(inst, states, psi, b0, L.bonds_along(inst, (1, 0)))) > 1e-3
    from dataclasses import replace
    chiral = L.triangular_j1j2chi(L.TRI12_L[0], L.TRI12_L[1], 1.0, 0.0, 1.0, L.Q0, irrep="A", flip=1,
                                  sublat_chain=L.TRI12_CHAIN)
    up, down = L.triangles(chiral)
    pure = replace(chiral, bonds=np.zeros((0, 2), np.int32), bond_J=np.zeros(0))
    reps, stabs = O.enumerate_basis(pure)
    x = np.linalg.eigvalsh(O.coo_matrix(pure, reps, stabs).toarray())[0]
    states, psi = O.sector_state(pure)
    X = O.chirality_correlation(pure, states, psi, tuple(up[0]), np.concatenate([up, down]))
    assert abs(x) > 1.0
    assert X.real == pytest.approx(x * x / (2 * 12), rel=1e-10)
    assert abs(X.imag) < 1e-12
