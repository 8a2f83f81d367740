"""Kagome J1-J2-J3-Jchi workloads (thesis chapter on the kagome chiral spin
liquid): the lattice and its group, and the oracle on kagome sectors, pinned
by the same definitions as the other lattices - the character formula, the
Kronecker-product Hamiltonian, projector-built symmetric vectors, the
partition of the spectrum over momentum sectors, and SU(2) multiplets."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import lattices as L

KAG = L.kagome_instances()


def _ids(i):
    return f"{i.name}-{i.sector}"


def test_kagome_geometry():
    inst = L.kagome_j1j2j3chi(L.KAG27_L[0], L.KAG27_L[1], 1.0, 0.2, 0.1, 0.3, L.Q0, "A", 1, L.KAG27_CHAIN)
    lat = inst.meta["lattice"]
    n = inst.n_sites
    assert n == 27 and len(lat.translations()) == 9 and len(lat.pg) == 6      # C6 (chirality on)
    deg = {J: np.bincount(inst.bonds[inst.bond_J == J].ravel(), minlength=n) for J in (1.0, 0.2, 0.1)}
    assert np.all(deg[1.0] == 4)        # two triangles, two neighbours in each
    assert np.all(deg[0.2] == 4)        # second neighbours at distance sqrt3
    assert np.all(deg[0.1] == 2)        # one diagonal in each of the two hexagons at a site
    assert np.all(np.bincount(inst.tris.ravel(), minlength=n) == 2) and len(inst.tris) == 2 * n // 3
    # distances in the plane
    xy = np.array([np.array(p, float) @ lat.cart for p in lat.coords])
    Lc = np.array([np.array(lat.L1, float) @ lat.cart, np.array(lat.L2, float) @ lat.cart])

    def dist(i, j):
        d = xy[j] - xy[i]
        return min(np.linalg.norm(d + a * Lc[0] + b * Lc[1]) for a in (-1, 0, 1) for b in (-1, 0, 1))
    for J, want in ((1.0, 1.0), (0.2, np.sqrt(3.0)), (0.1, 2.0)):
        assert all(abs(dist(i, j) - want) < 1e-9 for i, j in inst.bonds[inst.bond_J == J])
    # every group element maps the bond multiset and the oriented triangles onto themselves
    key = lambda i, j, J: (min(i, j), max(i, j), J)
    bset = sorted(key(i, j, J) for (i, j), J in zip(inst.bonds, inst.bond_J))
    tset = {tuple(np.roll(t, -int(np.argmin(t)))) for t in inst.tris}
    for p in inst.perms:
        assert sorted(key(p[i], p[j], J) for (i, j), J in zip(inst.bonds, inst.bond_J)) == bset
        mt = {tuple(np.roll(p[t], -int(np.argmin(p[t])))) for t in inst.tris}
        assert mt == tset


def test_kagome_full_point_group_and_momenta():
    lat = L.kagome_lattice(L.KAG12_L[0], L.KAG12_L[1], L.KAG12_CHAIN)
    assert lat.N == 12 and len(lat.pg) == 12 and lat.sublat_options == [3]
    qs = lat.momenta()
    assert len(qs) == 4 and all(0 <= x < L.F(1, 2) for q in qs for x in q)
    # the three sublattices are contiguous blocks of four labels, and the
    # point group permutes them
    blocks = [set(range(4 * k, 4 * k + 4)) for k in range(3)]
    for P in lat.pg:
        perm = lat.perm(P, (0, 0))
        for b in blocks:
            assert {int(perm[i]) for i in b} in blocks


@pytest.mark.parametrize("inst", KAG, ids=_ids)
def test_kagome_dimension_equals_character_formula(inst):
    reps, stabs = O.enumerate_basis(inst)
    assert len(reps) == O.character_formula_dim(inst) > 0
    assert np.all(inst.n_elem % stabs == 0)


@pytest.mark.parametrize("inst", KAG, ids=_ids)
def test_kagome_terms_match_kronecker(inst):
    states, Hs = O.unsym_sector_matrix(inst)
    Hk = O.kron_hamiltonian(inst)
    idx = states.astype(np.int64)
    assert np.max(np.abs(Hs.toarray() - Hk[idx][:, idx].toarray())) < 1e-13


@pytest.mark.parametrize("inst", KAG, ids=_ids)
def test_kagome_symmetrized_matrix_equals_projection(inst):
    reps, stabs = O.enumerate_basis(inst)
    Hsym = O.coo_matrix(inst, reps, stabs).toarray()
    states, Hs = O.unsym_sector_matrix(inst)
    B = O.projector_basis(inst, reps, states)
    assert np.max(np.abs(Hsym - B.conj().T @ (Hs @ B))) < 1e-12
    assert np.max(np.abs(B.conj().T @ B - np.eye(len(reps)))) < 1e-12


@pytest.mark.parametrize("Jchi", [0.0, 0.3])
def test_kagome_momentum_sectors_partition_the_spectrum(Jchi):
    """Translations times the spin flip form an abelian group: the spectra of
    all its sectors together are the Sz = 0 spectrum."""
    ev = []
    lat = L.kagome_lattice(L.KAG12_L[0], L.KAG12_L[1], L.KAG12_CHAIN, pg_gens=[])
    for q in lat.momenta():
        for fl in (1, -1):
            inst = L.kagome_j1j2j3chi(L.KAG12_L[0], L.KAG12_L[1], 1.0, 0.2, 0.1, Jchi, q, "A", fl, L.KAG12_CHAIN,
                                      pg_gens=[])
            reps, stabs = O.enumerate_basis(inst)
            if len(reps):
                ev.extend(np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray()))
    full_inst = L.kagome_j1j2j3chi(L.KAG12_L[0], L.KAG12_L[1], 1.0, 0.2, 0.1, Jchi, L.Q0, "A", None,
                                   L.KAG12_CHAIN, pg_gens=[])
    full = np.linalg.eigvalsh(O.kron_hamiltonian(full_inst).toarray())
    states, _ = O.unsym_sector_matrix(full_inst)
    Hs = O.kron_hamiltonian(full_inst)[states.astype(np.int64)][:, states.astype(np.int64)].toarray()
    sz0 = np.linalg.eigvalsh(Hs)
    assert len(ev) == len(sz0) == 924
    assert np.max(np.abs(np.sort(ev) - sz0)) < 1e-11
    assert full[0] <= sz0[0] + 1e-12


def test_kagome_su2_multiplets():
    """Every level at Sz = 1 of the Gamma.A1 sector is a level at Sz = 0 of
    the same sector, of one flip parity or the other."""
    def levels(n_up, flips):
        out = []
        for fl in flips:
            inst = L.kagome_j1j2j3chi(L.KAG12_L[0], L.KAG12_L[1], 1.0, 0.2, 0.1, 0.0, L.Q0, "A1", fl,
                                      L.KAG12_CHAIN, n_up=n_up)
            reps, stabs = O.enumerate_basis(inst)
            out.extend(np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray()))
        return np.array(out)
    e0 = levels(6, (1, -1))
    e1 = levels(7, (None,))
    assert len(e1) > 0
    assert all(np.min(np.abs(e0 - x)) < 1e-10 for x in e1)


def test_kagome27_chain_is_stable():
    """Both levels of the 27-site labelling (3 sublattices, then 9 cosets of
    the sqrt3 x sqrt3 cells) are kept by C6v and by the chiral C6."""
    for inst, dim in ((L.kagome27(J2=0.2, J3=0.1), 186_616), (L.kagome27(Jchi=0.3), 372_044)):
        assert inst.sublat_options == [3, 9]
        O.Fast(inst, 3).close()
        F = O.Fast(inst, 9)
        assert len(F.basis()[0]) == O.character_formula_dim(inst) == dim


def test_kagome_sectors_named_and_inside_the_spectrum():
    """Every one-dimensional sector of the 12-site kagome J1-J2-J3 model at
    Sz = 0 and 1: dimension = character formula, names in the thesis's form
    (Gamma, M, K of the kagome zone), and every sector level is a level of
    the unsymmetrized Sz sector."""
    for n_up in (6, 7):
        insts = L.kagome_sectors(L.KAG12_L, L.KAG12_CHAIN, J2=0.2, J3=0.1, n_up=n_up)
        full_inst = L.kagome_j1j2j3chi(L.KAG12_L[0], L.KAG12_L[1], 1.0, 0.2, 0.1, 0.0, L.Q0, "A", None,
                                       L.KAG12_CHAIN, pg_gens=[], n_up=n_up)
        _, Hs = O.unsym_sector_matrix(full_inst)
        full = np.linalg.eigvalsh(Hs.toarray())
        names = [(L.sector_label(i), i.meta["flip"]) for i in insts]
        assert len(set(names)) == len(names)
        moms = {n.split(".")[0] for n, _ in names}
        assert moms == {"Gamma", "M"}                 # the 2 x 2 cell torus holds Gamma and the three M
        assert {"Gamma.A1", "Gamma.A2", "Gamma.B1", "Gamma.B2"} <= {n for n, _ in names}
        for inst in insts:
            reps, stabs = O.enumerate_basis(inst)
            assert len(reps) == O.character_formula_dim(inst)
            if len(reps):
                ev = np.linalg.eigvalsh(O.coo_matrix(inst, reps, stabs).toarray())
                assert all(np.min(np.abs(full - e)) < 1e-10 for e in ev), L.sector_label(inst)


def test_kagome27_sector_momenta():
    """The 3 x 3 cell torus: Gamma, K (K and K' one star) and one six-member
    star; C6v irreps named as on the triangular lattice."""
    insts = L.kagome_sectors(L.KAG27_L, L.KAG27_CHAIN, n_up=13)
    names = {L.sector_label(i) for i in insts}
    assert names == {"Gamma.A1", "Gamma.A2", "Gamma.B1", "Gamma.B2", "K.A1", "K.ir1", "(0,1/3).A1", "(0,1/3).ir1"}
    lat = insts[0].meta["lattice"]
    stars = {frozenset(L._pg_orbit(lat, q)) for q in lat.momenta()}
    assert sorted(len(st) for st in stars) == [1, 2, 6]
