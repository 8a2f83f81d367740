"""Pins of the SU(d) part of the oracle (chapter on SU(N) chiral spin
liquids: H = J sum P_ij + i K3 sum (P_ijk - P_ijk^-1) with d colors per site).

Closed forms and independent constructions:
- the two-site exchange P_12 has eigenvalue +1 on the d(d+1)/2 symmetric and
  -1 on the d(d-1)/2 antisymmetric states;
- on three sites of distinct colors the ring term i(P - P^-1) has
  eigenvalues 0, -sqrt(3), +sqrt(3), each twice (P has the eigenvalues
  1, w, w^2 on each of its two 3-cycles);
- the oracle's unsymmetrized matrix equals the one built from explicit
  permutation matrices and Kronecker products;
- the symmetrized matrix equals B^dagger H B for explicit projected states;
- the sector dimensions equal the character formula and add up, over all
  momenta of a translation group, to the number of configurations;
- the union of the momentum-sector spectra is the unsymmetrized spectrum;
- for d = 2 the permutation model is the spin-1/2 model:
  P_ij = 2 S_i.S_j + 1/2 and i (P_ijk - P_ijk^-1) = 4 S_i.(S_j x S_k), checked
  on explicit three-site matrices and then on whole sector spectra against the
  spin-1/2 part of the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import lattices as L


def _trivial(inst):
    """The same model with the trivial group."""
    import dataclasses
    n = inst.n_sites
    return dataclasses.replace(inst, perms=np.arange(n, dtype=np.int32)[None, :], flips=np.zeros(1, np.uint8),
                               chi=np.ones(1, complex))


def test_two_site_exchange():
    for d in (2, 3, 4):
        P = O.sun_kron_operator(2, d, (0, 1), 2)
        ev = np.round(np.linalg.eigvalsh(P), 12)
        assert (ev == 1).sum() == d * (d + 1) // 2 and (ev == -1).sum() == d * (d - 1) // 2


def test_three_site_ring_closed_form():
    for d in (3, 4):
        P = O.sun_kron_operator(3, d, (0, 1, 2), 3)
        R = 1j * (P - P.T)
        # configurations of three distinct colors 0, 1, 2
        idx = [a * d * d + b * d + c for a in range(3) for b in range(3) for c in range(3) if len({a, b, c}) == 3]
        ev = np.sort(np.linalg.eigvalsh(R[np.ix_(idx, idx)]))
        s3 = np.sqrt(3.0)
        assert np.allclose(ev, [-s3, -s3, 0, 0, s3, s3], atol=1e-12)
    # and through the oracle's sector matrix of a 3-site ring with counts (1, 1, 1)
    inst = _trivial(L.sun_chain(3, 3, (1, 1, 1), J=0.0, K3=1.0))
    inst.tris = inst.tris[:1]
    inst.tri_Jchi = inst.tri_Jchi[:1]
    st, M = O.sun_full_matrix(inst)
    assert np.allclose(np.sort(np.linalg.eigvalsh(M)), [-np.sqrt(3)] * 2 + [0, 0] + [np.sqrt(3)] * 2, atol=1e-12)


@pytest.mark.parametrize("d,counts,K", [(3, (2, 1, 1), 0.0), (3, (2, 1, 1), 0.7), (4, (1, 1, 1, 1), -0.4)])
def test_full_matrix_equals_kronecker_product_form(d, counts, K):
    n = 4
    inst = _trivial(L.sun_chain(n, d, counts, J=1.3, K3=K))
    st, M = O.sun_full_matrix(inst)
    H = np.zeros((d ** n, d ** n), complex)
    for (i, j), J in zip(inst.bonds, inst.bond_J):
        H += J * O.sun_kron_operator(n, d, (int(i), int(j)), 2)
    for (i, j, k), Kt in zip(inst.tris, inst.tri_Jchi):
        P = O.sun_kron_operator(n, d, (int(i), int(j), int(k)), 3)
        H += 1j * Kt * (P - P.T)
    dg = O.sun_digits(st, n)
    idx = [sum(int(c) * d ** (n - 1 - s) for s, c in enumerate(row)) for row in dg]
    assert np.abs(H[np.ix_(idx, idx)] - M).max() < 1e-13
    # H preserves the color counts: nothing leaks out of the sector
    rest = np.setdiff1d(np.arange(d ** n), idx)
    assert np.abs(H[np.ix_(rest, idx)]).max() == 0


def _tri9(d, counts, K3, q=L.Q0):
    return L.sun_triangular((3, 0), (0, 3), d, counts, J=1.0, K3=K3, q=q, sublat_chain=[((1, 1), (2, -1))],
                            name="su_tri")


@pytest.mark.parametrize("make", [lambda: L.sun_chain(6, 3, (2, 2, 2), k=1), lambda: L.sun_chain(6, 3, (2, 2, 2), K3=0.6, k=2),
                                  lambda: L.sun_chain(8, 4, (2, 2, 2, 2), k=3), lambda: _tri9(3, (3, 3, 3), 0.4)],
                         ids=["chain6-k1", "chain6-ring-k2", "su4chain8-k3", "tri9-ring"])
def test_symmetrized_matrix_equals_projected(make):
    inst = make()
    reps, stabs = O.sun_enumerate_basis(inst)
    assert len(reps) == O.sun_character_formula_dim(inst)
    Hs = O.sun_coo_matrix(inst, reps, stabs).toarray()
    st, M = O.sun_full_matrix(inst)
    st2, B = O.sun_projector_basis(inst, reps)
    assert np.array_equal(st, st2)
    assert np.abs(B.conj().T @ B - np.eye(len(reps))).max() < 1e-12
    assert np.abs(B.conj().T @ M @ B - Hs).max() < 1e-12
    assert np.abs(Hs - Hs.conj().T).max() < 1e-13


def test_momentum_sectors_add_up():
    n, d, counts = 8, 3, (3, 3, 2)
    total = len(O.sun_states(n, d, counts))
    st, M = O.sun_full_matrix(_trivial(L.sun_chain(n, d, counts, K3=0.5)))
    full = np.sort(np.linalg.eigvalsh(M))
    dims, spec = 0, []
    for k in range(n):
        inst = L.sun_chain(n, d, counts, K3=0.5, k=k)
        reps, stabs = O.sun_enumerate_basis(inst)
        assert len(reps) == O.sun_character_formula_dim(inst)
        dims += len(reps)
        spec.append(np.linalg.eigvalsh(O.sun_coo_matrix(inst, reps, stabs).toarray()))
    assert dims == total
    assert np.allclose(np.sort(np.concatenate(spec)), full, atol=1e-10)


def test_su2_permutation_model_is_the_spin_half_model():
    # explicit three-site matrices
    P = O.sun_kron_operator(3, 2, (0, 1, 2), 3)
    S = O._spin_matrices(3)
    assert np.abs(1j * (P - P.T) - 4 * O.chirality_operator(S, 0, 1, 2).toarray()).max() < 1e-14
    S2 = O._spin_matrices(2)
    assert np.abs(O.sun_kron_operator(2, 2, (0, 1), 2) - 2 * O.bond_operator(S2, 0, 1).toarray()
                  - 0.5 * np.eye(4)).max() < 1e-14
    # whole sectors: SU(2) model (J, K) = spin-1/2 model (2J, Jchi = 4K) + sum(J)/2
    import dataclasses
    J, K = 0.8, 0.3
    for k in (0, 1, 3):
        su = L.sun_triangular((3, 0), (0, 3), 2, (5, 4), J=J, K3=K, q=L.Q0 if k == 0 else
                              (L.Fraction(k, 3), L.Fraction(0)), sublat_chain=[((1, 1), (2, -1))], name="su2")
        sp = dataclasses.replace(su, local_dim=0, counts=(), n_up=4, bond_J=2 * su.bond_J, tri_Jchi=4 * su.tri_Jchi)
        r1, s1 = O.sun_enumerate_basis(su)
        r2, s2 = O.enumerate_basis(sp)
        assert len(r1) == len(r2) > 0
        e1 = np.linalg.eigvalsh(O.sun_coo_matrix(su, r1, s1).toarray())
        e2 = np.linalg.eigvalsh(O.coo_matrix(sp, r2, s2).toarray()) + 0.5 * su.bond_J.sum()
        assert np.allclose(np.sort(e1), np.sort(e2), atol=1e-12)
