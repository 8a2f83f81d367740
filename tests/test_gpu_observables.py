"""Ground-state vectors (second Lanczos pass over the Ritz vector of T) and
expectation values of symmetric operators, against the oracle's dense
eigenvectors and closed forms."""
import sys
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from workloads import lattices as L
from workloads import vectors as V

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def S():
    _torch()
    from paper_2210_03511_amd import symed
    symed.lib()
    return symed


def _dev(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).cuda()


def _op(inst, bonds, J, tris=None, tJ=None):
    return replace(inst, bonds=np.asarray(bonds, np.int32), bond_J=np.asarray(J, float),
                   tris=np.zeros((0, 3), np.int32) if tris is None else np.asarray(tris, np.int32),
                   tri_Jchi=np.zeros(0) if tJ is None else np.asarray(tJ, float))


def test_ring4_correlations(S):
    torch = _torch()
    inst = L.chain(4)
    b = S.Basis.build(inst)
    e0, psi = b.ground_state(_dev(torch, np.array([1.0, 0.3])), 10)
    assert e0 == pytest.approx(-2.0, abs=1e-12)
    c1 = b.expectation(psi, *L.chain_distance_bonds(inst, 1)).real
    c2 = b.expectation(psi, *L.chain_distance_bonds(inst, 2)).real
    assert c1 == pytest.approx(-0.5, abs=1e-12)
    assert c2 == pytest.approx(0.25, abs=1e-12)


def test_chain16_correlations_against_oracle(S):
    torch = _torch()
    inst = L.chain16()
    reps, stabs = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps, stabs).toarray()
    w, v = np.linalg.eigh(H)
    ref = v[:, 0]
    b = S.Basis.build(inst)
    b.train_index(steps=300)
    b.build_hash()
    v0 = _dev(torch, V.start_vector(b.dim, 1002))
    out = {}
    for mode in (0, 1, 2):
        e0, psi = b.ground_state(v0, 90, mode=mode)
        assert e0 == pytest.approx(w[0], rel=1e-12)
        ph = psi.cpu().numpy()
        assert abs(abs(ph @ ref) - 1.0) < 1e-10
        cs = []
        for r in range(1, 9):
            bb, J = L.chain_distance_bonds(inst, r)
            c = b.expectation(psi, bb, J, mode=mode)
            Hr = O.coo_matrix(_op(inst, bb, J), reps, stabs).toarray()
            assert c.real == pytest.approx(float(ref @ Hr @ ref), abs=1e-9)
            cs.append(c.real)
        # <H> = E0
        assert b.expectation(psi, inst.bonds, inst.bond_J, mode=mode).real == pytest.approx(w[0], rel=1e-11)
        out[mode] = (ph, cs)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][0], out[2][0])
    assert out[0][1] == out[1][1] == out[2][1]


def test_complex_sector_chirality_against_oracle(S):
    torch = _torch()
    inst = L.small_instances()[15]          # triangular 12, K point, chirality on
    assert inst.is_complex
    reps, stabs = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps, stabs).toarray()
    w, v = np.linalg.eigh(H)
    ref = v[:, 0]
    b = S.Basis.build(inst)
    v0 = _dev(torch, V.start_vector(b.dim, 7, True))
    e0, psi = b.ground_state(v0, min(120, b.dim))
    assert e0 == pytest.approx(w[0], rel=1e-11)
    n_tri = len(inst.tri_Jchi)
    c = b.expectation(psi, tris=inst.tris, tri_Jchi=np.full(n_tri, 1.0 / n_tri))
    Oc = O.coo_matrix(_op(inst, np.zeros((0, 2)), np.zeros(0), inst.tris, np.full(n_tri, 1.0 / n_tri)), reps,
                      stabs).toarray()
    refc = np.vdot(ref, Oc @ ref)
    assert abs(c.real - refc.real) < 1e-9
    assert abs(c.imag) < 1e-12 and abs(refc.imag) < 1e-12


def test_square32_energy_decomposition(S):
    """At full cfg-2 size: <H> = E0, and the J1 and J2 bond energies add up."""
    torch = _torch()
    inst = L.square32()
    b = S.Basis.build(inst)
    v0 = _dev(torch, V.start_vector(b.dim, 2002))
    e0, psi = b.ground_state(v0, 90)
    assert e0 == pytest.approx(-16.00306361800979, rel=1e-10)   # stored oracle value (tests/golden)
    n = float(torch.linalg.vector_norm(psi).item())
    assert n == pytest.approx(1.0, abs=1e-12)
    eh = b.expectation(psi, inst.bonds, inst.bond_J).real
    assert eh == pytest.approx(e0, rel=1e-9)
    j1 = inst.bond_J == 1.0
    e1 = b.expectation(psi, inst.bonds[j1], inst.bond_J[j1]).real
    e2 = b.expectation(psi, inst.bonds[~j1], inst.bond_J[~j1]).real
    assert e1 + e2 == pytest.approx(eh, rel=1e-12)
    print("square32 E0", e0, "J1 part", e1, "J2 part", e2, flush=True)


def test_expectation_rejects_non_invariant_operator(S):
    torch = _torch()
    inst = L.chain16()
    b = S.Basis.build(inst)
    psi = _dev(torch, V.start_vector(b.dim, 1))
    with pytest.raises(S.EdError) as e:
        b.expectation(psi, np.array([[0, 1]]), np.array([1.0]))
    assert e.value.status == S.ED_EINVAL
    with pytest.raises(S.EdError):
        b.expectation(psi, tris=np.array([[0, 1, 2]]), tri_Jchi=np.array([1.0]))
