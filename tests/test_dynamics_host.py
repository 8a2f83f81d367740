"""Continued-fraction evaluation (host logic of the dynamical correlations):
from T-matrices of the oracle's Lanczos (no reorthogonalization) started at
O psi, against the oracle's spectral sum over the dense sector eigenpairs,
and against closed forms of short fractions."""
from dataclasses import replace

import numpy as np

from oracle import oracle as O
from workloads import lattices as L


def test_short_fractions_closed_form():
    from paper_2210_03511_amd import dynamics as D
    z = np.array([0.5 + 0.1j, -1.0 + 2.0j])
    assert np.allclose(D.continued_fraction([0.3], [], z, 2.0), 2.0 / (z - 0.3))
    # two levels: the 2 x 2 T-matrix's (0, 0) resolvent entry
    a0, a1, b0 = 0.2, -0.7, 0.4
    T = np.array([[a0, b0], [b0, a1]])
    ref = np.array([np.linalg.inv(zz * np.eye(2) - T)[0, 0] for zz in z])
    assert np.allclose(D.continued_fraction([a0, a1], [b0, 9.9], z), ref, rtol=1e-14)


def test_continued_fraction_equals_spectral_sum():
    from paper_2210_03511_amd import dynamics as D
    inst = L.triangular_j1j2chi(L.TRI12_L[0], L.TRI12_L[1], 1.0, 0.2, 0.0, L.Q0, irrep="A", flip=1,
                                sublat_chain=L.TRI12_CHAIN, pg_gens=[L.TRI_C2, L.TRI_MY])
    bonds = L.bonds_along(inst, (1, 0))
    op = replace(inst, bonds=bonds, bond_J=np.ones(len(bonds)))
    reps, stabs = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps, stabs)
    w, v = np.linalg.eigh(H.toarray())
    psi = v[:, 0]
    phi = O.coo_matrix(op, reps, stabs) @ psi
    a, b = O.lanczos(lambda x: H @ x, phi, len(reps))
    omegas = np.linspace(-0.5, 6.0, 27)
    z = omegas + w[0] + 0.1j
    ref = O.sector_resolvent(inst, psi, op, z)
    got = D.continued_fraction(a, b, z, float(np.vdot(phi, phi).real))
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))
    # weight: the integral of A(omega) is |O psi|^2 (checked on a wide, fine grid)
    om = np.linspace(-60, 60, 240001)
    A = D.spectral_function(D.continued_fraction(a, b, om + w[0] + 0.1j, float(np.vdot(phi, phi).real)))
    assert abs(np.trapezoid(A, om) - np.vdot(phi, phi).real) < 2e-3 * np.vdot(phi, phi).real
