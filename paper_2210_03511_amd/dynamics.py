"""Dynamical correlation functions by the continued-fraction expansion
(host orchestration only).

The thesis's outlook names the continued-fraction expansion of Gagliano and
Balseiro (1987) as the way to dynamical structure factors.  For a state
psi with energy E0 and an operator O,

    G(z) = <psi| O^dag (z - H)^-1 O |psi>,   z = omega + E0 + i eta,

equals |O psi|^2 / (z - a_0 - b_0^2 / (z - a_1 - b_1^2 / (z - ...))), where
a_k, b_k are the Lanczos coefficients of H started from O psi / |O psi|
(b_k: the norm produced at step k).  The spectral function is
A(omega) = -Im G / pi: poles at the excitation energies E_n - E0 with
weights |<n|O|psi>|^2, each broadened to a Lorentzian of half-width eta.

Here O is an operator of the form of H (bonds, chirality triangles)
invariant under the basis's group, so O psi stays in the sector.  O psi and
|O psi|^2 come from ed_apply_op and the coefficients from ed_lanczos_run,
both in the library; only the continued fraction (a few hundred numbers)
is evaluated here.
"""
from __future__ import annotations

import numpy as np


def continued_fraction(alpha, beta, z, weight=1.0):
    """weight / (z - a_0 - b_0^2 / (z - a_1 - ... - b_{n-2}^2 / (z - a_{n-1})))
    for the T-matrix with diagonal alpha[n] and off-diagonal beta[:n-1],
    evaluated from the bottom up at every z of an array."""
    a = np.asarray(alpha, np.float64)
    b = np.asarray(beta, np.float64)
    z = np.asarray(z, np.complex128)
    g = 1.0 / (z - a[-1])
    for k in range(len(a) - 2, -1, -1):
        g = 1.0 / (z - a[k] - b[k] ** 2 * g)
    return weight * g


def correlation(basis, psi, e0, omegas, eta, n_iter, op, mode=0, stream=None):
    """G(omega + E0 + i eta) for the normalized state psi (energy e0) and the
    operator ``op`` (a dict of bonds, bond_J, tris, tri_Jchi, as for
    ``Basis.expectation``).  Returns (G, |O psi|^2, alpha, beta)."""
    import torch
    y = torch.empty_like(psi)
    w = basis.apply_op(psi, y, z=y, mode=mode, stream=stream, **op).real
    if w <= 0.0:
        return np.zeros(len(np.atleast_1d(omegas)), np.complex128), 0.0, np.zeros(0), np.zeros(0)
    a, b, n, _ = basis.lanczos(y, min(n_iter, basis.dim), mode=mode, stream=stream)
    z = np.asarray(omegas, np.float64) + e0 + 1j * eta
    return continued_fraction(a[:n], b[:n], z, w), w, a[:n], b[:n]


def spectral_function(G):
    """A(omega) = -Im G(omega) / pi."""
    return -np.imag(G) / np.pi


def _peaks(omegas, A, count):
    i = [k for k in range(1, len(A) - 1) if A[k] >= A[k - 1] and A[k] > A[k + 1]]
    i.sort(key=lambda k: -A[k])
    return sorted((float(omegas[k]), float(A[k])) for k in i[:count])


def _main(argv=None):
    import argparse
    import time

    from workloads import lattices as L

    from . import tower

    ap = argparse.ArgumentParser(description="Spectral function A(omega) of the chirality sum (C6 sector) or of "
                                             "the bond sum along a1 (sector of {E, C2, mirrors}) in the Gamma "
                                             "ground state of the triangular J1-J2-Jchi model.")
    ap.add_argument("--sites", type=int, default=36, choices=[12, 36])
    ap.add_argument("--J2", type=float, default=0.1)
    ap.add_argument("--Jchi", type=float, default=0.2)
    ap.add_argument("--op", default="chirality", choices=["chirality", "bonds"])
    ap.add_argument("--steps", type=int, default=100, help="ground-state Lanczos steps")
    ap.add_argument("--cf-steps", type=int, default=200, help="continued-fraction steps")
    ap.add_argument("--eta", type=float, default=0.05)
    ap.add_argument("--mode", type=int, default=2, choices=[0, 2])
    a = ap.parse_args(argv)
    Lt, ch = {12: (L.TRI12_L, L.TRI12_CHAIN), 36: (L.TRI36_L, L.TRI36_CHAIN)}[a.sites]
    gens = None if a.op == "chirality" else [L.TRI_C2] + ([L.TRI_MY] if a.Jchi == 0.0 else [])
    inst = L.triangular_j1j2chi(Lt[0], Lt[1], 1.0, a.J2, a.Jchi, L.Q0, irrep="A", flip=1, sublat_chain=ch,
                                pg_gens=gens)
    if a.op == "chirality":
        up, down = L.triangles(inst)
        tris = np.concatenate([up, down])
        op = dict(tris=tris, tri_Jchi=np.ones(len(tris)))
    else:
        bonds = L.bonds_along(inst, (1, 0))
        op = dict(bonds=bonds, bond_J=np.ones(len(bonds)))
    from . import symed as S
    t0 = time.perf_counter()
    b = S.Basis.build(inst)
    if a.mode == 2:
        b.build_hash()
    e0, psi = b.ground_state(tower._start(b.dim, b.is_complex, 1), min(a.steps, b.dim), mode=a.mode)
    t1 = time.perf_counter()
    omegas = np.linspace(0.0, 8.0, 1601)
    G, w, alpha, beta = correlation(b, psi, e0, omegas, a.eta, a.cf_steps, op, mode=a.mode)
    t2 = time.perf_counter()
    A = spectral_function(G)
    print(f"{a.op}: dim {b.dim}, E0 {e0:.10f} ({t1 - t0:.1f} s), |O psi|^2 {w:.8f}, {len(alpha)} steps "
          f"({t2 - t1:.1f} s), integral of A over [0, 8] {np.trapezoid(A, omegas):.6f}", flush=True)
    for om, val in _peaks(omegas, A, 6):
        print(f"    peak omega {om:.4f}  A {val:.6f}", flush=True)
    b.free()


if __name__ == "__main__":
    _main()
