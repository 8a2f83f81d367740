"""CPU oracle for symmetrized exact diagonalization (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It shares no code with the HIP library: the C part
(``oracle.c`` and ``fast.c``, built into ``liboracle.so``) does brute-force
orbit scans, binary search and the host sublattice-coding method; this
module adds the dense and Lanczos layers in numpy/scipy.

What each function follows (thesis sections / equations):
  * ``enumerate_basis``  - representatives = orbit minima ("representative
    condition"), kept iff chi is trivial on the stabilizer, norm
    sqrt(|G| |Stab|) (1-D symmetry-adapted states).
  * ``coo_matrix``       - symmetrized matrix element of every non-branching
    piece ("Computations in the symmetrized basis"), push form.
  * ``row_entries``      - the same elements, row by row (gather form).
  * ``character_formula_dim`` - the character formula n_rho = |G|^-1 sum_g
    conj(chi(g)) Tr Gamma(g) (tower-of-states appendix), with Tr Gamma(g)
    counted from the cycle structure of g in the Sz sector.
  * ``kron_hamiltonian`` - H built from explicit spin matrices and Kronecker
    products (site 0 = leftmost factor = most significant bit).
  * ``projector_basis``  - symmetry-adapted vectors sum_g conj(chi(g)) g|s>
    written out in the unsymmetrized basis.
  * ``spin_correlations`` / ``structure_factor`` - <S_i.S_j> of a state
    from the definition of the spin operators, and their Fourier sum.
  * ``chirality_correlation`` / ``bond_correlation`` - the summed
    chirality-chirality and (connected) bond-bond correlations of the
    chirality and nematic order parameters (chapter on the triangular
    J1-J2-Jchi model), from explicit spin matrices; ``sector_state`` writes
    a sector eigenvector out in the unsymmetrized basis.
  * ``Fast``             - the thesis's own CPU method (``fast.c``): sublattice
    coding with 64-bit SymmetryAction tables per sublattice ("Sublattice
    Coding techniques", algorithms "Preparation of lookup tables for
    sublattice coding" and "Sublattice coding algorithm for finding the
    representative"), the sector basis by a substate walk with prefix
    pruning, and whole H.v products in the gather form of ``row_entries``.
    It reuses only the piece generator and the binary search of ``oracle.c``
    and is pinned against the brute-force functions above, so that whole
    products and short Lanczos runs at 36 and 40 sites have a CPU value.
  * ``lanczos``          - the real-symmetric two-vector step and the
    complex-Hermitian three-vector step ("The Lanczos algorithm"), no
    reorthogonalization; T-matrix eigenvalues by a library tridiagonal solver.
  * ``sun_*``            - SU(d) permutation models (chapter on SU(N) chiral
    spin liquids: H = J sum P_ij + i K3 sum (P_ijk - P_ijk^-1), d colors per
    site, fixed color counts): the same definitions as above - orbit minima,
    stabilizers, push-form matrix - over configurations written with two
    bits per site, in plain numpy.
  * ``mlp_*``            - float64 reference of the learned-index network
    (two hidden layers of 32 units, half relu(z) and half min(z, 0);
    forward, loss, analytic backward) used to check the GPU training
    kernels; its gradients are pinned by central differences.
"""
from __future__ import annotations

import ctypes
import os
from math import comb

import numpy as np
import scipy.linalg
import scipy.sparse

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_elem", ctypes.c_int32),
        ("perm", ctypes.c_void_p), ("flip", ctypes.c_void_p),
        ("chi_re", ctypes.c_void_p), ("chi_im", ctypes.c_void_p), ("chi_one", ctypes.c_void_p),
        ("n_bonds", ctypes.c_int32), ("bonds", ctypes.c_void_p), ("bond_J", ctypes.c_void_p),
        ("n_tri", ctypes.c_int32), ("tris", ctypes.c_void_p), ("tri_J", ctypes.c_void_p),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle.build import build
            build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(_Problem)
        vp = ctypes.c_void_p
        L.orc_enumerate.restype = ctypes.c_int64
        L.orc_enumerate.argtypes = [P, ctypes.c_int, vp, vp, ctypes.c_int64]
        L.orc_coo.restype = ctypes.c_int64
        L.orc_coo.argtypes = [P, vp, vp, ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int64]
        L.orc_rows.restype = ctypes.c_int64
        L.orc_rows.argtypes = [P, vp, ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int64, vp, vp]
        L.orc_rep_many.restype = None
        L.orc_rep_many.argtypes = [P, vp, ctypes.c_int64, vp, vp, vp, vp]
        L.orc_act.restype = ctypes.c_uint64
        L.orc_act.argtypes = [ctypes.c_int, vp, ctypes.c_int, ctypes.c_uint64]
        L.orc_find.restype = ctypes.c_int64
        L.orc_find.argtypes = [vp, ctypes.c_int64, ctypes.c_uint64]
        L.orc_max_terms.restype = ctypes.c_int
        L.orc_max_terms.argtypes = [P]
        L.orf_build.restype = vp
        L.orf_build.argtypes = [P, ctypes.c_int]
        L.orf_free.restype = None
        L.orf_free.argtypes = [vp]
        L.orf_enumerate.restype = ctypes.c_int64
        L.orf_enumerate.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int64]
        L.orf_find_rep_many.restype = None
        L.orf_find_rep_many.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp, vp]
        L.orf_rep_of.restype = ctypes.c_uint64
        L.orf_rep_of.argtypes = [vp, ctypes.c_int, ctypes.c_uint64]
        L.orf_sym_of.restype = ctypes.c_int
        L.orf_sym_of.argtypes = [vp, ctypes.c_int, ctypes.c_uint64, vp, ctypes.c_int]
        L.orf_apply.restype = ctypes.c_int
        L.orf_apply.argtypes = [P, vp, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int]
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


class Problem:
    """Keeps the instance arrays alive and exposes the C struct."""

    def __init__(self, inst):
        self.inst = inst
        self.perm = np.ascontiguousarray(inst.perms, dtype=np.int32)
        self.flip = np.ascontiguousarray(inst.flips, dtype=np.uint8)
        self.chi_re = np.ascontiguousarray(inst.chi.real, dtype=np.float64)
        self.chi_im = np.ascontiguousarray(inst.chi.imag, dtype=np.float64)
        # chi(g) == 1 decided in float64 with a tolerance far below the gap
        # between distinct roots of unity of order <= |G|
        self.chi_one = (np.abs(inst.chi - 1.0) < 1e-6).astype(np.uint8)
        self.bonds = np.ascontiguousarray(inst.bonds, dtype=np.int32).reshape(-1)
        self.bond_J = np.ascontiguousarray(inst.bond_J, dtype=np.float64)
        self.tris = np.ascontiguousarray(inst.tris, dtype=np.int32).reshape(-1)
        self.tri_J = np.ascontiguousarray(inst.tri_Jchi, dtype=np.float64)
        self.s = _Problem(inst.n_sites, inst.n_elem, _ptr(self.perm), _ptr(self.flip), _ptr(self.chi_re),
                          _ptr(self.chi_im), _ptr(self.chi_one), len(inst.bonds), _ptr(self.bonds),
                          _ptr(self.bond_J), len(inst.tris), _ptr(self.tris), _ptr(self.tri_J))

    @property
    def ref(self):
        return ctypes.byref(self.s)


class Fast:
    """The thesis's CPU method (fast.c): sublattice-coding tables with 64-bit
    SymmetryAction entries for n_sub sublattices (section "Sublattice Coding
    techniques", algorithms "Preparation of lookup tables for sublattice
    coding" and "Sublattice coding algorithm for finding the
    representative"), the sector basis, and whole H.v products in the pull
    form of row_entries.  Independent of the brute-force functions above,
    which pin it."""

    def __init__(self, inst, n_sub):
        self.inst = inst
        self.p = Problem(inst)
        self.h = lib().orf_build(self.p.ref, int(n_sub))
        if not self.h:
            raise ValueError(f"{n_sub} sublattices are not stable under the group (or the tables are too large)")

    def close(self):
        if self.h:
            lib().orf_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def rep_sym(self, X, s):
        """(Rep_X(s) as a substate, Sym_X(s)) for substate s of sublattice X."""
        L = lib()
        out = np.zeros(self.inst.n_elem, np.int32)
        k = L.orf_sym_of(self.h, int(X), int(s), _ptr(out), len(out))
        return int(L.orf_rep_of(self.h, int(X), int(s))), [int(g) for g in out[:k]]

    def rep_many(self, states):
        """(representative, first minimizing element, |Stab|, chi trivial on Stab)."""
        states = np.ascontiguousarray(states, np.uint64)
        n = len(states)
        rep = np.zeros(n, np.uint64)
        g = np.zeros(n, np.int32)
        st = np.zeros(n, np.int32)
        tv = np.zeros(n, np.int8)
        lib().orf_find_rep_many(self.h, _ptr(states), n, _ptr(rep), _ptr(g), _ptr(st), _ptr(tv))
        return rep, g, st, tv.astype(bool)

    def basis(self):
        L = lib()
        dim = L.orf_enumerate(self.h, self.inst.n_up, None, None, 0)
        if dim < 0:
            raise MemoryError("fast oracle: no memory for the enumeration counts")
        reps = np.zeros(dim, np.uint64)
        stabs = np.zeros(dim, np.int32)
        if dim:
            d2 = L.orf_enumerate(self.h, self.inst.n_up, _ptr(reps), _ptr(stabs), dim)
            assert d2 == dim
        return reps, stabs

    def apply(self, reps, stabs, x):
        """y = H x over the whole basis (x real or complex, basis order)."""
        reps = np.ascontiguousarray(reps, np.uint64)
        stabs = np.ascontiguousarray(stabs, np.int32)
        cplx = bool(np.iscomplexobj(x))
        xv = np.ascontiguousarray(x, np.complex128 if cplx else np.float64)
        y = np.zeros_like(xv)
        if lib().orf_apply(self.p.ref, self.h, _ptr(reps), _ptr(stabs), len(reps), _ptr(xv), _ptr(y), int(cplx)):
            raise MemoryError("fast oracle: no memory for the table of limits")
        return y


def enumerate_basis(inst):
    """Ascending list of sector representatives and their stabilizer sizes."""
    p = Problem(inst)
    L = lib()
    dim = L.orc_enumerate(p.ref, inst.n_up, None, None, 0)
    reps = np.zeros(dim, np.uint64)
    stabs = np.zeros(dim, np.int32)
    d2 = L.orc_enumerate(p.ref, inst.n_up, _ptr(reps), _ptr(stabs), dim)
    assert d2 == dim
    return reps, stabs


def coo_matrix(inst, reps, stabs):
    """Symmetrized Hamiltonian in the sector basis (push form), scipy CSR."""
    p = Problem(inst)
    L = lib()
    dim = len(reps)
    reps = np.ascontiguousarray(reps, np.uint64)
    stabs = np.ascontiguousarray(stabs, np.int32)
    nnz = L.orc_coo(p.ref, _ptr(reps), _ptr(stabs), dim, None, None, None, None, 0)
    ri = np.zeros(nnz, np.int64)
    ci = np.zeros(nnz, np.int64)
    vr = np.zeros(nnz)
    vi = np.zeros(nnz)
    n2 = L.orc_coo(p.ref, _ptr(reps), _ptr(stabs), dim, _ptr(ri), _ptr(ci), _ptr(vr), _ptr(vi), nnz)
    assert n2 == nnz
    vals = vr + 1j * vi if inst.is_complex else vr
    return scipy.sparse.csr_matrix((vals, (ri, ci)), shape=(dim, dim))


def row_entries(inst, rows):
    """Gather form for the given sector representatives.

    Returns (row_ptr, target_states, coefficients, row_ok, n_elements) so that
    y(rows[r]) = sum_{e in row r} coefficients[e] * x(target_states[e]).
    """
    p = Problem(inst)
    L = lib()
    rows = np.ascontiguousarray(rows, np.uint64)
    n = len(rows)
    rp = np.zeros(n + 1, np.int64)
    ok = np.zeros(n, np.int8)
    ne = np.zeros(n, np.int32)
    tot = L.orc_rows(p.ref, _ptr(rows), n, _ptr(rp), None, None, None, 0, _ptr(ok), _ptr(ne))
    tgt = np.zeros(tot, np.uint64)
    cr = np.zeros(tot)
    cim = np.zeros(tot)
    t2 = L.orc_rows(p.ref, _ptr(rows), n, _ptr(rp), _ptr(tgt), _ptr(cr), _ptr(cim), tot, _ptr(ok), _ptr(ne))
    assert t2 == tot
    return rp, tgt, cr + 1j * cim, ok.astype(bool), ne


def rows_apply(inst, rows, xfun):
    """y at the given rows for an input vector given as a function of the
    representative's integer value."""
    rp, tgt, coef, ok, ne = row_entries(inst, rows)
    vals = coef * xfun(tgt)
    y = np.zeros(len(rows), complex)
    np.add.at(y, np.repeat(np.arange(len(rows)), np.diff(rp)), vals)
    return y, ok, ne


def rep_many(inst, states):
    p = Problem(inst)
    L = lib()
    s = np.ascontiguousarray(states, np.uint64)
    n = len(s)
    rep = np.zeros(n, np.uint64)
    g = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    tv = np.zeros(n, np.int8)
    L.orc_rep_many(p.ref, _ptr(s), n, _ptr(rep), _ptr(g), _ptr(st), _ptr(tv))
    return rep, g, st, tv.astype(bool)


def act(inst, g, state):
    L = lib()
    perm = np.ascontiguousarray(inst.perms[g], np.int32)
    return int(L.orc_act(inst.n_sites, perm.ctypes.data, int(inst.flips[g]), int(state)))


# ---------------------------------------------------------------------------
# exact counts
# ---------------------------------------------------------------------------

def _cycles(perm):
    n = len(perm)
    seen = [False] * n
    out = []
    for i in range(n):
        if not seen[i]:
            L = 0
            j = i
            while not seen[j]:
                seen[j] = True
                j = int(perm[j])
                L += 1
            out.append(L)
    return out


def fixed_count(perm, flip, n_up):
    """Number of configurations with n_up up spins left invariant by g."""
    cyc = _cycles(perm)
    n = len(perm)
    if flip:
        if any(c % 2 for c in cyc) or 2 * n_up != n:
            return 0
        return 2 ** len(cyc)
    # subsets of cycles with total length n_up
    ways = [0] * (n_up + 1)
    ways[0] = 1
    for c in cyc:
        for s in range(n_up, c - 1, -1):
            ways[s] += ways[s - c]
    return ways[n_up]


def character_formula_dim(inst):
    tot = 0j
    for g in range(inst.n_elem):
        tot += np.conj(inst.chi[g]) * fixed_count(inst.perms[g], inst.flips[g], inst.n_up)
    d = tot / inst.n_elem
    assert abs(d.imag) < 1e-6 and abs(d.real - round(d.real)) < 1e-6, d
    return int(round(d.real))


def sz_states(n, n_up):
    """All n-bit integers with n_up set bits, ascending (n <= 24)."""
    x = np.arange(1 << n, dtype=np.uint64)
    pc = np.zeros(len(x), np.int64)
    for b in range(n):
        pc += ((x >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return x[pc == n_up]


# ---------------------------------------------------------------------------
# dense layer (small N)
# ---------------------------------------------------------------------------

_SZ = np.diag([-0.5, 0.5])                 # local basis (down, up): index bit 1 = up
_SP = np.array([[0.0, 0.0], [1.0, 0.0]])   # S^+ |down> = |up>
_SM = _SP.T
_SX = 0.5 * (_SP + _SM)
_SY = (_SP - _SM) / 2j


def _site_op(op, i, n):
    return scipy.sparse.kron(scipy.sparse.kron(scipy.sparse.identity(1 << i, format="csr"),
                                               scipy.sparse.csr_matrix(op)),
                             scipy.sparse.identity(1 << (n - 1 - i), format="csr"), format="csr")


def kron_hamiltonian(inst):
    """Full 2^N Hamiltonian from spin matrices and Kronecker products (sparse,
    N <= 14); site 0 is the leftmost factor."""
    n = inst.n_sites
    assert n <= 14
    S = {a: [_site_op(m, i, n) for i in range(n)] for a, m in (("x", _SX), ("y", _SY), ("z", _SZ))}
    H = scipy.sparse.csr_matrix((1 << n, 1 << n), dtype=complex)
    for (i, j), J in zip(inst.bonds.tolist(), inst.bond_J):
        for a in "xyz":
            H = H + J * (S[a][i] @ S[a][j])
    eps = {("x", "y", "z"): 1, ("y", "z", "x"): 1, ("z", "x", "y"): 1,
           ("x", "z", "y"): -1, ("z", "y", "x"): -1, ("y", "x", "z"): -1}
    for (i, j, k), J in zip(inst.tris.tolist(), inst.tri_Jchi):
        for (a, b, c), e in eps.items():
            H = H + (J * e) * (S[a][i] @ S[b][j] @ S[c][k])
    return H.tocsr()


def apply_group_numpy(inst, g, states):
    """g|s> on an array of states, via bit arrays (independent of orc_act)."""
    n = inst.n_sites
    s = np.asarray(states, np.uint64)
    bits = np.stack([(s >> np.uint64(n - 1 - i)) & np.uint64(1) for i in range(n)], axis=1)
    out_bits = np.zeros_like(bits)
    out_bits[:, inst.perms[g]] = bits
    if inst.flips[g]:
        out_bits = np.uint64(1) - out_bits
    out = np.zeros(len(s), np.uint64)
    for i in range(n):
        out |= out_bits[:, i] << np.uint64(n - 1 - i)
    return out


def projector_basis(inst, reps, states):
    """Columns sum_g conj(chi(g)) g|rep>, normalized, in the basis `states`."""
    pos = {int(s): k for k, s in enumerate(states)}
    B = np.zeros((len(states), len(reps)), complex)
    imgs = np.stack([apply_group_numpy(inst, g, reps) for g in range(inst.n_elem)])
    for c in range(len(reps)):
        for g in range(inst.n_elem):
            B[pos[int(imgs[g, c])], c] += np.conj(inst.chi[g])
    nrm = np.linalg.norm(B, axis=0)
    return B / nrm


def unsym_sector_matrix(inst):
    """Unsymmetrized Sz-sector Hamiltonian (trivial group) via the C oracle."""
    from dataclasses import replace
    triv = replace(inst, perms=np.arange(inst.n_sites, dtype=np.int32)[None, :],
                   flips=np.zeros(1, np.uint8), chi=np.ones(1, complex))
    reps, stabs = enumerate_basis(triv)
    return reps, coo_matrix(triv, reps, stabs)


def spin_correlations(inst, states, psi):
    """C[i, j] = <psi|S_i . S_j|psi> for a normalized psi over the ascending
    Sz configurations ``states`` (trivial group), from the definition
    S_i . S_j = S^z_i S^z_j + (S^+_i S^-_j + S^-_i S^+_j) / 2, bit by bit;
    C[i, i] = 3/4."""
    n = inst.n_sites
    s = np.asarray(states, np.uint64)
    p = np.asarray(psi)
    w = np.abs(p) ** 2
    bits = [((s >> np.uint64(n - 1 - i)) & np.uint64(1)).astype(bool) for i in range(n)]
    C = np.full((n, n), 0.75)
    for i in range(n):
        for j in range(i + 1, n):
            same = bits[i] == bits[j]
            zz = np.sum(w[same]) * 0.25 - np.sum(w[~same]) * 0.25
            anti = np.nonzero(~same)[0]
            t = s[anti] ^ (np.uint64(1) << np.uint64(n - 1 - i)) ^ (np.uint64(1) << np.uint64(n - 1 - j))
            k = np.searchsorted(s, t)
            flip = 0.5 * np.sum(np.conj(p[k]) * p[anti])
            C[i, j] = C[j, i] = zz + flip.real
    return C


def structure_factor(C, coords, q):
    """S(q) = (1/N) sum_{i,j} exp(2 pi i q.(r_i - r_j)) C[i, j], with r in
    lattice coordinates and q in the matching reciprocal units."""
    r = np.asarray(coords, float)
    ph = np.exp(2j * np.pi * (r @ np.asarray([float(c) for c in q], float)))
    return float(np.real(np.conj(ph) @ C @ ph)) / len(r)


def _spin_matrices(n):
    """S^a_i, a in x, y, z, as sparse 2^n matrices (site 0 leftmost)."""
    assert n <= 14
    return {a: [_site_op(m, i, n) for i in range(n)] for a, m in (("x", _SX), ("y", _SY), ("z", _SZ))}


def bond_operator(S, i, j):
    """S_i . S_j = sum_a S^a_i S^a_j."""
    return sum(S[a][i] @ S[a][j] for a in "xyz")


def chirality_operator(S, i, j, k):
    """S_i . (S_j x S_k) = sum_abc eps_abc S^a_i S^b_j S^c_k."""
    out = 0
    for (a, b, c), e in (((("x", "y", "z"), 1), (("y", "z", "x"), 1), (("z", "x", "y"), 1),
                          (("x", "z", "y"), -1), (("z", "y", "x"), -1), (("y", "x", "z"), -1))):
        out = out + e * (S[a][i] @ S[b][j] @ S[c][k])
    return out


def sector_state(inst, k=0):
    """The k-th lowest eigenvector of the symmetrized sector matrix written
    out in the unsymmetrized Sz configurations (ascending): returns (states,
    psi), psi normalized."""
    reps, stabs = enumerate_basis(inst)
    w, v = np.linalg.eigh(coo_matrix(inst, reps, stabs).toarray())
    states, _ = unsym_sector_matrix(inst)
    psi = projector_basis(inst, reps, states) @ v[:, k]
    return states, psi / np.linalg.norm(psi)


def _restricted(M, states):
    idx = np.asarray(states, np.int64)
    return M.tocsr()[idx][:, idx]


def chirality_correlation(inst, states, psi, t0, triangles):
    """sum_t <psi|chi_t0 chi_t|psi> over the triangles t (each (i, j, k)),
    chi = S_i . (S_j x S_k): the summed scalar-chirality correlation of the
    chirality order parameter (chapter on the triangular J1-J2-Jchi model),
    from spin matrices."""
    S = _spin_matrices(inst.n_sites)
    p = np.asarray(psi, complex)
    a = _restricted(chirality_operator(S, *t0), states) @ p
    tot = 0.0
    for t in triangles:
        tot += np.vdot(a, _restricted(chirality_operator(S, *t), states) @ p)
    return tot


def bond_correlation(inst, states, psi, b0, bonds, connected=True):
    """sum_b <psi|(S.S)_b0 (S.S)_b|psi> over the bonds b (each (i, j)), minus
    <(S.S)_b0><(S.S)_b> when connected: the nematic order parameter's sum
    over the bonds parallel to b0 (same chapter), from spin matrices."""
    S = _spin_matrices(inst.n_sites)
    p = np.asarray(psi, complex)
    B0 = _restricted(bond_operator(S, *b0), states)
    a = B0 @ p
    e0 = np.vdot(p, a)
    tot = 0.0
    for b in bonds:
        y = _restricted(bond_operator(S, *b), states) @ p
        tot += np.vdot(a, y) - (e0 * np.vdot(p, y) if connected else 0.0)
    return tot


def sector_resolvent(inst, psi, op_inst, z):
    """G(z) = <psi|O^dag (z - H)^-1 O|psi> for a vector psi of the sector
    (symmetrized basis, dense) and an operator O given as an instance with
    the sector's group: the spectral sum sum_n |<n|O psi>|^2 / (z - E_n)
    over the eigenpairs of the dense sector matrix (the quantity the
    continued-fraction expansion approximates, outlook chapter)."""
    reps, stabs = enumerate_basis(inst)
    w, V = np.linalg.eigh(coo_matrix(inst, reps, stabs).toarray())
    phi = coo_matrix(op_inst, reps, stabs).toarray() @ np.asarray(psi)
    amp2 = np.abs(V.conj().T @ phi) ** 2
    z = np.asarray(z, complex)
    return (amp2[None, :] / (z.reshape(-1, 1) - w[None, :])).sum(axis=1).reshape(z.shape)


# ---------------------------------------------------------------------------
# Lanczos
# ---------------------------------------------------------------------------

def lanczos(matvec, v0, n_iter, hermitian_complex=False, breakdown_tol=1e-14):
    """T-matrix coefficients from the two-vector (real) or three-vector
    (complex) Lanczos step.  Returns alpha[n], beta[n] where beta[k] is the
    norm produced at step k (so the T off-diagonal is beta[:-1])."""
    v = np.array(v0, dtype=complex if hermitian_complex else float)
    v = v / np.linalg.norm(v)
    alphas, betas = [], []
    if not hermitian_complex:
        w = np.zeros_like(v)
        beta = 0.0
        for _ in range(n_iter):
            w = matvec(v) - beta * w
            alpha = float(np.dot(w, v))
            w = w - alpha * v
            beta = float(np.sqrt(np.dot(w, w)))
            alphas.append(alpha)
            betas.append(beta)
            if beta < breakdown_tol * max(1.0, max(abs(a) for a in alphas)):
                break
            v, w = w, v
            v = v / beta
    else:
        vprev = np.zeros_like(v)
        beta = 0.0
        for _ in range(n_iter):
            w = matvec(v)
            alpha = float(np.vdot(w, v).real)
            w = w - alpha * v - beta * vprev
            vprev = v
            beta = float(np.sqrt(np.vdot(w, w).real))
            alphas.append(alpha)
            betas.append(beta)
            if beta < breakdown_tol * max(1.0, max(abs(a) for a in alphas)):
                break
            v = w / beta
    return np.array(alphas), np.array(betas)


def tmatrix_eigs(alpha, beta):
    n = len(alpha)
    if n == 1:
        return np.array(alpha, float)
    return scipy.linalg.eigh_tridiagonal(np.asarray(alpha, float), np.asarray(beta[: n - 1], float),
                                         eigvals_only=True)


# ---------------------------------------------------------------------------
# learned-index network reference (float64)
# ---------------------------------------------------------------------------

def _act(z):
    """Hidden activation: first half of the units relu(z), second half min(z, 0)."""
    h = z.shape[1] // 2
    out = z.copy()
    out[:, :h] = np.maximum(z[:, :h], 0.0)
    out[:, h:] = np.minimum(z[:, h:], 0.0)
    return out


def _dact(z):
    h = z.shape[1] // 2
    d = np.zeros_like(z)
    d[:, :h] = z[:, :h] > 0
    d[:, h:] = z[:, h:] < 0
    return d


def mlp_forward(params, X):
    """y = W3 act(W2 act(W1 x + b1) + b2) + b3 ; returns (y, cache)."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    a1 = _act(z1)
    z2 = a1 @ W2.T + b2
    a2 = _act(z2)
    y = a2 @ W3.T + b3
    return y[:, 0], (X, z1, a1, z2, a2)


def mlp_loss_grad(params, X, t):
    """Mean squared error 0.5 * mean((y - t)^2) and its analytic gradient."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, z1, a1, z2, a2) = mlp_forward(params, X)
    m = len(t)
    r = (y - t) / m
    loss = 0.5 * float(np.dot(y - t, y - t)) / m
    gW3 = r[None, :] @ a2
    gb3 = np.array([r.sum()])
    d2 = (r[:, None] @ W3) * _dact(z2)
    gW2 = d2.T @ a1
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * _dact(z1)
    gW1 = d1.T @ X
    gb1 = d1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def binom(n, k):
    return comb(n, k)


# ---------------------------------------------------------------------------
# SU(d) permutation models (chapter on SU(N) chiral spin liquids)
#
# A configuration of n sites with colors 0..d-1 is the integer
# sum_i color_i 4^(n-1-i): two bits per site, site 0 most significant, as
# for spin 1/2 with one bit.  The exchange P_ij swaps the colors of sites i
# and j; the ring exchange P_ijk moves the color of i to j, of j to k and of
# k to i.  H = sum_b J_b P_b + sum_t K_t i (P_t - P_t^-1).
# ---------------------------------------------------------------------------

def sun_digits(keys, n):
    """Colors [len(keys), n] of the configurations (site 0 first)."""
    keys = np.asarray(keys, np.uint64)
    return np.stack([((keys >> np.uint64(2 * (n - 1 - i))) & np.uint64(3)).astype(np.int64) for i in range(n)],
                    axis=1).reshape(len(keys), n)


def sun_keys(digits):
    digits = np.asarray(digits, np.int64)
    n = digits.shape[1]
    k = np.zeros(digits.shape[0], np.uint64)
    for i in range(n):
        k = (k << np.uint64(2)) | digits[:, i].astype(np.uint64)
    return k


def sun_states(n, d, counts):
    """All configurations with counts[c] sites of color c, ascending."""
    assert sum(counts) == n and len(counts) == d
    # multiset permutations, built color by color (plain recursion over sites)
    res = []

    def rec(prefix, left):
        if len(prefix) == n:
            res.append(list(prefix))
            return
        for c in range(d):
            if left[c]:
                left[c] -= 1
                prefix.append(c)
                rec(prefix, left)
                prefix.pop()
                left[c] += 1

    rec([], list(counts))
    keys = sun_keys(np.array(res, np.int64).reshape(-1, n))
    return np.sort(keys)


def sun_act(perm, keys, n):
    """Keys after the site permutation (the color at site i moves to perm[i])."""
    dg = sun_digits(keys, n)
    out = np.empty_like(dg)
    out[:, np.asarray(perm)] = dg
    return sun_keys(out)


def sun_rep_many(inst, keys):
    """Representative (orbit minimum), the first group element reaching it,
    stabilizer size and whether chi is trivial on the stabilizer."""
    keys = np.asarray(keys, np.uint64)
    n = inst.n_sites
    imgs = np.stack([sun_act(inst.perms[g], keys, n) for g in range(inst.n_elem)], axis=1)
    g = np.argmin(imgs, axis=1)
    rep = imgs[np.arange(len(keys)), g]
    fixed = imgs == keys[:, None]
    stab = fixed.sum(axis=1)
    chi_fixed = np.where(fixed, inst.chi[None, :], 1.0)
    triv = np.all(np.abs(chi_fixed - 1.0) < 1e-9, axis=1)
    return rep, g, stab, triv


def sun_enumerate_basis(inst):
    """Ascending sector representatives and stabilizer sizes."""
    st = sun_states(inst.n_sites, inst.local_dim, inst.counts)
    rep, g, stab, triv = sun_rep_many(inst, st)
    keep = (rep == st) & triv
    return st[keep], stab[keep].astype(np.int32)


def sun_terms(inst, keys):
    """Every non-branching piece applied to the configurations: a list of
    (targets, amplitudes); a piece that leaves a configuration unchanged is
    diagonal."""
    n = inst.n_sites
    dg = sun_digits(keys, n)
    out = []
    for (i, j), J in zip(inst.bonds.reshape(-1, 2), inst.bond_J):
        t = dg.copy()
        t[:, i], t[:, j] = dg[:, j], dg[:, i]
        out.append((sun_keys(t), np.full(len(keys), complex(J))))
    for (i, j, k), K in zip(inst.tris.reshape(-1, 3), inst.tri_Jchi):
        fwd = dg.copy()
        fwd[:, j], fwd[:, k], fwd[:, i] = dg[:, i], dg[:, j], dg[:, k]
        bwd = dg.copy()
        bwd[:, i], bwd[:, j], bwd[:, k] = dg[:, j], dg[:, k], dg[:, i]
        out.append((sun_keys(fwd), np.full(len(keys), 1j * K)))
        out.append((sun_keys(bwd), np.full(len(keys), -1j * K)))
    return out


def sun_coo_matrix(inst, reps, stabs):
    """Symmetrized Hamiltonian in the sector basis (push form), scipy CSR:
    H[i, j] += conj(chi(g)) sqrt(|Stab rep_i| / |Stab rep_j|) h for every
    piece h taking rep_j to a configuration whose representative rep_i =
    g(target) lies in the sector."""
    reps = np.asarray(reps, np.uint64)
    dim = len(reps)
    rows, cols, vals = [], [], []
    for tgt, h in sun_terms(inst, reps):
        rt, g, st, tv = sun_rep_many(inst, tgt)
        i = np.searchsorted(reps, rt)
        ok = tv & (i < dim)
        ok[ok] &= reps[i[ok]] == rt[ok]
        j = np.nonzero(ok)[0]
        v = np.conj(inst.chi[g[j]]) * np.sqrt(st[j] / stabs[j]) * h[j]
        rows.append(i[j])
        cols.append(j)
        vals.append(v)
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    if not inst.is_complex:
        vals = vals.real
    return scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def sun_rows_apply(inst, rows, xfun):
    """Pull form y(rep_i) = sum chi(g) sqrt(|Stab t~| / |Stab rep_i|) conj(h) x(t~)
    over the pieces of the given sector representatives (Hermiticity)."""
    rows = np.asarray(rows, np.uint64)
    _, _, srow, _ = sun_rep_many(inst, rows)
    y = np.zeros(len(rows), complex)
    for tgt, h in sun_terms(inst, rows):
        rt, g, st, tv = sun_rep_many(inst, tgt)
        c = np.where(tv, inst.chi[g] * np.sqrt(st / srow) * np.conj(h), 0.0)
        y += c * np.where(tv, xfun(rt), 0.0)
    return y


def sun_character_formula_dim(inst):
    """dim = |G|^-1 sum_g conj(chi(g)) Fix(g), Fix(g) = colorings constant on
    the cycles of g with the sector's color counts (dynamic programming over
    the cycles)."""
    d, counts = inst.local_dim, tuple(inst.counts)
    tot = 0j
    mag = 0
    for g in range(inst.n_elem):
        lens = _cycles(inst.perms[g])
        ways = {tuple([0] * d): 1}
        for L in lens:
            nxt = {}
            for used, w in ways.items():
                for c in range(d):
                    u = list(used)
                    u[c] += L
                    if u[c] <= counts[c]:
                        nxt[tuple(u)] = nxt.get(tuple(u), 0) + w
            ways = nxt
        tot += np.conj(inst.chi[g]) * ways.get(counts, 0)
        mag += ways.get(counts, 0)
    v = tot / inst.n_elem
    # the rounding error of the complex characters scales with the counts summed
    tol = 1e-12 * max(1.0, mag / inst.n_elem)
    assert abs(v.imag) < tol and abs(v.real - round(v.real)) < tol
    return int(round(v.real))


def sun_full_matrix(inst):
    """H on all configurations with the sector's color counts (no symmetry):
    the exchange and ring operators as permutations of the configurations."""
    st = sun_states(inst.n_sites, inst.local_dim, inst.counts)
    M = np.zeros((len(st), len(st)), complex)
    for tgt, h in sun_terms(inst, st):
        i = np.searchsorted(st, tgt)
        np.add.at(M, (i, np.arange(len(st))), h)
    return st, M


def sun_kron_operator(n, d, sites, cyc):
    """The permutation of colors on `sites` as a d^n x d^n matrix from
    Kronecker products (site 0 = leftmost factor): cyc = 2 gives P_ij, cyc =
    3 the ring P_ijk (color of i -> j -> k -> i)."""
    dim = d ** n
    M = np.zeros((dim, dim))
    for col in range(dim):
        dig = [(col // d ** (n - 1 - s)) % d for s in range(n)]
        new = list(dig)
        if cyc == 2:
            i, j = sites
            new[i], new[j] = dig[j], dig[i]
        else:
            i, j, k = sites
            new[j], new[k], new[i] = dig[i], dig[j], dig[k]
        row = sum(c * d ** (n - 1 - s) for s, c in enumerate(new))
        M[row, col] = 1.0
    return M


def sun_projector_basis(inst, reps):
    """Symmetry-adapted vectors sum_g conj(chi(g)) g|rep>, normalized, written
    out on the configurations of the sector (columns)."""
    st = sun_states(inst.n_sites, inst.local_dim, inst.counts)
    B = np.zeros((len(st), len(reps)), complex)
    for c, r in enumerate(np.asarray(reps, np.uint64)):
        for g in range(inst.n_elem):
            img = sun_act(inst.perms[g], np.array([r], np.uint64), inst.n_sites)[0]
            B[np.searchsorted(st, img), c] += np.conj(inst.chi[g])
        B[:, c] /= np.linalg.norm(B[:, c])
    return st, B
