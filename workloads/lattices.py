"""Problem instances for symmetrized exact diagonalization of spin-1/2 models.

This module only *describes* a problem: sites, bonds, oriented triangles, a
finite group of site permutations (optionally times a global spin flip) and a
one-dimensional irrep of that group given by its characters.  It holds none of
the method's arithmetic (no representative search, no matrix elements): both
the CPU oracle and the HIP library take the arrays it produces as input.

Conventions (thesis, section "Representing Hilbert spaces and operators",
eq. for int(sigma)):
  * a configuration of N spins is an N-bit integer; site 0 (the thesis's site
    1) is the most significant bit, spin up = 1;
  * a group element g moves the spin at site i to site perm[g, i]; if
    flip[g] is set, every spin is reversed afterwards;
  * composition: (g h) applies h first, perm_{gh} = perm_g o perm_h.

Sites are labelled so that every sublattice of the chosen decomposition is a
contiguous block of labels, sublattice 0 on the most significant bits
(section "Generic sublattice coding algorithm": site numbering).  A nested
chain of decompositions (coarse to fine) is kept contiguous in one labelling,
so the representative - which depends only on the labelling - is the same
for every N_sub in ``Instance.sublat_options``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np


@dataclass
class Instance:
    name: str
    n_sites: int
    bonds: np.ndarray          # int32 [nb, 2]
    bond_J: np.ndarray         # f64 [nb]
    tris: np.ndarray           # int32 [nt, 3], counter-clockwise (i, j, k)
    tri_Jchi: np.ndarray       # f64 [nt]
    n_up: int
    perms: np.ndarray          # int32 [n_elem, n_sites]
    flips: np.ndarray          # uint8 [n_elem]
    chi: np.ndarray            # complex128 [n_elem]
    sublat_options: list       # N_sub values contiguous in this labelling
    sector: str = ""
    meta: dict = field(default_factory=dict)
    # SU(d) permutation models (thesis chapter on SU(N) chiral spin liquids):
    # d colors per site, bond_J multiplies the exchange P_ij and tri_Jchi the
    # ring term i (P_ijk - P_ijk^-1); counts[c] sites carry color c.  0: the
    # spin-1/2 model above.
    local_dim: int = 0
    counts: tuple = ()

    def __post_init__(self):
        n = self.n_sites
        assert self.bonds.reshape(-1, 2).shape[0] == len(self.bond_J)
        assert self.tris.reshape(-1, 3).shape[0] == len(self.tri_Jchi)
        assert self.perms.ndim == 2 and self.perms.shape[1] == n
        assert len(self.flips) == len(self.chi) == self.perms.shape[0]
        assert self.bonds.size == 0 or (self.bonds.min() >= 0 and self.bonds.max() < n)
        if self.local_dim:
            assert 2 <= self.local_dim <= 4 and len(self.counts) == self.local_dim and sum(self.counts) == n
            assert not np.any(self.flips)

    @property
    def n_elem(self) -> int:
        return int(self.perms.shape[0])

    @property
    def is_complex(self) -> bool:
        return bool(np.any(np.abs(self.chi.imag) > 1e-12) or np.any(self.tri_Jchi != 0))

    @property
    def n_sublat(self) -> int:
        return int(max(self.sublat_options))


# ---------------------------------------------------------------------------
# integer lattice helpers (2D tori given in lattice coordinates)
# ---------------------------------------------------------------------------

def _cross(a, b):
    return a[0] * b[1] - a[1] * b[0]


def _reduce(r, L1, L2):
    """Canonical representative of r modulo the lattice spanned by L1, L2."""
    det = _cross(L1, L2)
    # coefficients a, b with r = a L1 + b L2 (rational)
    a = Fraction(_cross(r, L2), det)
    b = Fraction(_cross(L1, r), det)
    fa = a.numerator // a.denominator
    fb = b.numerator // b.denominator
    return (r[0] - fa * L1[0] - fb * L2[0], r[1] - fa * L1[1] - fb * L2[1])


def _in_lattice(r, L1, L2):
    return _reduce(r, L1, L2) == (0, 0)


def _matvec(P, r):
    return (P[0][0] * r[0] + P[0][1] * r[1], P[1][0] * r[0] + P[1][1] * r[1])


def _matmul(A, B):
    return tuple(tuple(sum(A[i][k] * B[k][j] for k in range(2)) for j in range(2)) for i in range(2))


def _group_closure(gens):
    I = ((1, 0), (0, 1))
    elems = [I]
    frontier = [I]
    while frontier:
        nxt = []
        for e in frontier:
            for g in gens:
                h = _matmul(g, e)
                if h not in elems:
                    elems.append(h)
                    nxt.append(h)
        frontier = nxt
    return elems


def one_dim_irreps(elems):
    """All one-dimensional irreps (homomorphisms to U(1)) of a small finite
    group of 2x2 integer matrices, as dicts element -> complex character."""
    order = len(elems)
    idx = {e: i for i, e in enumerate(elems)}
    mul = [[idx[_matmul(a, b)] for b in elems] for a in elems]
    # candidate values: order-th roots of unity; brute force on generators
    gens = []
    span = {idx[((1, 0), (0, 1))]}
    for e in elems:
        if idx[e] in span:
            continue
        gens.append(idx[e])
        # closure of gens
        cur = set(span) | {idx[e]}
        changed = True
        while changed:
            changed = False
            for a in list(cur):
                for g in gens:
                    c = mul[g][a]
                    if c not in cur:
                        cur.add(c)
                        changed = True
        span = cur
    roots = [np.exp(2j * np.pi * m / order) for m in range(order)]
    found = []
    for vals in itertools.product(range(order), repeat=len(gens)):
        chi = {idx[((1, 0), (0, 1))]: 1.0 + 0j}
        for g, v in zip(gens, vals):
            chi[g] = roots[v]
        ok = True
        changed = True
        while changed and ok:
            changed = False
            for a in list(chi):
                for g in gens:
                    c = mul[g][a]
                    val = chi[g] * chi[a]
                    if c in chi:
                        if abs(chi[c] - val) > 1e-9:
                            ok = False
                            break
                    else:
                        chi[c] = val
                        changed = True
                if not ok:
                    break
        if not ok or len(chi) != order:
            continue
        # full homomorphism check
        for a in range(order):
            for b in range(order):
                if abs(chi[mul[a][b]] - chi[a] * chi[b]) > 1e-9:
                    ok = False
                    break
            if not ok:
                break
        if ok:
            vec = tuple(np.round(chi[i].real, 12) + 1j * np.round(chi[i].imag, 12) for i in range(order))
            if vec not in [f[0] for f in found]:
                found.append((vec, {elems[i]: chi[i] for i in range(order)}))
    # trivial irrep first, then real ones, then complex
    found.sort(key=lambda f: (any(abs(v - 1) > 1e-9 for v in f[0]),
                              any(abs(v.imag) > 1e-9 for v in f[0])))
    return [f[1] for f in found]


def _torus_points(L1, L2):
    """Canonical representatives of all lattice points modulo L1, L2."""
    pts = set()
    R = max(abs(c) for c in tuple(L1) + tuple(L2)) + 1
    for x in range(-2 * R, 2 * R + 1):
        for y in range(-2 * R, 2 * R + 1):
            pts.add(_reduce((x, y), L1, L2))
    assert len(pts) == abs(_cross(L1, L2)), (len(pts), abs(_cross(L1, L2)))
    return pts


def _label_sites(pts, chain, L1, L2):
    """Site order: by coset along the sublattice chain (coarse to fine), then
    by coordinates.  Returns (ordered points, index, classes per level)."""
    coset_ids, opts = [], []
    for B1, B2 in chain:
        assert _in_lattice(L1, B1, B2) and _in_lattice(L2, B1, B2)
        reps = sorted({_reduce(p, B1, B2) for p in pts})
        coset_ids.append({p: reps.index(_reduce(p, B1, B2)) for p in pts})
        opts.append(len(reps))
    order = sorted(pts, key=lambda p: tuple(c[p] for c in coset_ids) + (p[1], p[0]))
    return order, {p: i for i, p in enumerate(order)}, opts


class Torus2D:
    """A Bravais lattice on a torus, in integer lattice coordinates.

    ``L1``, ``L2``: the torus periods; ``pg_gens``: generators of the point
    group (integer matrices acting on lattice coordinates); only elements
    that map the torus onto itself are kept.  ``sublat_chain``: sublattice
    subgroups (pairs of basis vectors) from coarse to fine; the finest one
    fixes the labelling.
    """

    def __init__(self, L1, L2, pg_gens, sublat_chain, cart=((1.0, 0.0), (0.0, 1.0))):
        self.L1, self.L2 = tuple(L1), tuple(L2)
        self.cart = np.array(cart, dtype=float)  # rows: a1, a2 cartesian
        pts = _torus_points(self.L1, self.L2)
        self.N = len(pts)
        self.pg = self._point_group(pg_gens)
        self.sublat_chain = [tuple(map(tuple, s)) for s in sublat_chain]
        self.coords, self.index, self.sublat_options = _label_sites(pts, self.sublat_chain, self.L1, self.L2)

    def _point_group(self, gens):
        """The elements of the group generated by ``gens`` that map the torus
        onto itself."""
        return [P for P in _group_closure(gens)
                if _in_lattice(_matvec(P, self.L1), self.L1, self.L2)
                and _in_lattice(_matvec(P, self.L2), self.L1, self.L2)]

    def site(self, r):
        return self.index[_reduce(r, self.L1, self.L2)]

    def translations(self):
        return list(self.coords)

    def perm(self, P, t):
        return np.array([self.site(_add(_matvec(P, r), t)) for r in self.coords], dtype=np.int32)

    def bonds(self, vectors):
        out = []
        for r in self.coords:
            for d in vectors:
                out.append((self.site(r), self.site(_add(r, d))))
        return out

    # momenta are defined modulo the dual of the translation lattice: the
    # integers for a Bravais torus
    q_period = Fraction(1)

    def reduce_q(self, q):
        m = self.q_period
        return tuple(x - m * ((x / m).numerator // (x / m).denominator) for x in q)

    def little_group(self, q):
        """Point-group elements P with P^T q = q modulo the dual lattice."""
        out = []
        for P in self.pg:
            qp = (P[0][0] * q[0] + P[1][0] * q[1], P[0][1] * q[0] + P[1][1] * q[1])
            if self.reduce_q(qp) == self.reduce_q(q):
                out.append(P)
        return out

    def momenta(self):
        """All allowed q (chi(t) = exp(2 pi i q.t)) as Fractions in [0,1)^2."""
        det = _cross(self.L1, self.L2)
        # dual basis: g_i . L_j = delta_ij  ->  G = (L^T)^-1
        L = [[self.L1[0], self.L2[0]], [self.L1[1], self.L2[1]]]  # columns L1, L2
        # (L^T)^-1 = adj(L^T)/det
        g1 = (Fraction(L[1][1], det), Fraction(-L[0][1], det))
        g2 = (Fraction(-L[1][0], det), Fraction(L[0][0], det))
        qs = set()
        for m1 in range(self.N):
            for m2 in range(self.N):
                q = (m1 * g1[0] + m2 * g2[0], m1 * g1[1] + m2 * g2[1])
                q = (q[0] - (q[0].numerator // q[0].denominator), q[1] - (q[1].numerator // q[1].denominator))
                qs.add(q)
        assert len(qs) == self.N
        return sorted(qs)

    def q_cart(self, q):
        """Cartesian k with k . (n1 a1 + n2 a2) = 2 pi (q1 n1 + q2 n2)."""
        A = self.cart  # rows a1, a2
        return np.linalg.solve(A, 2 * np.pi * np.array([float(q[0]), float(q[1])]))


def _add(a, b):
    return (a[0] + b[0], a[1] + b[1])


def _kagome_site(p):
    """A point of the fine triangular lattice is a kagome site unless both
    coordinates are even (those points are the hexagon centres)."""
    return (p[0] % 2, p[1] % 2) != (0, 0)


class KagomeTorus(Torus2D):
    """The kagome lattice on a torus, in coordinates of the triangular lattice
    of half its lattice constant (the "fine" lattice, a1 = (1, 0), a2 =
    (1/2, sqrt3/2)): its sites are the fine points with a coordinate odd, three
    per unit cell of the Bravais lattice 2 a1, 2 a2.  The removed points are
    the hexagon centres, so C6v about the origin maps the lattice onto itself.
    ``L1``, ``L2``: torus periods (even vectors); ``sublat_chain``: as for
    ``Torus2D``, even vectors, the classes of kagome sites modulo each being
    the sublattices (modulo (2, 0), (0, 2): the three kagome sublattices)."""

    q_period = Fraction(1, 2)

    def __init__(self, L1, L2, pg_gens, sublat_chain):
        self.L1, self.L2 = tuple(L1), tuple(L2)
        assert all(c % 2 == 0 for c in self.L1 + self.L2), "kagome torus periods must be even"
        self.cart = np.array(TRI_CART, dtype=float)
        pts = _torus_points(self.L1, self.L2)
        self.trans = sorted(p for p in pts if not _kagome_site(p))
        pts = {p for p in pts if _kagome_site(p)}
        self.N = len(pts)
        self.pg = self._point_group(pg_gens)
        self.sublat_chain = [tuple(map(tuple, c)) for c in sublat_chain]
        assert all(c % 2 == 0 for B in self.sublat_chain for v in B for c in v)
        self.coords, self.index, self.sublat_options = _label_sites(pts, self.sublat_chain, self.L1, self.L2)

    def translations(self):
        """The Bravais translations (even fine vectors) modulo the torus."""
        return list(self.trans)

    def momenta(self):
        """All allowed q (chi(t) = exp(2 pi i q.t) for even t) as Fractions
        in [0, 1/2)^2."""
        det = _cross(self.L1, self.L2)
        L = [[self.L1[0], self.L2[0]], [self.L1[1], self.L2[1]]]
        g1 = (Fraction(L[1][1], det), Fraction(-L[0][1], det))
        g2 = (Fraction(-L[1][0], det), Fraction(L[0][0], det))
        qs = set()
        for m1 in range(abs(det)):
            for m2 in range(abs(det)):
                qs.add(self.reduce_q((m1 * g1[0] + m2 * g2[0], m1 * g1[1] + m2 * g2[1])))
        assert len(qs) == len(self.trans)
        return sorted(qs)


def _pg_orbit(lat, q):
    orb = set()
    for P in lat.pg:
        qp = (P[0][0] * q[0] + P[1][0] * q[1], P[0][1] * q[0] + P[1][1] * q[1])
        orb.add(lat.reduce_q(qp))
    return orb


def build_group(lat: Torus2D, q, pg_irrep, flip_parity, little=None):
    """Group T x| L_q (x Z2 flip) with characters exp(2 pi i q.t) chi_rho(P) (+-1)^f.

    Characters of the space group follow the little-group construction
    (appendix "Representation theory for space groups"); the spin flip is a
    direct factor (section "Discrete symmetries", product of characters).
    """
    if little is None:
        little = lat.little_group(q)
    perms, flips, chis = [], [], []
    fl = [0] if flip_parity is None else [0, 1]
    for P in little:
        for t in lat.translations():
            perm = lat.perm(P, t)
            ph = np.exp(2j * np.pi * float(q[0] * t[0] + q[1] * t[1]))
            for f in fl:
                c = ph * pg_irrep[P] * (flip_parity if f else 1)
                perms.append(perm)
                flips.append(f)
                chis.append(c)
    chis = np.array(chis, dtype=np.complex128)
    chis.real[np.abs(chis.real) < 1e-15] = 0.0
    chis.imag[np.abs(chis.imag) < 1e-15] = 0.0
    return np.array(perms, dtype=np.int32), np.array(flips, dtype=np.uint8), chis


# ---------------------------------------------------------------------------
# concrete lattices
# ---------------------------------------------------------------------------

SQ_R90 = ((0, -1), (1, 0))
SQ_MX = ((-1, 0), (0, 1))
TRI_R60 = ((0, -1), (1, 1))        # a1 -> a2, a2 -> a2 - a1
TRI_MY = ((1, 1), (0, -1))         # a1 -> a1, a2 -> a1 - a2
TRI_C2 = ((-1, 0), (0, -1))        # inversion through a site
TRI_CART = ((1.0, 0.0), (0.5, np.sqrt(3.0) / 2.0))


def square_lattice(L1, L2, sublat_chain, mirrors=True, pg_gens=None):
    gens = pg_gens if pg_gens is not None else [SQ_R90] + ([SQ_MX] if mirrors else [])
    lat = Torus2D(L1, L2, gens, sublat_chain)
    lat.kind = "square"
    return lat


def triangular_lattice(L1, L2, sublat_chain, mirrors=False, pg_gens=None):
    gens = pg_gens if pg_gens is not None else [TRI_R60] + ([TRI_MY] if mirrors else [])
    lat = Torus2D(L1, L2, gens, sublat_chain, cart=TRI_CART)
    lat.kind = "triangular"
    return lat


def _irrep_by_name(little, name):
    irreps = one_dim_irreps(little)
    if name in ("A", "A1"):
        return irreps[0]
    if isinstance(name, int):
        return irreps[name]
    raise ValueError(name)


def square_j1j2(L1, L2, J1, J2, q, irrep="A1", flip=1, sublat_chain=None, mirrors=True,
                n_up=None, name="square", pg_gens=None):
    lat = square_lattice(L1, L2, sublat_chain, mirrors=mirrors, pg_gens=pg_gens)
    vec1 = [(1, 0), (0, 1)]
    vec2 = [(1, 1), (1, -1)]
    b1 = lat.bonds(vec1)
    b2 = lat.bonds(vec2) if J2 != 0 else []
    bonds = b1 + b2
    bJ = [J1] * len(b1) + [J2] * len(b2)
    little = lat.little_group(q)
    rho = _irrep_by_name(little, irrep)
    perms, flips, chis = build_group(lat, q, rho, flip, little)
    n = lat.N
    return Instance(name=name, n_sites=n, bonds=np.array(bonds, np.int32), bond_J=np.array(bJ, float),
                    tris=np.zeros((0, 3), np.int32), tri_Jchi=np.zeros(0), n_up=n // 2 if n_up is None else n_up,
                    perms=perms, flips=flips, chi=chis, sublat_options=lat.sublat_options,
                    sector=f"q={tuple(map(str, q))}.{irrep}.{_flipname(flip)}",
                    meta=dict(lattice=lat, little=little, q=q, irrep=0 if irrep in ("A", "A1") else irrep,
                              flip=flip))


def triangular_j1j2chi(L1, L2, J1, J2, Jchi, q, irrep="A", flip=1, sublat_chain=None, mirrors=None,
                       n_up=None, name="triangular", pg_gens=None):
    """Triangular J1-J2-Jchi model.  Point group: C6, with the mirrors when
    Jchi = 0 (``mirrors``), or the group generated by ``pg_gens``."""
    if mirrors is None:
        mirrors = (Jchi == 0)
    lat = triangular_lattice(L1, L2, sublat_chain, mirrors=mirrors, pg_gens=pg_gens)
    vec1 = [(1, 0), (0, 1), (-1, 1)]
    vec2 = [(1, 1), (-1, 2), (-2, 1)]
    b1 = lat.bonds(vec1)
    b2 = lat.bonds(vec2) if J2 != 0 else []
    bonds = b1 + b2
    bJ = [J1] * len(b1) + [J2] * len(b2)
    tris = []
    if Jchi != 0:
        up, down = _triangles(lat)
        tris = [t for pair in zip(up, down) for t in pair]
    little = lat.little_group(q)
    rho = _irrep_by_name(little, irrep)
    perms, flips, chis = build_group(lat, q, rho, flip, little)
    n = lat.N
    return Instance(name=name, n_sites=n, bonds=np.array(bonds, np.int32), bond_J=np.array(bJ, float),
                    tris=np.array(tris, np.int32).reshape(-1, 3), tri_Jchi=np.full(len(tris), float(Jchi)),
                    n_up=n // 2 if n_up is None else n_up, perms=perms, flips=flips, chi=chis,
                    sublat_options=lat.sublat_options,
                    sector=f"q={tuple(map(str, q))}.{irrep}.{_flipname(flip)}",
                    meta=dict(lattice=lat, little=little, q=q, irrep=0 if irrep in ("A", "A1") else irrep,
                              flip=flip))


KAG_VEC1 = [(1, 0), (0, 1), (-1, 1)]      # nearest neighbours (fine units)
KAG_VEC2 = [(1, 1), (-1, 2), (-2, 1)]      # second neighbours, distance sqrt3
KAG_VEC3 = [(1, 0), (0, 1), (-1, 1)]       # hexagon diagonals: r -> r + 2 d through a centre


def kagome_lattice(L1, L2, sublat_chain, mirrors=True, pg_gens=None):
    gens = pg_gens if pg_gens is not None else [TRI_R60] + ([TRI_MY] if mirrors else [])
    lat = KagomeTorus(L1, L2, gens, sublat_chain)
    lat.kind = "kagome"
    return lat


def kagome_j1j2j3chi(L1, L2, J1, J2, J3, Jchi, q, irrep="A", flip=1, sublat_chain=None, mirrors=None,
                     n_up=None, name="kagome", pg_gens=None):
    """Kagome J1-J2-J3-Jchi model (thesis chapter on the kagome chiral spin
    liquid, its Hamiltonian): J1 on nearest-neighbour bonds, J2 on second
    neighbours, J3 on third neighbours across the hexagons (the hexagon
    diagonals), Jchi S_i.(S_j x S_k) on every elementary triangle (up and
    down), counter-clockwise.  Point group C6v about a hexagon centre (C6
    when Jchi != 0)."""
    if mirrors is None:
        mirrors = (Jchi == 0)
    lat = kagome_lattice(L1, L2, sublat_chain, mirrors=mirrors, pg_gens=pg_gens)
    site = lat.index

    def pairs(vecs, step=1):
        out = []
        for r in lat.coords:
            for d in vecs:
                t = _reduce((r[0] + step * d[0], r[1] + step * d[1]), lat.L1, lat.L2)
                if t in site and (step == 1 or not _kagome_site(_add(r, d))):
                    out.append((site[r], site[t]))
        return out

    b1 = pairs(KAG_VEC1)
    b2 = pairs(KAG_VEC2) if J2 != 0 else []
    b3 = pairs(KAG_VEC3, 2) if J3 != 0 else []
    bonds = b1 + b2 + b3
    bJ = [J1] * len(b1) + [J2] * len(b2) + [J3] * len(b3)
    tris = []
    if Jchi != 0:
        # the fine triangles with no hexagon centre among their corners: up
        # triangles (r, r + a1, r + a2) at r with both coordinates odd, down
        # triangles (r + a1, r + a1 + a2, r + a2) at the centres
        for r in lat.coords + lat.translations():
            for tri in ((r, _add(r, (1, 0)), _add(r, (0, 1))),
                        (_add(r, (1, 0)), _add(r, (1, 1)), _add(r, (0, 1)))):
                red = [_reduce(v, lat.L1, lat.L2) for v in tri]
                if all(v in site for v in red):
                    tris.append(tuple(site[v] for v in red))
    little = lat.little_group(q)
    rho = _irrep_by_name(little, irrep)
    perms, flips, chis = build_group(lat, q, rho, flip, little)
    n = lat.N
    return Instance(name=name, n_sites=n, bonds=np.array(bonds, np.int32).reshape(-1, 2),
                    bond_J=np.array(bJ, float), tris=np.array(tris, np.int32).reshape(-1, 3),
                    tri_Jchi=np.full(len(tris), float(Jchi)),
                    n_up=n // 2 if n_up is None else n_up, perms=perms, flips=flips, chi=chis,
                    sublat_options=lat.sublat_options,
                    sector=f"q={tuple(map(str, q))}.{irrep}.{_flipname(flip)}",
                    meta=dict(lattice=lat, little=little, q=q, irrep=0 if irrep in ("A", "A1") else irrep,
                              flip=flip))


def _triangles(lat):
    """Elementary triangles, counter-clockwise: up (r, r + a1, r + a2) and
    down (r + a1, r + a1 + a2, r + a2), one of each per site r."""
    up = [(lat.site(r), lat.site(_add(r, (1, 0))), lat.site(_add(r, (0, 1)))) for r in lat.coords]
    down = [(lat.site(_add(r, (1, 0))), lat.site(_add(r, (1, 1))), lat.site(_add(r, (0, 1)))) for r in lat.coords]
    return up, down


def triangles(inst):
    """(up, down) counter-clockwise elementary triangles of a triangular
    instance, int32 arrays (N, 3) in its site labels."""
    up, down = _triangles(inst.meta["lattice"])
    return np.array(up, np.int32), np.array(down, np.int32)


def bonds_along(inst, d):
    """Bonds (r, r + d) for every site r of a torus instance, int32 (N, 2)."""
    lat = inst.meta["lattice"]
    return np.array([(lat.site(r), lat.site(_add(r, d))) for r in lat.coords], np.int32)


def _flipname(flip):
    return {None: "noflip", 1: "even", -1: "odd"}[flip]


def chain(N, J=1.0, k=0, flip=None, n_up=None, sublat=(2, 4), reflection=False, J2=0.0):
    """Periodic chain; translations T_n (site p -> p+n), chi(T_n) = exp(2 pi i k n / N).

    Labels: sublattices are residues mod m (nested chain ``sublat``), sites of
    one residue class contiguous, ordered by position.
    """
    pos = list(range(N))
    chain_m = list(sublat)
    order = sorted(pos, key=lambda p: tuple(p % m for m in chain_m) + (p,))
    lab = {p: i for i, p in enumerate(order)}
    bonds = [(lab[p], lab[(p + 1) % N]) for p in pos]
    bJ = [J] * N
    if J2 != 0:
        bonds += [(lab[p], lab[(p + 2) % N]) for p in pos]
        bJ += [J2] * N
    perms, flips, chis = [], [], []
    fl = [0] if flip is None else [0, 1]
    refl = [False, True] if reflection else [False]
    for r in refl:
        for t in range(N):
            perm = np.empty(N, np.int32)
            for p in pos:
                img = ((-p if r else p) + t) % N
                perm[lab[p]] = lab[img]
            ph = np.exp(2j * np.pi * k * t / N)
            for f in fl:
                perms.append(perm.copy())
                flips.append(f)
                chis.append(ph * (flip if f else 1))
    chis = np.array(chis, np.complex128)
    chis.real[np.abs(chis.real) < 1e-15] = 0.0
    chis.imag[np.abs(chis.imag) < 1e-15] = 0.0
    opts = [m for m in chain_m if N % m == 0]
    return Instance(name=f"chain{N}", n_sites=N, bonds=np.array(bonds, np.int32), bond_J=np.array(bJ, float),
                    tris=np.zeros((0, 3), np.int32), tri_Jchi=np.zeros(0),
                    n_up=N // 2 if n_up is None else n_up, perms=np.array(perms, np.int32),
                    flips=np.array(flips, np.uint8), chi=chis, sublat_options=opts,
                    sector=f"k={k}.{_flipname(flip)}", meta=dict(positions=order))


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

SQ32_L = ((4, 4), (-4, 4))
SQ32_CHAIN = [((1, 1), (1, -1)), ((2, 0), (0, 2)), ((2, 2), (-2, 2)), ((4, 0), (0, 4))]
SQ40_L = ((6, 2), (-2, 6))
SQ40_CHAIN = [((1, 1), (1, -1)), ((2, 0), (0, 2)), ((2, 2), (-2, 2))]
TRI36_L = ((6, 0), (0, 6))
TRI36_CHAIN = [((2, 0), (0, 2)), ((2, 2), (6, 0))]   # index 4, then 12 (= 4 x sqrt3 x sqrt3)
Q0 = (Fraction(0), Fraction(0))


def chain16():
    """Heisenberg chain N=16, periodic, J=1, Sz=0, translations only, k=0."""
    inst = chain(16, J=1.0, k=0, flip=None, sublat=(2, 4))
    inst.name = "chain16_k0"
    return inst


def square32(J2=0.5, q=Q0, irrep="A1", flip=1, sublat_chain=SQ32_CHAIN):
    """32-site square J1-J2 (torus (4,4),(-4,4)), full T x| C4v x Z2 at Gamma."""
    inst = square_j1j2(SQ32_L[0], SQ32_L[1], 1.0, J2, q, irrep=irrep, flip=flip, sublat_chain=sublat_chain)
    inst.name = "square32"
    return inst


def square40(J2=0.5, q=Q0, irrep="A", flip=1, sublat_chain=SQ40_CHAIN):
    """40-site square J1-J2 on the torus (6,2),(-2,6); point group C4 (no mirror
    maps this torus onto itself)."""
    inst = square_j1j2(SQ40_L[0], SQ40_L[1], 1.0, J2, q, irrep=irrep, flip=flip, sublat_chain=sublat_chain,
                       mirrors=False)
    inst.name = "square40"
    return inst


def tri36_K(J2=0.1, Jchi=0.2, flip=1, sublat_chain=TRI36_CHAIN):
    """36-site triangular J1-J2-Jchi at the K point, chi_K(t) = exp(2 pi i (t1 - t2)/3)."""
    q = (Fraction(1, 3), Fraction(-1, 3) + 1)
    inst = triangular_j1j2chi(TRI36_L[0], TRI36_L[1], 1.0, J2, Jchi, q, irrep="A", flip=flip,
                              sublat_chain=sublat_chain)
    inst.name = "triangular36_K"
    return inst


def _all_sectors(lat, make, n_up, name):
    """Every one-dimensional sector (k orbit x 1-D irrep of L_k, x flip parity
    at Sz = 0) of a torus model at the given number of up spins; ``make(q,
    irrep_index, flip)`` builds one instance.  Away from Sz = 0 the spin flip
    is not a symmetry of the sector, so it is left out of the group.
    Two-dimensional irreps of the little group are outside the
    one-dimensional method and not listed."""
    n = lat.N
    flips = (1, -1) if 2 * n_up == n else (None,)
    seen = set()
    out = []
    for q in lat.momenta():
        if q in seen:
            continue
        seen |= _pg_orbit(lat, q)
        little = lat.little_group(q)
        for ir_i, _ in enumerate(one_dim_irreps(little)):
            for fl in flips:
                inst = make(q, ir_i, fl)
                inst.name = (f"{name}{n}_Sz{Fraction(2 * n_up - n, 2)}_q{float(q[0]):.3f}_{float(q[1]):.3f}_ir{ir_i}"
                             + ("" if fl is None else f"_{_flipname(fl)}"))
                out.append(inst)
    return out


def square_sectors(L, chain, J2=0.5, n_up=None, name="square"):
    """Every one-dimensional sector of the square J1-J2 model (J1 = 1, point
    group C4v) on the torus L at the given number of up spins.  ``meta`` of
    each instance holds q, the irrep index (0 = A1, the trivial irrep) and
    the flip parity (None away from Sz = 0)."""
    lat = square_lattice(L[0], L[1], chain)
    n_up = lat.N // 2 if n_up is None else n_up
    return _all_sectors(lat, lambda q, ir, fl: square_j1j2(L[0], L[1], 1.0, J2, q, irrep=ir, flip=fl,
                                                           sublat_chain=chain, n_up=n_up), n_up, name)


def triangular_sectors(L, chain, J2=0.0, n_up=None, name="triangular"):
    """Every one-dimensional sector of the triangular J1-J2 model (J1 = 1,
    no chirality, point group C6v) on the torus L at the given number of up
    spins; ``meta`` as for ``square_sectors``."""
    lat = triangular_lattice(L[0], L[1], chain, mirrors=True)
    n_up = lat.N // 2 if n_up is None else n_up
    return _all_sectors(lat, lambda q, ir, fl: triangular_j1j2chi(L[0], L[1], 1.0, J2, 0.0, q, irrep=ir, flip=fl,
                                                                  sublat_chain=chain, mirrors=True, n_up=n_up),
                        n_up, name)


def pg_character(inst, P):
    """Character of the sector's point-group irrep on the little-group
    element P (an integer matrix on lattice coordinates)."""
    little = inst.meta["little"]
    return one_dim_irreps(little)[inst.meta["irrep"]][P]


def _momentum_name(kind, q):
    if kind == "kagome":
        # kagome momenta are taken modulo half the fine reciprocal lattice:
        # twice q names the point of the kagome Brillouin zone
        return _momentum_name("triangular", tuple(2 * x for x in q))
    h = Fraction(1, 2)
    names = {(Fraction(0), Fraction(0)): "Gamma"}
    if kind == "square":
        names[(h, h)] = "M"
    else:
        names.update({(Fraction(0), h): "M", (h, Fraction(0)): "M", (h, h): "M",
                      (Fraction(1, 3), Fraction(2, 3)): "K", (Fraction(2, 3), Fraction(1, 3)): "K"})
    return names.get(tuple(q), "(" + ",".join(str(c) for c in q) + ")")


def sector_label(inst):
    """'<momentum>.<irrep>' of a torus sector in the thesis's tower-of-states
    names: Gamma, M (square (1/2, 1/2); triangular the three edge centres), K
    (triangular corners (1/3, 2/3), (2/3, 1/3)); the trivial irrep is A1.  On
    the triangular lattice at Gamma the other one-dimensional irreps of C6v
    are named by their characters on the 60-degree rotation and on the
    mirror that contains the bond a1: A2 (+1, -1), B1 (-1, +1), B2 (-1, -1).
    Without mirrors (chirality on, point group C6) the trivial irrep is A;
    at Gamma the others are named by chi(C6) = exp(2 pi i m / 6): B (m = 3),
    E1a / E1b (m = 1 / 5), E2a / E2b (m = 2 / 4); at M (little group C2) the
    odd one is B.  Sectors of ``two_dim_sectors`` carry their E label.  Other
    irreps are 'ir<index>'."""
    if "label" in inst.meta:
        return inst.meta["label"]
    lat = inst.meta["lattice"]
    mom = _momentum_name(lat.kind, inst.meta["q"])
    ir = inst.meta["irrep"]
    little = inst.meta["little"]
    mirrored = any(P[0][0] * P[1][1] - P[0][1] * P[1][0] < 0 for P in little)
    if ir == 0:
        return f"{mom}.A1" if mirrored else f"{mom}.A"
    if lat.kind in ("triangular", "kagome") and mom == "Gamma" and TRI_MY in little:
        c = (round(pg_character(inst, TRI_R60).real), round(pg_character(inst, TRI_MY).real))
        return "Gamma." + {(1, -1): "A2", (-1, 1): "B1", (-1, -1): "B2"}[c]
    if lat.kind in ("triangular", "kagome") and mom == "Gamma" and TRI_R60 in little and not mirrored:
        m = int(round(np.angle(pg_character(inst, TRI_R60)) * 6 / (2 * np.pi))) % 6
        return "Gamma." + {3: "B", 1: "E1a", 5: "E1b", 2: "E2a", 4: "E2b"}[m]
    if mom == "M" and not mirrored and TRI_C2 in little and len(little) == 2:
        return "M.B"
    return f"{mom}.ir{ir}"


def two_dim_sectors(kind, L, chain, J2=0.0, n_up=None, name=None):
    """Sectors that hold the levels of the two-dimensional irreps of the
    point group, which the one-dimensional method cannot build directly.
    Where the little group of q is C_nv with n >= 3 (Gamma and M of the
    square lattice, Gamma and K of the triangular one), each 2-D irrep
    restricted to the rotations C_n is the pair of 1-D irreps with
    chi(R) = exp(+-2 pi i m / n), R the smallest rotation: m = 1 for E of
    C3v and C4v, m = 1 (E1) and m = 2 (E2) for C6v.  One sector per pair is
    built (the other holds the same levels), with the group T x| C_n
    (x flip at Sz = 0); ``meta['label']`` is '<momentum>.E', '.E1' or '.E2'.
    Each level of such a sector is one 2-D multiplet of the full group."""
    if kind == "square":
        full = square_lattice(L[0], L[1], chain, mirrors=True)
        rot = square_lattice(L[0], L[1], chain, mirrors=False)
        R, turns = SQ_R90, 4
    else:
        full = triangular_lattice(L[0], L[1], chain, mirrors=True)
        rot = triangular_lattice(L[0], L[1], chain, mirrors=False)
        R, turns = TRI_R60, 6
    n = full.N
    n_up = n // 2 if n_up is None else n_up
    flips = (1, -1) if 2 * n_up == n else (None,)
    seen = set()
    out = []
    for q in full.momenta():
        if q in seen:
            continue
        seen |= _pg_orbit(full, q)
        little = rot.little_group(q)
        order = len(little)
        if order < 3 or len(full.little_group(q)) != 2 * order:
            continue
        gen = ((1, 0), (0, 1))
        for _ in range(turns // order):
            gen = _matmul(R, gen)
        irreps = one_dim_irreps(little)
        mom = _momentum_name(kind, q)
        for m in range(1, (order - 1) // 2 + 1):
            target = np.exp(2j * np.pi * m / order)
            idx = next(i for i, ir in enumerate(irreps) if abs(ir[gen] - target) < 1e-9)
            lab = f"{mom}.E{m}" if order == 6 else f"{mom}.E"
            for fl in flips:
                if kind == "square":
                    inst = square_j1j2(L[0], L[1], 1.0, J2, q, irrep=idx, flip=fl, sublat_chain=chain,
                                       mirrors=False, n_up=n_up)
                else:
                    inst = triangular_j1j2chi(L[0], L[1], 1.0, J2, 0.0, q, irrep=idx, flip=fl, sublat_chain=chain,
                                              mirrors=False, n_up=n_up)
                inst.meta["label"] = lab
                inst.name = (f"{name or kind}{n}_Sz{Fraction(2 * n_up - n, 2)}_{lab}"
                             + ("" if fl is None else f"_{_flipname(fl)}"))
                out.append(inst)
    return out


def triangular_chiral_sectors(L, chain, J2=0.0, Jchi=0.0, n_up=None, name="triangular"):
    """Every one-dimensional sector of the triangular J1-J2-Jchi model with
    the point group C6 (the chirality is odd under the mirrors); every irrep
    of C6 and of its little groups is one-dimensional."""
    lat = triangular_lattice(L[0], L[1], chain, mirrors=False)
    n_up = lat.N // 2 if n_up is None else n_up
    return _all_sectors(lat, lambda q, ir, fl: triangular_j1j2chi(L[0], L[1], 1.0, J2, Jchi, q, irrep=ir, flip=fl,
                                                                  sublat_chain=chain, mirrors=False, n_up=n_up),
                        n_up, name)


def square32_sectors(J2=0.5, n_up=None):
    """Every one-dimensional sector of the 32-site square J1-J2 model."""
    out = square_sectors(SQ32_L, SQ32_CHAIN, J2, n_up)
    if n_up is None:
        for inst in out:
            q = inst.meta["q"]
            inst.name = (f"square32_q{float(q[0]):.3f}_{float(q[1]):.3f}_ir{inst.meta['irrep']}_"
                         f"{_flipname(inst.meta['flip'])}")
    return out


def square16_sectors(J2=0.0, n_up=None):
    """Every one-dimensional sector of the 16-site (4 x 4) square J1-J2 model."""
    return square_sectors(SQ16_L, SQ16_CHAIN, J2, n_up)


def triangular12_sectors(J2=0.0, n_up=None):
    """Every one-dimensional sector of the 12-site triangular J1-J2 model
    (C6v, with the K points)."""
    return triangular_sectors(TRI12_L, TRI12_CHAIN, J2, n_up)


def triangular36_sectors(J2=0.0, n_up=None):
    """Every one-dimensional sector of the 36-site (6 x 6) triangular J1-J2
    model (C6v)."""
    return triangular_sectors(TRI36_L, TRI36_CHAIN, J2, n_up)


# ---------------------------------------------------------------------------
# small instances: every feature of the method on sizes a dense check handles
# ---------------------------------------------------------------------------

SQ16_L = ((4, 0), (0, 4))
SQ16_CHAIN = [((1, 1), (1, -1)), ((2, 0), (0, 2))]
SQ20_L = ((4, 2), (-2, 4))
SQ20_CHAIN = [((1, 1), (1, -1)), ((2, 0), (0, 2))]
SQ8_L = ((2, 2), (-2, 2))
SQ8_CHAIN = [((1, 1), (1, -1))]
TRI12_L = ((2, 2), (-2, 4))
TRI12_CHAIN = [((2, 0), (0, 2))]
F = Fraction


def small_instances():
    """Diverse small sectors: translations only, dihedral chains, square and
    triangular point groups, spin flip, complex momenta, chirality."""
    out = []
    out.append(chain(8, k=0))
    out.append(chain(8, k=3))
    out.append(chain(10, k=0, flip=1))
    out.append(chain(10, k=5, flip=-1))
    out.append(chain(12, k=2, flip=-1, sublat=(2, 4)))
    out.append(chain(12, k=0, reflection=True, sublat=(2,), J2=0.4))
    out.append(chain(12, k=0, n_up=4, sublat=(2, 4)))
    s8 = square_j1j2(SQ8_L[0], SQ8_L[1], 1.0, 0.3, Q0, "A1", 1, SQ8_CHAIN, name="square8")
    out.append(s8)
    out.append(square_j1j2(SQ16_L[0], SQ16_L[1], 1.0, 0.5, Q0, "A1", 1, SQ16_CHAIN, name="square16"))
    out.append(square_j1j2(SQ16_L[0], SQ16_L[1], 1.0, 0.5, Q0, 1, -1, SQ16_CHAIN, name="square16"))
    out.append(square_j1j2(SQ16_L[0], SQ16_L[1], 1.0, 0.5, (F(1, 2), F(1, 2)), 2, 1, SQ16_CHAIN, name="square16"))
    out.append(square_j1j2(SQ16_L[0], SQ16_L[1], 1.0, 0.5, (F(1, 4), F(0)), 0, -1, SQ16_CHAIN, name="square16"))
    out.append(square_j1j2(SQ16_L[0], SQ16_L[1], 1.0, 0.5, (F(1, 4), F(1, 4)), 1, 1, SQ16_CHAIN, name="square16"))
    out.append(square_j1j2(SQ20_L[0], SQ20_L[1], 1.0, 0.5, Q0, "A", 1, SQ20_CHAIN, mirrors=False, name="square20"))
    out.append(square_j1j2(SQ20_L[0], SQ20_L[1], 1.0, 0.5, Q0, 2, -1, SQ20_CHAIN, mirrors=False, name="square20"))
    out.append(triangular_j1j2chi(TRI12_L[0], TRI12_L[1], 1.0, 0.1, 0.2, (F(1, 3), F(2, 3)), "A", 1,
                                  TRI12_CHAIN, name="triangular12"))
    out.append(triangular_j1j2chi(TRI12_L[0], TRI12_L[1], 1.0, 0.1, 0.2, (F(1, 3), F(2, 3)), 1, -1,
                                  TRI12_CHAIN, name="triangular12"))
    out.append(triangular_j1j2chi(TRI12_L[0], TRI12_L[1], 1.0, 0.1, 0.0, Q0, "A1", 1, TRI12_CHAIN,
                                  mirrors=True, name="triangular12"))
    out.append(triangular_j1j2chi(TRI12_L[0], TRI12_L[1], 1.0, 0.0, 0.3, (F(1, 2), F(0)), 1, None,
                                  TRI12_CHAIN, name="triangular12"))
    return out


KAG12_L = ((4, 0), (0, 4))                        # 2 x 2 unit cells
KAG12_CHAIN = [((2, 0), (0, 2))]                   # the three kagome sublattices
KAG27_L = ((6, 0), (0, 6))                        # 3 x 3 unit cells
KAG27_CHAIN = [((2, 0), (0, 2)), ((2, 2), (-2, 4))]   # 3 sublattices, then 9 (sqrt3 x sqrt3 cells)


def kagome_instances():
    """Small kagome sectors (J1-J2-J3-Jchi): C6v and chiral C6, momenta
    modulo the kagome reciprocal lattice, spin flip, Sz != 0."""
    Mq = (F(1, 4), F(0))           # an M point: half a reciprocal vector of the kagome lattice
    return [
        kagome_j1j2j3chi(KAG12_L[0], KAG12_L[1], 1.0, 0.0, 0.0, 0.0, Q0, "A1", 1, KAG12_CHAIN, name="kagome12"),
        kagome_j1j2j3chi(KAG12_L[0], KAG12_L[1], 1.0, 0.2, 0.1, 0.0, Q0, 1, -1, KAG12_CHAIN, name="kagome12"),
        kagome_j1j2j3chi(KAG12_L[0], KAG12_L[1], 1.0, 0.2, 0.1, 0.0, Mq, 2, 1, KAG12_CHAIN, name="kagome12"),
        kagome_j1j2j3chi(KAG12_L[0], KAG12_L[1], 1.0, 0.0, 0.0, 0.3, Q0, 1, 1, KAG12_CHAIN, name="kagome12"),
        kagome_j1j2j3chi(KAG12_L[0], KAG12_L[1], 1.0, 0.1, 0.0, 0.3, Mq, "A", None, KAG12_CHAIN, n_up=5,
                         name="kagome12"),
    ]


def kagome_sectors(L, chain, J2=0.0, J3=0.0, n_up=None, name="kagome"):
    """Every one-dimensional sector of the kagome J1-J2-J3 model (J1 = 1, no
    chirality, point group C6v about a hexagon centre) on the torus L at the
    given number of up spins; ``meta`` as for ``square_sectors``."""
    lat = kagome_lattice(L[0], L[1], chain, mirrors=True)
    n_up = lat.N // 2 if n_up is None else n_up
    return _all_sectors(lat, lambda q, ir, fl: kagome_j1j2j3chi(L[0], L[1], 1.0, J2, J3, 0.0, q, irrep=ir, flip=fl,
                                                                sublat_chain=chain, mirrors=True, n_up=n_up),
                        n_up, name)


def kagome27(J2=0.0, J3=0.0, Jchi=0.0, q=Q0, irrep="A", n_up=13):
    """27-site kagome (3 x 3 unit cells), Sz = 1/2 by default."""
    inst = kagome_j1j2j3chi(KAG27_L[0], KAG27_L[1], 1.0, J2, J3, Jchi, q, irrep, None, KAG27_CHAIN, n_up=n_up,
                            name="kagome27")
    return inst


def chain_distance_bonds(inst, r):
    """Bonds (i, i + r) for every position i of a chain instance, in its site
    labels, each with weight 1/N: sum_i S_i.S_(i+r) / N, the correlation at
    distance r of a translation-invariant state."""
    pos = inst.meta["positions"]          # label -> position
    n = inst.n_sites
    lab = {p: i for i, p in enumerate(pos)}
    bonds = np.array([(lab[p], lab[(p + r) % n]) for p in range(n)], np.int32)
    return bonds, np.full(n, 1.0 / n)


def site_coords(inst):
    """Lattice coordinates of every site label: (N, 2) integer lattice
    coordinates on a torus, or (N, 1) chain positions."""
    if "lattice" in inst.meta:
        return np.array(inst.meta["lattice"].coords, dtype=np.int64)
    return np.array(inst.meta["positions"], dtype=np.int64)[:, None]


def momentum_star(inst, q, pg=None):
    """The momenta P^T q (mod 1) over the point group of a torus instance
    (or over the matrices ``pg``), as Fractions (q itself for a chain)."""
    if "lattice" not in inst.meta:
        return [tuple(q)]
    out = []
    for P in (inst.meta["lattice"].pg if pg is None else pg):
        qp = (P[0][0] * q[0] + P[1][0] * q[1], P[0][1] * q[0] + P[1][1] * q[1])
        qp = tuple(c - (c.numerator // c.denominator) for c in qp)
        if qp not in out:
            out.append(qp)
    return out


# ---------------------------------------------------------------------------
# SU(N) permutation models: N colors per site (local dimension d = N)
# ---------------------------------------------------------------------------

def _sun_name(counts):
    return "c" + "-".join(str(c) for c in counts)


def sun_chain(N, d, counts, J=1.0, K3=0.0, k=0, reflection=False, sublat=(2, 4)):
    """Periodic SU(d) chain: J sum_i P_{i,i+1} (+ K3 on the triangles
    (i, i+1, i+2) when K3 != 0); translations with chi(T_n) = exp(2 pi i k n / N)."""
    base = chain(N, J=J, k=k, flip=None, sublat=sublat, reflection=reflection)
    lab = {p: i for i, p in enumerate(base.meta["positions"])}
    tris = np.zeros((0, 3), np.int32)
    if K3 != 0:
        tris = np.array([(lab[p], lab[(p + 1) % N], lab[(p + 2) % N]) for p in range(N)], np.int32)
    return Instance(name=f"su{d}chain{N}", n_sites=N, bonds=base.bonds, bond_J=base.bond_J, tris=tris,
                    tri_Jchi=np.full(len(tris), float(K3)), n_up=0, perms=base.perms, flips=base.flips,
                    chi=base.chi, sublat_options=base.sublat_options,
                    sector=f"k={k}.{_sun_name(counts)}", meta=base.meta, local_dim=d, counts=tuple(counts))


def sun_triangular(L1, L2, d, counts, J=1.0, K3=0.0, q=None, irrep="A", sublat_chain=None, pg_gens=None,
                   name="su_triangular"):
    """SU(d) Heisenberg model with imaginary ring exchange on the triangular
    lattice, H = J sum_<ij> P_ij + i K3 sum_(ijk) (P_ijk - P_ijk^-1), the
    ring term on every elementary triangle (up and down), counter-clockwise.
    Point group C6 (the ring term is odd under the mirrors) unless pg_gens
    is given."""
    q = Q0 if q is None else q
    lat = triangular_lattice(L1, L2, sublat_chain, mirrors=(K3 == 0) if pg_gens is None else False,
                             pg_gens=pg_gens)
    bonds = lat.bonds([(1, 0), (0, 1), (-1, 1)])
    tris = []
    if K3 != 0:
        up, down = _triangles(lat)
        tris = [t for pair in zip(up, down) for t in pair]
    little = lat.little_group(q)
    rho = _irrep_by_name(little, irrep)
    perms, flips, chis = build_group(lat, q, rho, None, little)
    return Instance(name=f"{name}{lat.N}", n_sites=lat.N, bonds=np.array(bonds, np.int32),
                    bond_J=np.full(len(bonds), float(J)), tris=np.array(tris, np.int32).reshape(-1, 3),
                    tri_Jchi=np.full(len(tris), float(K3)), n_up=0, perms=perms, flips=flips, chi=chis,
                    sublat_options=lat.sublat_options,
                    sector=f"q={tuple(map(str, q))}.{irrep}.{_sun_name(counts)}",
                    meta=dict(lattice=lat, little=little, q=q, irrep=0 if irrep in ("A", "A1") else irrep),
                    local_dim=d, counts=tuple(counts))
