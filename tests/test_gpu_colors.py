"""SU(d) permutation models on the GPU (ed_basis_build_colors and the
color kernels) against the oracle: small sectors entry by entry (basis,
stabilizers, element count, H.v in the plain and hashed lookups, index
lookup, Lanczos ground state), larger sectors on oracle-sampled rows, and
the d = 2 model against the spin-1/2 path at the same size
(J P_ij = 2 J S_i.S_j + J/2, K i (P_ijk - P_ijk^-1) = 4 K S_i.(S_j x S_k))."""
import sys

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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).cuda()


def _tri9(d, counts, K3, q=L.Q0):
    return L.sun_triangular((3, 0), (0, 3), d, counts, J=1.0, K3=K3, q=q, sublat_chain=[((1, 1), (2, -1))])


def _tri12(d, counts, K3, q=L.Q0):
    return L.sun_triangular((2, 2), (-2, 4), d, counts, J=1.0, K3=K3, q=q, sublat_chain=[((2, 0), (0, 2))])


def tri21_su3(K3=0.3):
    """SU(3) on the 21-site C6-symmetric triangular cluster, 7 sites of each
    color; sublattices: the seven cosets of the sqrt(7) superlattice."""
    return L.sun_triangular((4, 1), (-1, 5), 3, (7, 7, 7), J=1.0, K3=K3, sublat_chain=[((1, 2), (-2, 3))])


def tri16_su4(K3=0.25):
    """SU(4) on the 16-site (4 x 4) triangular cluster, 4 sites of each color."""
    return L.sun_triangular((4, 0), (0, 4), 4, (4, 4, 4, 4), J=1.0, K3=K3, sublat_chain=[((2, 0), (0, 2))])


SMALL = [
    L.sun_chain(6, 3, (2, 2, 2), k=1),
    L.sun_chain(6, 3, (2, 2, 2), K3=0.6, k=2),
    L.sun_chain(9, 3, (3, 3, 3), K3=-0.3, k=0, sublat=(3,)),
    L.sun_chain(10, 3, (4, 3, 3), k=5, reflection=True, sublat=(2,)),
    L.sun_chain(8, 4, (2, 2, 2, 2), k=3),
    L.sun_chain(12, 4, (3, 3, 3, 3), K3=0.4, k=0),
    L.sun_chain(12, 2, (6, 6), K3=0.3, k=4),
    _tri9(3, (3, 3, 3), 0.4),
    _tri9(3, (3, 3, 3), 0.0, q=(L.Fraction(1, 3), L.Fraction(1, 3))),
    _tri12(3, (4, 4, 4), 0.3),
    _tri12(4, (3, 3, 3, 3), 0.0),
]


def _rand(rng, d, cplx):
    x = rng.standard_normal(d)
    return x + 1j * rng.standard_normal(d) if cplx else x


@pytest.mark.parametrize("inst", SMALL, ids=lambda i: f"{i.name}-{i.sector}")
def test_small_color_sector_full_parity(S, inst):
    torch = _torch()
    _say("case", inst.name, inst.sector)
    reps_o, stabs_o = O.sun_enumerate_basis(inst)
    assert len(reps_o) == O.sun_character_formula_dim(inst)
    b = S.Basis.build(inst)
    info = b.info()
    assert info["n_colors"] == inst.local_dim and info["n_sites"] == inst.n_sites
    assert bool(info["is_complex"]) == inst.is_complex
    reps, stab = b.export()
    assert np.array_equal(reps, np.asarray(reps_o, np.uint64))
    assert np.array_equal(stab.astype(np.int64), np.asarray(stabs_o, np.int64))
    # element count: the diagonal plus every piece that changes the representative
    ne = len(reps_o)
    for tgt, h in O.sun_terms(inst, np.asarray(reps_o, np.uint64)):
        ne += int(np.count_nonzero((tgt != np.asarray(reps_o, np.uint64)) & (h != 0)))
    assert info["n_elements"] == ne
    H = O.sun_coo_matrix(inst, reps_o, stabs_o)
    rng = np.random.default_rng(23)
    x = _rand(rng, len(reps), inst.is_complex)
    ref = H @ x
    xt = _dev(torch, x)
    b.build_hash()
    for mode in (0, 2):
        yt = torch.zeros_like(xt)
        b.apply_H(xt, yt, mode=mode)
        torch.cuda.synchronize()
        err = np.max(np.abs(yt.cpu().numpy() - ref)) if len(reps) else 0.0
        _say("  mode", mode, "dim", len(reps), "max err", err)
        assert err < 1e-12
    # lookup of every representative, and of configurations that are not ones
    keys = _dev(torch, reps.view(np.int64))
    idx = torch.empty_like(keys)
    b.lookup(keys, idx)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), np.arange(len(reps)))
    rset = set(reps.tolist())
    nonrep = np.array([s for s in O.sun_states(inst.n_sites, inst.local_dim, inst.counts)[:3000].tolist()
                       if s not in rset], np.uint64)
    if len(nonrep):
        kt = _dev(torch, nonrep.view(np.int64))
        it = torch.empty_like(kt)
        b.lookup(kt, it)
        torch.cuda.synchronize()
        assert (it.cpu().numpy() == -1).all()
    # the learned index and the spin-1/2 observables do not take SU(d) bases
    with pytest.raises(S.EdError):
        b.train_index()
    b.free()


@pytest.mark.parametrize("inst", [SMALL[2], SMALL[9], SMALL[1]], ids=lambda i: f"{i.name}-{i.sector}")
def test_color_lanczos_ground_state(S, inst):
    torch = _torch()
    _say("lanczos", inst.name, inst.sector)
    reps_o, stabs_o = O.sun_enumerate_basis(inst)
    H = O.sun_coo_matrix(inst, reps_o, stabs_o)
    b = S.Basis.build(inst)
    v0 = V.start_vector(len(reps_o), 1003, inst.is_complex)
    n_iter = min(100, len(reps_o))
    exact = np.linalg.eigvalsh(H.toarray())[0]
    b.build_hash()
    for mode in (0, 2):
        a, beta, n, broken = b.lanczos(_dev(torch, v0), n_iter, mode=mode)
        e_gpu = S.eigenvalues(a, beta, 1)[0]
        _say("  mode", mode, "E0", e_gpu, "exact", exact)
        assert abs(e_gpu - exact) <= 1e-9 * abs(exact)
    ao, bo = O.lanczos(lambda v: H @ v, v0, n_iter, hermitian_complex=inst.is_complex)
    k = min(10, len(a), len(ao))
    assert np.max(np.abs(a[:k] - ao[:k])) < 1e-10
    b.free()


def _sampled_rows(inst, count, seed):
    st = V.random_color_states(inst.n_sites, inst.counts, count, seed)
    rep, g, stab, triv = O.sun_rep_many(inst, st)
    return np.unique(rep[triv])


def _large_color_parity(S, inst, n_rows, seed):
    torch = _torch()
    _say("large", inst.name, inst.sector)
    b = S.Basis.build(inst)
    info = b.info()
    _say("  built", info["dim"], "in", round(info["build_seconds"], 2), "s; sublattices", info["n_sub_rep"],
         info["n_sub_act"])
    assert info["dim"] == O.sun_character_formula_dim(inst)
    reps, _ = b.export()
    assert np.all(reps[1:] > reps[:-1])
    rows = _sampled_rows(inst, n_rows, seed)
    kt = _dev(torch, rows.view(np.int64))
    it = torch.empty_like(kt)
    b.lookup(kt, it)
    torch.cuda.synchronize()
    idx = it.cpu().numpy()
    assert (idx >= 0).all()
    assert np.array_equal(reps[idx], rows)
    ref = O.sun_rows_apply(inst, rows, lambda t: V.state_vector(t, 5151, inst.is_complex))
    if not inst.is_complex:
        ref = ref.real
    x = V.state_vector(reps, 5151, inst.is_complex)
    del reps
    xt = _dev(torch, x)
    del x
    b.build_hash()
    it_t = torch.from_numpy(idx).cuda()
    for mode in (0, 2):
        yt = torch.zeros_like(xt)
        b.apply_H(xt, yt, mode=mode)
        y = yt[it_t].cpu().numpy()
        del yt
        err = np.max(np.abs(y - ref))
        _say("  mode", mode, "rows", len(rows), "max err", err)
        assert err < 1e-12
    b.free()


def test_su3_triangular21_full_size(S):
    _large_color_parity(S, tri21_su3(), 4000, 7001)


def test_su4_triangular16_full_size(S):
    _large_color_parity(S, tri16_su4(), 4000, 7002)


def test_su3_triangular21_momentum_sector(S):
    inst = L.sun_triangular((4, 1), (-1, 5), 3, (7, 7, 7), J=1.0, K3=0.2, q=(L.Fraction(1, 7), L.Fraction(3, 7)),
                            sublat_chain=[((1, 2), (-2, 3))])
    _large_color_parity(S, inst, 3000, 7003)


def _spread(keys, n):
    """Spin-1/2 keys (one bit per site) to SU(2) keys (two bits per site)."""
    keys = np.asarray(keys, np.uint64)
    out = np.zeros_like(keys)
    for i in range(n):
        out |= ((keys >> np.uint64(i)) & np.uint64(1)) << np.uint64(2 * i)
    return out


def test_su2_model_equals_spin_half_path_at_27_sites(S):
    """The d = 2 permutation model and the spin-1/2 model with (2J, 4K) give
    the same basis (same digit strings, same order) and H.v up to sum J / 2."""
    import dataclasses
    torch = _torch()
    J, K = 0.8, 0.3
    su = L.sun_triangular((3, 3), (-3, 6), 2, (14, 13), J=J, K3=K, sublat_chain=[((1, 1), (-1, 2)), ((3, 0), (0, 3))])
    sp = dataclasses.replace(su, local_dim=0, counts=(), n_up=13, bond_J=2 * su.bond_J, tri_Jchi=4 * su.tri_Jchi)
    bc = S.Basis.build(su)
    bs = S.Basis.build(sp)
    rc, sc = bc.export()
    rs, ss = bs.export()
    _say("su2 vs spin-1/2 at 27 sites: dim", len(rc))
    assert len(rc) == len(rs) > 0
    assert np.array_equal(rc, _spread(rs, 27))
    assert np.array_equal(sc, ss)
    x = V.start_vector(len(rc), 4711, True)
    xt = _dev(torch, x)
    yc, ys = torch.zeros_like(xt), torch.zeros_like(xt)
    bc.apply_H(xt, yc)
    bs.apply_H(xt, ys)
    torch.cuda.synchronize()
    d = yc.cpu().numpy() - (ys.cpu().numpy() + 0.5 * su.bond_J.sum() * x)
    _say("  max diff", np.max(np.abs(d)))
    assert np.max(np.abs(d)) < 1e-11
    bc.free()
    bs.free()


def test_color_build_errors(S):
    import dataclasses
    inst = L.sun_chain(6, 3, (2, 2, 2), k=0)
    bad = dataclasses.replace(inst)
    bad.counts = (2, 2, 1)
    with pytest.raises(S.EdError) as e:
        S.Basis.build(bad)
    assert e.value.status == S.ED_EINVAL
    big = L.sun_chain(32, 2, (16, 16), k=0, sublat=(2,))
    with pytest.raises(S.EdError):
        S.Basis.build(big)  # 64 bits: more than 31 sites
    # an empty sector builds and applies
    b = S.Basis.build(L.sun_chain(6, 3, (6, 0, 0), k=1))
    assert b.info()["dim"] == 0
    b.free()
