"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Small sectors: every representative, stabilizer, H.v entry and lookup is
compared with the oracle (bit-exact for integers, 1e-12 absolute for H.v),
Lanczos ground-state energies to 1e-10 relative.  Benchmark-size sectors:
basis size against the character formula, ordering and membership of
oracle-sampled representatives, and H.v on oracle-sampled rows for an input
vector defined by a counter-based hash of each representative.
"""
import os
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


SMALL = L.small_instances() + [L.chain16()]


@pytest.mark.parametrize("inst", SMALL, ids=lambda i: f"{i.name}-{i.sector}")
def test_small_sector_full_parity(S, inst):
    torch = _torch()
    _say("case", inst.name, inst.sector)
    reps_o, stabs_o = O.enumerate_basis(inst)
    b = S.Basis.build(inst)
    info = b.info()
    reps, stab = b.export()
    assert np.array_equal(reps, reps_o)
    assert np.array_equal(stab.astype(np.int64), stabs_o.astype(np.int64))
    # element count (diagonal + non-zero flipped pairs)
    _, _, _, ok, ne = O.row_entries(inst, reps_o)
    assert ok.all()
    assert info["n_elements"] == int(ne.sum())
    # H.v
    H = O.coo_matrix(inst, reps_o, stabs_o)
    rng = np.random.default_rng(17)
    d = len(reps)
    if inst.is_complex:
        x = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        xt = _dev(torch, x.astype(np.complex128))
        yt = torch.zeros_like(xt)
    else:
        x = rng.standard_normal(d)
        xt = _dev(torch, x)
        yt = torch.zeros_like(xt)
    b.apply_H(xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    ref = H @ x
    assert np.max(np.abs(y - ref)) < 1e-12
    # lookup: every representative found at its index, non-representatives absent
    keys = _dev(torch, reps.view(np.int64))
    idx = torch.empty_like(keys)
    b.lookup(keys, idx)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), np.arange(d))
    rset = set(reps.tolist())
    nonrep = np.array([s for s in O.sz_states(inst.n_sites, inst.n_up)[:4000].tolist() if s not in rset],
                      np.uint64)
    if len(nonrep):
        kt = _dev(torch, nonrep.view(np.int64))
        it = torch.empty_like(kt)
        b.lookup(kt, it)
        torch.cuda.synchronize()
        assert (it.cpu().numpy() == -1).all()
    b.free()


@pytest.mark.parametrize("case", [(8, 2, 2), (8, 2, 4), (8, 4, 4), (13, 2, 4), (13, 4, 4), (15, 4, 4),
                                  (5, 2, 2), (4, 2, 2), (8, 1, 4), (11, 1, 2), (12, 1, 4)], ids=str)
def test_explicit_decompositions(S, case):
    """Same basis and H.v for every admissible pair of decompositions.  R = 1
    (the whole lattice, always admissible) at 16 sites gives 16-bit Rep/Sym
    tables of over 512 KiB, which stay in device memory instead of LDS."""
    torch = _torch()
    k, R, A = case
    inst = L.small_instances()[k]
    if (R != 1 and R not in inst.sublat_options) or A not in inst.sublat_options:
        pytest.skip("decomposition not in this labelling")
    reps_o, stabs_o = O.enumerate_basis(inst)
    b = S.Basis.build(inst, n_sub_rep=R, n_sub_act=A, prefix_bits=3)
    info = b.info()
    assert (info["n_sub_rep"], info["n_sub_act"], info["prefix_bits"]) == (R, A, 3)
    if R == 1 and inst.n_sites == 16:
        assert info["table_bytes"] < 64 * 1024     # the Rep/Sym tables are not in the LDS blob
    reps, stab = b.export()
    assert np.array_equal(reps, reps_o)
    H = O.coo_matrix(inst, reps_o, stabs_o)
    x = V.start_vector(len(reps), 9, inst.is_complex)
    xt = _dev(torch, x)
    yt = torch.zeros_like(xt)
    b.apply_H(xt, yt)
    torch.cuda.synchronize()
    assert np.max(np.abs(yt.cpu().numpy() - H @ x)) < 1e-12


@pytest.mark.parametrize("inst", [L.chain16(), L.small_instances()[13], L.small_instances()[14],
                                  L.small_instances()[15], L.small_instances()[11]],
                         ids=lambda i: f"{i.name}-{i.sector}")
def test_lanczos_ground_state(S, inst):
    torch = _torch()
    _say("lanczos", inst.name, inst.sector)
    reps_o, stabs_o = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps_o, stabs_o)
    b = S.Basis.build(inst)
    v0 = V.start_vector(len(reps_o), 1002, inst.is_complex)
    n_iter = min(100, len(reps_o))
    a, beta, n, broken = b.lanczos(_dev(torch, v0), n_iter)
    ao, bo = O.lanczos(lambda v: H @ v, v0, n_iter, hermitian_complex=inst.is_complex)
    e_gpu = S.eigenvalues(a, beta, 1)[0]
    e_orc = O.tmatrix_eigs(ao, bo)[0]
    exact = np.linalg.eigvalsh(H.toarray())[0]
    assert abs(e_gpu - e_orc) <= 1e-10 * abs(e_orc)
    assert abs(e_gpu - exact) <= 1e-9 * abs(exact)
    # first alphas agree closely (no reorthogonalization: drift grows later)
    k = min(10, len(a), len(ao))
    assert np.max(np.abs(a[:k] - ao[:k])) < 1e-10
    b.free()


def test_chain16_reference_config(S):
    """Heisenberg chain N=16, k=0 (810 states), 100 Lanczos steps from a
    seeded N(0,1) start vector; energy agrees with the oracle to 1e-10."""
    torch = _torch()
    inst = L.chain16()
    reps_o, stabs_o = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps_o, stabs_o)
    b = S.Basis.build(inst)
    assert b.dim == 810
    v0 = V.start_vector(810, 1002)
    a, beta, n, broken = b.lanczos(_dev(torch, v0), 100)
    ao, bo = O.lanczos(lambda v: H @ v, v0, 100)
    e = S.eigenvalues(a, beta, 1)[0]
    eo = O.tmatrix_eigs(ao, bo)[0]
    assert abs(e - eo) <= 1e-10 * abs(eo)


def test_determinism(S):
    torch = _torch()
    inst = L.small_instances()[13]
    b = S.Basis.build(inst)
    x = _dev(torch, V.start_vector(b.dim, 3))
    y1 = torch.zeros_like(x)
    y2 = torch.zeros_like(x)
    b.apply_H(x, y1)
    b.apply_H(x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    a1, b1, _, _ = b.lanczos(x, 40)
    a2, b2, _, _ = b.lanczos(x, 40)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


def test_breakdown_on_tiny_sector(S):
    torch = _torch()
    inst = L.chain(4)
    b = S.Basis.build(inst)
    a, beta, n, broken = b.lanczos(_dev(torch, np.array([1.0, 0.3])), 10)
    assert broken and n == 2
    assert np.allclose(np.sort(S.eigenvalues(a, beta, 2)), [-2.0, 1.0])


def test_memory_cap(S):
    inst = L.small_instances()[13]
    with pytest.raises(S.EdError) as e:
        S.Basis.build(inst, mem_limit_bytes=1000)
    assert e.value.status == S.ED_ENOMEM


def test_memory_cap_counts_build_temporaries(S):
    """The cap counts the build's temporaries (chunk counts and offsets,
    scan sums) while they are held: a cap of exactly what the finished basis
    owns fails with ED_ENOMEM; one with room for the temporaries succeeds and
    the basis then owns the same bytes as without a cap."""
    inst = L.small_instances()[13]
    b = S.Basis.build(inst)
    owned = b.info()["bytes_device"]
    b.free()
    with pytest.raises(S.EdError) as e:
        S.Basis.build(inst, mem_limit_bytes=owned)
    assert e.value.status == S.ED_ENOMEM
    b2 = S.Basis.build(inst, mem_limit_bytes=owned + (64 << 20))
    assert b2.info()["bytes_device"] == owned
    b2.free()


def test_lanczos_arrays_are_replaced_not_kept(S):
    """Growing the alpha/beta arrays frees the old ones: after a 300-step run
    the basis owns the first run's bytes plus the growth of the two arrays
    (256 -> 512 entries each), not both generations."""
    torch = _torch()
    inst = L.chain16()
    b = S.Basis.build(inst)
    v0 = _dev(torch, V.start_vector(b.dim, 1002))
    b.lanczos(v0, 10)
    before = b.info()["bytes_device"]
    b.lanczos(v0, 300)
    after = b.info()["bytes_device"]
    assert after - before == 2 * (512 - 256) * 8
    b.free()


# --- benchmark-size sectors --------------------------------------------------

def _sampled_rows(inst, count, seed):
    """Oracle-side sample of sector representatives (rep of random configurations)."""
    st = V.random_sector_states(inst.n_sites, inst.n_up, count, seed)
    rep, g, stab, triv = O.rep_many(inst, st)
    return np.unique(rep[triv])


def _large_parity(S, inst, n_rows, seed, opts=None):
    """H.v of the full sector on oracle-sampled rows, in every lookup mode
    (plain, learned, hashed), against the oracle's gather form."""
    torch = _torch()
    _say("large", inst.name, inst.sector)
    b = S.Basis.build(inst, **(opts or {}))
    info = b.info()
    _say("  built", info["dim"], "in", round(info["build_seconds"], 2), "s")
    assert info["dim"] == O.character_formula_dim(inst)
    # ascending order on the device copy, checked on the host
    reps, _ = b.export()
    assert np.all(reps[1:] > reps[:-1])
    rows = _sampled_rows(inst, n_rows, seed)
    _say("  sampled rows", len(rows))
    assert len(rows) >= 0.9 * n_rows
    # oracle rows are sector representatives: they must be in the GPU basis
    kt = _dev(torch, rows.view(np.int64))
    it = torch.empty_like(kt)
    b.lookup(kt, it)
    torch.cuda.synchronize()
    idx = it.cpu().numpy()
    assert (idx >= 0).all()
    assert np.array_equal(reps[idx], rows)
    yo, ok, ne = O.rows_apply(inst, rows, lambda t: V.state_vector(t, 4242, inst.is_complex))
    assert ok.all()
    ref = yo if inst.is_complex else yo.real
    _say("  oracle elements", int(ne.sum()))
    # H.v on those rows with x(s) = hash(s), in all three lookups
    x = V.state_vector(reps, 4242, inst.is_complex)
    del reps
    xt = _dev(torch, x)
    del x
    b.train_index()
    b.build_hash()
    it_t = torch.from_numpy(idx).cuda()
    for mode in (0, 1, 2):
        yt = torch.zeros_like(xt)
        b.apply_H(xt, yt, mode=mode)
        y = yt[it_t].cpu().numpy()
        del yt
        err = np.max(np.abs(y - ref))
        _say("  mode", mode, "rows", len(rows), "max err", err)
        assert err < 1e-12
    del xt
    b.free()


def test_square32_full_size(S):
    _large_parity(S, L.square32(), 100_000, 2001)


def test_triangular36_full_size(S):
    _large_parity(S, L.tri36_K(), 100_000, 3001)


def test_square40_full_size(S):
    _large_parity(S, L.square40(), 100_000, 5001)


def test_square32_every_16th_row(S):
    """The whole 32-site sector at every 16th row (74,030 rows, about 4.9
    million matrix elements), element by element against the oracle's
    gather form, in every lookup mode."""
    torch = _torch()
    inst = L.square32()
    b = S.Basis.build(inst)
    reps, _ = b.export()
    rows_idx = np.arange(0, len(reps), 16)
    rows = reps[rows_idx]
    yo, ok, ne = O.rows_apply(inst, rows, lambda t: V.state_vector(t, 4242))
    assert ok.all()
    _say("  every 16th row:", len(rows), "rows,", int(ne.sum()), "elements")
    xt = _dev(torch, V.state_vector(reps, 4242))
    b.train_index()
    b.build_hash()
    it_t = torch.from_numpy(rows_idx).cuda()
    for mode in (0, 1, 2):
        yt = torch.zeros_like(xt)
        b.apply_H(xt, yt, mode=mode)
        y = yt[it_t].cpu().numpy()
        err = np.max(np.abs(y - yo.real))
        _say("  mode", mode, "max err", err)
        assert err < 1e-12
    b.free()


def test_square32_against_stored_oracle_values(S):
    """The 32-site square sector against values the oracle wrote
    (tests/golden/make_golden.py): basis checksums, H.v of a counter-based
    vector on every row (sum and squared norm), and 100 Lanczos steps from
    the seeded start vector, in every lookup mode."""
    import json
    torch = _torch()
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "square32_gamma_a1_even.json")))
    inst = L.square32()
    b = S.Basis.build(inst)
    assert b.dim == gold["dim"]
    # 16-bit coarse substates: the Rep/Sym tables (1.4 MB) stay out of LDS
    info = b.info()
    assert info["n_sub_rep"] == 2 and info["table_bytes"] < 64 * 1024
    reps, stab = b.export()
    assert int(np.sum(reps, dtype=np.uint64)) == gold["reps_sum_mod_2_64"]
    assert int(np.bitwise_xor.reduce(reps)) == gold["reps_xor"]
    assert int(stab.astype(np.int64).sum()) == gold["stab_sum"]
    b.train_index()
    b.build_hash()
    x = _dev(torch, V.state_vector(reps, gold["hv_state_vector_seed"]))
    v0 = _dev(torch, V.start_vector(b.dim, gold["lanczos_seed"]))
    for mode in (0, 1, 2):
        y = torch.zeros_like(x)
        b.apply_H(x, y, mode=mode)
        torch.cuda.synchronize()
        yh = y.cpu().numpy()
        assert abs(yh.sum() - gold["hv_sum"]) <= 1e-9 * gold["hv_norm2"] ** 0.5
        assert abs(np.dot(yh, yh) - gold["hv_norm2"]) <= 1e-10 * gold["hv_norm2"]
        a, be, n, broken = b.lanczos(v0, gold["lanczos_steps"], mode=mode)
        assert n == gold["lanczos_steps"] and not broken
        assert np.max(np.abs(a[:10] - np.array(gold["alpha_first10"]))) < 1e-10
        assert np.max(np.abs(be[:10] - np.array(gold["beta_first10"]))) < 1e-10
        e = S.eigenvalues(a, be, 1)[0]
        _say("  mode", mode, "E0", repr(e))
        assert abs(e - gold["E0_after_100"]) <= 1e-10 * abs(gold["E0_after_100"])
    b.free()


def test_lanczos_resume_equals_one_run(S):
    """A run resumed in chunks (across the growth of the alpha/beta arrays
    and across lookup modes) gives the coefficients of one run, bit for bit."""
    torch = _torch()
    inst = L.chain16()
    b = S.Basis.build(inst)
    b.train_index(steps=200)
    b.build_hash()
    v0 = _dev(torch, V.start_vector(b.dim, 1002))
    a1, b1, n1, br1 = b.lanczos(v0, 300, mode=0)
    assert n1 == 300 and not br1
    a2, b2, n2, _ = b.lanczos(v0, 120, mode=0)
    parts_a, parts_b = [a2], [b2]
    for mode, k in ((1, 100), (2, 80)):
        a3, b3, n3, br3 = b.lanczos_resume(k, mode=mode)
        assert n3 == k and not br3
        parts_a.append(a3)
        parts_b.append(b3)
    assert np.array_equal(np.concatenate(parts_a), a1)
    assert np.array_equal(np.concatenate(parts_b), b1)
    b.free()


def test_lanczos_resume_errors(S):
    torch = _torch()
    b = S.Basis.build(L.chain(4))
    with pytest.raises(S.EdError) as e:
        b.lanczos_resume(3)
    assert e.value.status == S.ED_EINVAL
    a, beta, n, broken = b.lanczos(_dev(torch, np.array([1.0, 0.3])), 10)
    assert broken and n == 2
    a2, b2, n2, broken2 = b.lanczos_resume(5)
    assert broken2 and n2 == 0


def test_single_state_and_empty_sectors(S):
    """Degenerate sectors: one state (all spins down: four bonds give +1/4
    each) and none (k = 1 with all spins down: the character is not trivial
    on the stabilizer)."""
    torch = _torch()
    one = L.chain(4, n_up=0)
    b = S.Basis.build(one)
    assert b.dim == 1
    x = _dev(torch, np.array([2.0]))
    for mode in (0, 2):
        if mode == 2:
            b.build_hash()
        y = torch.zeros_like(x)
        b.apply_H(x, y, mode=mode)
        torch.cuda.synchronize()
        assert y.item() == 2.0
    a, beta, n, broken = b.lanczos(x, 5)
    assert n == 1 and broken and a[0] == pytest.approx(1.0, abs=1e-15)
    keys = _dev(torch, np.array([0, 1, 5], np.int64))
    idx = torch.empty_like(keys)
    b.lookup(keys, idx)
    torch.cuda.synchronize()
    assert idx.cpu().tolist() == [0, -1, -1]
    b.free()
    empty = L.chain(4, k=1, n_up=0)
    e = S.Basis.build(empty)
    assert e.dim == 0 and e.info()["n_elements"] == 0
    z = torch.zeros(0, dtype=torch.complex128, device="cuda")
    e.apply_H(z, torch.zeros_like(z))           # nothing to do
    keys = _dev(torch, np.array([0, 3], np.int64))
    idx = torch.empty_like(keys)
    e.lookup(keys, idx)
    torch.cuda.synchronize()
    assert idx.cpu().tolist() == [-1, -1]
    for call in (lambda: e.lanczos(z, 3), lambda: e.build_hash(), lambda: e.train_index(steps=10)):
        with pytest.raises(S.EdError) as err:
            call()
        assert err.value.status == S.ED_EINVAL
    e.free()


@pytest.mark.parametrize("case", [(48, 3, 0, (2, 4, 8, 16)), (60, 57, 7, (2, 4, 12)), (63, 3, 0, (3, 9)),
                                  (63, 60, 5, (3, 9)), (56, 53, 11, (2, 4, 8))], ids=str)
def test_large_n_sparse_sectors(S, case):
    """Up to 63 sites (the largest N of the 64-bit encoding), at Sz far from 0
    so the oracle finishes in milliseconds; with most spins up the
    representatives carry bits up to the top of the encoding.  The 48-, 56-
    and 60-site rings keep their 12- to 15-bit Rep/Sym tables in device
    memory.  Basis bit-exact, H.v against the oracle and identical in all
    three lookups."""
    torch = _torch()
    N, n_up, k, sub = case
    inst = L.chain(N, k=k, n_up=n_up, sublat=sub)
    _say("large N", N, n_up, k)
    reps_o, stabs_o = O.enumerate_basis(inst)
    b = S.Basis.build(inst)
    reps, stab = b.export()
    assert np.array_equal(reps, reps_o) and np.array_equal(stab.astype(np.int64), stabs_o.astype(np.int64))
    H = O.coo_matrix(inst, reps_o, stabs_o)
    x = V.start_vector(len(reps), 21, inst.is_complex)
    ref = H @ x
    b.train_index(steps=200)
    b.build_hash()
    xt = _dev(torch, x)
    ys = []
    for mode in (0, 1, 2):
        yt = torch.zeros_like(xt)
        b.apply_H(xt, yt, mode=mode)
        torch.cuda.synchronize()
        ys.append(yt)
        assert np.max(np.abs(yt.cpu().numpy() - ref)) < 1e-12
    assert torch.equal(ys[0], ys[1]) and torch.equal(ys[0], ys[2])
    keys = _dev(torch, reps.view(np.int64))
    for mode in (0, 1, 2):
        idx = torch.empty_like(keys)
        b.lookup(keys, idx, mode=mode)
        torch.cuda.synchronize()
        assert np.array_equal(idx.cpu().numpy(), np.arange(len(reps)))
    b.free()


def test_no_admissible_decomposition_is_refused(S):
    """A 48-site ring labelled by residues mod 2 and 4 only: 4 sublattices of
    12 bits give more distinct SymmetryAction tables than 48 KiB hold, and
    finer contiguous decompositions do not exist in that labelling.  The
    build refuses it with ED_ENOTSTABLE and says why."""
    _torch()
    with pytest.raises(S.EdError) as e:
        S.Basis.build(L.chain(48, n_up=3, sublat=(2, 4)))
    assert e.value.status == S.ED_ENOTSTABLE
    assert "SymmetryAction" in str(e.value)


# --- stored values of the fast CPU oracle at 36 and 40 sites -----------------

def _fast_oracle_gold(name):
    import json
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not written (tests/golden/make_golden_large.py)")
    return json.load(open(path))


@pytest.mark.parametrize("make,name", [(L.tri36_K, "triangular36_K.json"),
                                       (L.square40, "square40_gamma_a_even.json")],
                         ids=["triangular36_K", "square40"])
def test_full_size_against_fast_oracle(S, make, name):
    """The 36-site triangular K sector and the 40-site square sector against
    whole-sector values of the fast CPU oracle: basis checksums; one H.x over
    every row (sum, squared norm, <x, Hx>, and every stride-th row element
    by element); the first Lanczos coefficients and the lowest Ritz value
    from the seeded start vector - in every lookup mode."""
    torch = _torch()
    gold = _fast_oracle_gold(name)
    inst = make()
    cplx = inst.is_complex
    _say("fast-oracle gold", inst.name, inst.sector)
    b = S.Basis.build(inst)
    assert b.dim == gold["dim"]
    reps, stab = b.export()
    assert int(np.sum(reps, dtype=np.uint64)) == gold["reps_sum_mod_2_64"]
    assert int(np.bitwise_xor.reduce(reps)) == gold["reps_xor"]
    assert int(stab.astype(np.int64).sum()) == gold["stab_sum"]
    x = V.state_vector(reps, gold["hv_state_vector_seed"], cplx)
    del reps, stab
    xt = _dev(torch, x)
    rows = np.arange(0, gold["dim"], gold["hv_stride"])
    ref = np.array(gold["hv_rows"])
    if cplx:
        ref = ref[:, 0] + 1j * ref[:, 1]
    hv_sum = complex(*gold["hv_sum"])
    norm = gold["hv_norm2"] ** 0.5
    b.train_index()
    b.build_hash()
    v0 = _dev(torch, V.start_vector(gold["dim"], gold["lanczos_seed"], cplx))
    it_t = torch.from_numpy(rows).cuda()
    for mode in (0, 1, 2):
        yt = torch.zeros_like(xt)
        b.apply_H(xt, yt, mode=mode)
        torch.cuda.synchronize()
        err = float(np.max(np.abs(yt[it_t].cpu().numpy() - ref)))
        s = complex(yt.sum().item())
        n2 = float(torch.vdot(yt, yt).real.item()) if cplx else float(torch.dot(yt, yt).item())
        xhx = float(torch.vdot(xt, yt).real.item()) if cplx else float(torch.dot(xt, yt).item())
        del yt
        _say("  mode", mode, "rows", len(rows), "max err", err, "sum", s, "norm2", n2)
        assert err < 1e-12
        assert abs(s - hv_sum) <= 1e-10 * norm
        assert abs(n2 - gold["hv_norm2"]) <= 1e-11 * gold["hv_norm2"]
        assert abs(xhx - gold["hv_xHx"]) <= 1e-10 * norm * float(torch.linalg.vector_norm(xt).item())
        k = gold["lanczos_steps"]
        a, be, n, broken = b.lanczos(v0, k, mode=mode)
        assert n == k and not broken
        assert np.max(np.abs(a[:k] - np.array(gold["alpha"]))) <= 1e-10 * max(1.0, np.max(np.abs(gold["alpha"])))
        assert np.max(np.abs(be[:k] - np.array(gold["beta"]))) <= 1e-10 * max(1.0, np.max(gold["beta"]))
        e = S.eigenvalues(a, be, 1)[0]
        _say("  mode", mode, "Ritz value after", k, "steps", repr(e), "oracle", gold["ritz0"])
        assert abs(e - gold["ritz0"]) <= 1e-10 * abs(gold["ritz0"])
    del xt, v0
    b.free()


# --- kagome J1-J2-J3-Jchi ----------------------------------------------------

@pytest.mark.parametrize("inst", L.kagome_instances(), ids=lambda i: f"{i.name}-{i.sector}")
def test_kagome_sector_full_parity(S, inst):
    """12-site kagome sectors (C6v, chiral C6, M point, flip, Sz != 0):
    basis, element count, H.v on every row and lookups against the oracle,
    as for the other small sectors; and the Lanczos ground state against the
    oracle's dense spectrum."""
    test_small_sector_full_parity(S, inst)
    torch = _torch()
    reps_o, stabs_o = O.enumerate_basis(inst)
    exact = np.linalg.eigvalsh(O.coo_matrix(inst, reps_o, stabs_o).toarray())[0]
    b = S.Basis.build(inst)
    v0 = V.start_vector(len(reps_o), 1002, inst.is_complex)
    a, beta, n, broken = b.lanczos(_dev(torch, v0), len(reps_o))
    e = S.eigenvalues(a[:n], beta[:n], 1)[0]
    _say("  E0", repr(e), "dense", repr(exact))
    assert abs(e - exact) <= 1e-9 * max(1.0, abs(exact))
    b.free()


@pytest.mark.parametrize("make", [lambda: L.kagome27(J2=0.2, J3=0.1), lambda: L.kagome27(Jchi=0.3)],
                         ids=["kagome27_C6v", "kagome27_chiral"])
def test_kagome27_sampled_rows(S, make):
    """27-site kagome at Sz = 1/2 (C6v: 186,616 states; chiral C6: 372,044
    complex): basis count, order and membership, and H.v on oracle-sampled
    rows in every lookup mode."""
    _large_parity(S, make(), 20_000, 7001)
