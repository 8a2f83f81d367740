"""Lookup mode 2 (hashed staging table of {representative, x} records).

Every row sums the same terms in the same order whichever way x_j is found,
so H.v in mode 2 must equal mode 0 bit for bit, and so must the Lanczos
coefficients; both are also compared with the oracle.
"""
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
def test_hash_mode_equals_plain_and_oracle(S, inst):
    torch = _torch()
    _say("hash", inst.name, inst.sector)
    b = S.Basis.build(inst)
    st = b.build_hash()
    d = b.dim
    assert st["slots"] >= 2 * d - 1 and st["slots"] > d
    default = 0.25 if inst.is_complex else 0.15
    assert st["load"] == pytest.approx(default, abs=1.0 / d)   # the default load
    assert 1.0 <= st["mean_probes"] <= st["max_probes"]
    reps, stabs = b.export()
    x = V.start_vector(d, 31, inst.is_complex)
    xt = _dev(torch, x)
    y0 = torch.zeros_like(xt)
    y2 = torch.full_like(xt, 5.0)
    b.apply_H(xt, y0, mode=0)
    b.apply_H(xt, y2, mode=2)
    torch.cuda.synchronize()
    assert torch.equal(y0, y2)
    H = O.coo_matrix(inst, reps, stabs)
    assert np.max(np.abs(y2.cpu().numpy() - H @ x)) < 1e-12
    # lookups: members at their positions, non-members absent
    keys = _dev(torch, reps.view(np.int64))
    idx = torch.empty_like(keys)
    b.lookup(keys, idx, mode=2)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), np.arange(d))
    rset = set(reps.tolist())
    nonrep = np.array([s for s in O.sz_states(inst.n_sites, inst.n_up)[:3000].tolist() if s not in rset], np.uint64)
    if len(nonrep):
        kt = _dev(torch, nonrep.view(np.int64))
        it = torch.empty_like(kt)
        b.lookup(kt, it, mode=2)
        torch.cuda.synchronize()
        assert (it.cpu().numpy() == -1).all()
    b.free()


@pytest.mark.parametrize("load", [0.05, 0.3, 0.95])
def test_hash_loads(S, load):
    torch = _torch()
    inst = L.small_instances()[15]        # complex sector
    b = S.Basis.build(inst)
    st = b.build_hash(load=load)
    assert st["load"] == pytest.approx(load, rel=0.02, abs=2.0 / b.dim)
    x = _dev(torch, V.start_vector(b.dim, 5, True))
    y0 = torch.zeros_like(x)
    y2 = torch.zeros_like(x)
    b.apply_H(x, y0, mode=0)
    b.apply_H(x, y2, mode=2)
    torch.cuda.synchronize()
    assert torch.equal(y0, y2)
    # same load again: the stats; another load: refused
    assert b.build_hash(load=load)["slots"] == st["slots"]
    with pytest.raises(S.EdError):
        b.build_hash(load=0.5 if load != 0.5 else 0.4)
    b.free()


def test_hash_errors(S):
    torch = _torch()
    b = S.Basis.build(L.chain16())
    x = _dev(torch, V.start_vector(b.dim, 1))
    y = torch.zeros_like(x)
    with pytest.raises(S.EdError) as e:
        b.apply_H(x, y, mode=2)
    assert e.value.status == S.ED_EINVAL
    with pytest.raises(S.EdError):
        b.lanczos(x, 5, mode=2)
    for bad in (0.99, 0.01, -1.0):
        with pytest.raises(S.EdError):
            b.build_hash(load=bad)
    b.free()


@pytest.mark.parametrize("inst", [L.chain16(), L.small_instances()[13], L.small_instances()[15],
                                  L.small_instances()[11]], ids=lambda i: f"{i.name}-{i.sector}")
def test_hash_lanczos_identical(S, inst):
    torch = _torch()
    b = S.Basis.build(inst)
    b.build_hash()
    v0 = _dev(torch, V.start_vector(b.dim, 1002, inst.is_complex))
    n = min(60, b.dim)
    a0, b0, n0, br0 = b.lanczos(v0, n, mode=0)
    a2, b2, n2, br2 = b.lanczos(v0, n, mode=2)
    assert n0 == n2 and br0 == br2
    assert np.array_equal(a0, a2) and np.array_equal(b0, b2)
    reps, stabs = b.export()
    H = O.coo_matrix(inst, reps, stabs)
    ao, bo = O.lanczos(lambda v: H @ v, v0.cpu().numpy(), n, hermitian_complex=inst.is_complex)
    e2 = S.eigenvalues(a2, b2, 1)[0]
    eo = O.tmatrix_eigs(ao, bo)[0]
    assert abs(e2 - eo) <= 1e-10 * abs(eo)
    b.free()


@pytest.mark.parametrize("make", [L.square32, L.tri36_K, L.square40], ids=["square32", "triangular36", "square40"])
def test_hash_full_size_equals_plain(S, make):
    """At benchmark sizes: mode 2 equals mode 0 on every row."""
    torch = _torch()
    inst = make()
    _say("hash full size", inst.name)
    b = S.Basis.build(inst)
    st = b.build_hash()
    _say("  slots", st["slots"], "mean probes", round(st["mean_probes"], 3), "max", st["max_probes"],
         "build", round(st["build_seconds"], 2), "s")
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    dt = torch.complex128 if inst.is_complex else torch.float64
    x = torch.randn(b.dim, dtype=dt, device="cuda", generator=g)
    y0 = torch.zeros_like(x)
    b.apply_H(x, y0, mode=0)
    y2 = torch.zeros_like(x)
    b.apply_H(x, y2, mode=2)
    torch.cuda.synchronize()
    assert torch.equal(y0, y2)
    del y0, y2, x
    b.free()
