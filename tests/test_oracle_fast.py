"""CPU pins of the fast oracle (oracle/fast.c): the thesis's own CPU method
for the symmetrized H.v (section "Sublattice Coding techniques").

It is pinned against things it does not compute itself:
  - the printed sublattice-coding worked examples (Rep and Sym of every
    sublattice, the representative and its group element);
  - the brute-force orbit oracle (oracle.c), which it shares no arithmetic
    with: the sector basis and whole H.v products on every small instance and
    every stable sublattice count;
  - the 32-site stored values written by tests/golden/make_golden.py from the
    brute-force oracle (dimension, checksums of the representatives and
    stabilizers, sum and norm of one H.x);
  - representatives of 10^6 random configurations at each of 32, 36 and 40
    sites against the brute-force orbit minimum;
  - the character-formula dimension of the 36-site sector.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from workloads import lattices as L
from workloads import vectors as V

GOLD_DIR = os.path.join(os.path.dirname(__file__), "golden")
GOLD = json.load(open(os.path.join(GOLD_DIR, "worked_examples.json")))


def _state(bits):
    v = 0
    for ch in bits:
        v = (v << 1) | (ch == "u")
    return v


def _stable_counts(inst):
    out = []
    for ns in range(1, inst.n_sites + 1):
        if inst.n_sites % ns:
            continue
        try:
            F = O.Fast(inst, ns)
        except ValueError:
            continue
        out.append((ns, F))
    return out


@pytest.mark.parametrize("key,n_sub", [("two_sublattice", 2), ("three_sublattice", 3)])
def test_worked_example_tables_and_representative(key, n_sub):
    g = GOLD[key]
    inst = L.chain(g["n_sites"], sublat=(n_sub,))
    assert inst.meta["positions"] == g["chain_positions_by_label"]
    F = O.Fast(inst, n_sub)
    labels = "ABC"[:n_sub]
    for X, lab in enumerate(labels):
        rep, sym = F.rep_sym(X, _state(g["substates"][lab]))
        assert rep == g["rep"][lab], lab
        if lab in g["sym"]:
            assert sym == g["sym"][lab], lab
    s = _state(g["state"])
    rep, gm, st, tv = F.rep_many(np.array([s], np.uint64))
    assert int(rep[0]) == g["representative"] == _state(g["representative_state"])
    assert int(gm[0]) == g["g"]


def test_unstable_sublattices_rejected():
    # the 12-site triangular torus is not stable under 2, 3 or 6 sublattices
    # of consecutive sites in its 4-sublattice labelling
    inst = next(i for i in L.small_instances() if i.name.startswith("triangular12"))
    counts = [ns for ns, _ in _stable_counts(inst)]
    assert 1 in counts and inst.n_sites in counts
    for ns in (2, 3, 6):
        if ns not in counts:
            with pytest.raises(ValueError):
                O.Fast(inst, ns)


@pytest.mark.parametrize("inst", L.small_instances() + [L.chain16()] + L.kagome_instances(),
                         ids=lambda i: f"{i.name}-{i.sector}")
def test_basis_and_hv_equal_bruteforce(inst):
    reps, stabs = O.enumerate_basis(inst)
    H = O.coo_matrix(inst, reps, stabs)
    x = V.start_vector(len(reps), 7, inst.is_complex) if len(reps) else np.zeros(0)
    y_ref = H @ x
    stable = _stable_counts(inst)
    assert len(stable) >= 2
    for ns, F in stable:
        r2, s2 = F.basis()
        assert np.array_equal(r2, reps), ns
        assert np.array_equal(s2, stabs), ns
        if len(reps):
            y = F.apply(reps, stabs, x)
            scale = max(1.0, float(np.max(np.abs(y_ref))))
            assert np.max(np.abs(y - y_ref)) <= 1e-12 * scale, ns


def test_square32_stored_values():
    g = json.load(open(os.path.join(GOLD_DIR, "square32_gamma_a1_even.json")))
    F = O.Fast(L.square32(), 2)
    reps, stabs = F.basis()
    assert len(reps) == g["dim"]
    assert int(np.sum(reps, dtype=np.uint64)) == g["reps_sum_mod_2_64"]
    assert int(np.bitwise_xor.reduce(reps)) == g["reps_xor"]
    assert int(stabs.astype(np.int64).sum()) == g["stab_sum"]
    x = V.state_vector(reps, g["hv_state_vector_seed"])
    y = F.apply(reps, stabs, x)
    assert y.sum() == pytest.approx(g["hv_sum"], rel=1e-12)
    assert np.dot(y, y) == pytest.approx(g["hv_norm2"], rel=1e-12)


@pytest.mark.parametrize("make,n_sub", [(L.square32, 4), (L.tri36_K, 4), (L.square40, 4)],
                         ids=["square32", "triangular36_K", "square40"])
def test_representatives_at_full_size(make, n_sub):
    """10^6 uniformly random configurations of the Sz sector per lattice."""
    inst = make()
    F = O.Fast(inst, n_sub)
    rng = np.random.default_rng(11)
    n, m = inst.n_sites, 1_000_000
    states = np.zeros(m, np.uint64)
    for a in range(0, m, 250_000):
        # the n_up sites with the smallest of n uniform keys: a uniform subset
        up = np.argsort(rng.random((min(250_000, m - a), n)), axis=1)[:, :inst.n_up]
        states[a:a + len(up)] = np.bitwise_or.reduce(np.uint64(1) << (np.uint64(n - 1) - up.astype(np.uint64)),
                                                      axis=1)
    assert np.all(np.bitwise_count(states) == inst.n_up)
    rep, g, st, tv = F.rep_many(states)
    rep0, g0, st0, tv0 = O.rep_many(inst, states)
    assert np.array_equal(rep, rep0)
    assert np.array_equal(st, st0)
    assert np.array_equal(tv, tv0.astype(bool))
    # the reported element maps each state onto its representative
    for i in range(0, len(states), 9973):
        assert O.act(inst, int(g[i]), int(states[i])) == int(rep[i])


def test_triangular36_dimension_equals_character_formula():
    inst = L.tri36_K()
    F = O.Fast(inst, 4)
    dim = O.lib().orf_enumerate(F.h, inst.n_up, None, None, 0)
    assert dim == O.character_formula_dim(inst)
