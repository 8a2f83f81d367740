"""Learned index: gradients of the training kernels against the float64
oracle network, exact agreement of learned and plain lookups (every query,
found or absent), identical H.v and Lanczos results, and the gain of the
trained network over an untrained one."""
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


def _unpack(flat, F, H=32):
    o = 0
    W1 = flat[o:o + H * F].reshape(H, F); o += H * F
    b1 = flat[o:o + H]; o += H
    W2 = flat[o:o + H * H].reshape(H, H); o += H * H
    b2 = flat[o:o + H]; o += H
    W3 = flat[o:o + H].reshape(1, H); o += H
    b3 = flat[o:o + 1]; o += 1
    return [W1, b1, W2, b2, W3, b3], o


@pytest.mark.parametrize("F", [1, 5, 8])
def test_mlp_gradient_matches_oracle(S, F):
    torch = _torch()
    rng = np.random.default_rng(F)
    H = 32
    n_par = H * F + H + H * H + H + H + 1
    flat = (rng.standard_normal(n_par) * 0.3).astype(np.float32)
    n = 1000
    X = (rng.random((n, F)) - 0.5).astype(np.float32)
    t = rng.random(n).astype(np.float32)
    loss, grad = S.mlp_loss_grad(F, torch.from_numpy(flat).cuda(), torch.from_numpy(X).cuda(),
                                 torch.from_numpy(t).cuda())
    torch.cuda.synchronize()
    params, _ = _unpack(flat.astype(np.float64), F)
    ref_loss, ref_grads = O.mlp_loss_grad(params, X.astype(np.float64), t.astype(np.float64))
    ref = np.concatenate([g.reshape(-1) for g in ref_grads])
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(loss - ref_loss) <= 1e-4 * abs(ref_loss)
    scale = np.abs(ref).max()
    assert np.max(np.abs(g - ref)) <= 1e-3 * scale, np.max(np.abs(g - ref)) / scale


def _check_agreement(S, torch, b, reps, inst):
    d = len(reps)
    keys = torch.from_numpy(reps.view(np.int64)).cuda()
    i0 = torch.empty_like(keys)
    i1 = torch.empty_like(keys)
    b.lookup(keys, i0, mode=0)
    b.lookup(keys, i1, mode=1)
    torch.cuda.synchronize()
    assert torch.equal(i0, i1)
    assert np.array_equal(i1.cpu().numpy(), np.arange(d))
    # absent keys: random configurations of the sector that are not representatives,
    # neighbours of representatives, out-of-range keys
    st = V.random_sector_states(inst.n_sites, inst.n_up, 20000, 11)
    extra = np.concatenate([st, reps[:5000] + np.uint64(1), reps[:5000] - np.uint64(1),
                            np.array([0, (1 << inst.n_sites) - 1, 1 << inst.n_sites], np.uint64)])
    kt = torch.from_numpy(extra.view(np.int64)).cuda()
    j0 = torch.empty_like(kt)
    j1 = torch.empty_like(kt)
    b.lookup(kt, j0, mode=0)
    b.lookup(kt, j1, mode=1)
    torch.cuda.synchronize()
    assert torch.equal(j0, j1)


@pytest.mark.parametrize("inst", [L.chain16(), L.small_instances()[13], L.small_instances()[15], L.square32()],
                         ids=lambda i: f"{i.name}-{i.sector}")
def test_learned_lookup_is_exact(S, inst):
    torch = _torch()
    _say("learned", inst.name)
    b = S.Basis.build(inst)
    st = b.train_index(steps=600)
    _say("  stats", st)
    assert st["max_err"] <= 64
    reps, _ = b.export()
    _check_agreement(S, torch, b, reps, inst)
    # H.v identical to the plain lookup (same targets, same accumulation order)
    x = torch.from_numpy(V.start_vector(len(reps), 5, inst.is_complex)).cuda()
    y0 = torch.zeros_like(x)
    y1 = torch.zeros_like(x)
    b.apply_H(x, y0, mode=0)
    b.apply_H(x, y1, mode=1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    # another input: the records the learned gather reads must follow it
    x2 = (0.5 * x.flip(0)).contiguous()
    b.apply_H(x2, y0, mode=0)
    b.apply_H(x2, y1, mode=1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    a0, b0, _, _ = b.lanczos(x, 30, mode=0)
    a1, b1, _, _ = b.lanczos(x, 30, mode=1)
    assert np.array_equal(a0, a1) and np.array_equal(b0, b1)
    b.free()


def test_trained_network_gains_over_untrained(S):
    """The trained network shrinks the search windows of the same leaf and
    bucket tables (the buckets alone, behind an untrained network, already
    beat the plain Limits prefix table), and both beat the plain lookup."""
    torch = _torch()
    inst = L.square32()
    b = S.Basis.build(inst)
    plain = b.info()["limits_mean_window"]
    untrained = b.train_index(steps=1, lr=1e-9, log2_leaves=15)
    trained = b.train_index(steps=1500, log2_leaves=15)
    _say("plain", plain)
    _say("untrained", untrained)
    _say("trained", trained)
    assert trained["final_loss"] < 0.05 * untrained["final_loss"]
    assert trained["used_leaves"] > 4 * untrained["used_leaves"]
    assert trained["mean_window"] < 0.8 * untrained["mean_window"]
    assert trained["mean_window"] < 0.2 * plain
    reps, _ = b.export()
    _check_agreement(S, torch, b, reps, inst)
    # after retraining, the gather over the index's records still equals plain
    x = torch.from_numpy(V.start_vector(len(reps), 8, inst.is_complex)).cuda()
    y0 = torch.zeros_like(x)
    y1 = torch.zeros_like(x)
    b.apply_H(x, y0, mode=0)
    b.apply_H(x, y1, mode=1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)


def test_learned_index_requires_training(S):
    torch = _torch()
    b = S.Basis.build(L.chain16())
    x = torch.zeros(b.dim, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(S.EdError):
        b.apply_H(x, y, mode=1)


def test_large_leaf_table_stays_in_bounds(S):
    """2^24 leaves: the network output near 1 must map to the last leaf (the
    float value of 2^24 - 0.5 rounds up to 2^24, so the leaf index is clamped
    as an integer)."""
    torch = _torch()
    inst = L.square32()
    b = S.Basis.build(inst)
    st = b.train_index(steps=300, log2_leaves=24)
    assert st["n_leaves"] == 1 << 24
    reps, _ = b.export()
    _check_agreement(S, torch, b, reps, inst)


def test_expanded_network_equals_network(S):
    """The piecewise-linear expansion used for inference reproduces the
    trained float32 network evaluated in float64 by the oracle."""
    torch = _torch()
    inst = L.small_instances()[13]
    b = S.Basis.build(inst)
    st = b.train_index(steps=800)
    stats, w = b.index_weights()
    assert stats["n_pieces"] >= 2
    reps, _ = b.export()
    keys = torch.from_numpy(reps.view(np.int64)).cuda()
    u, y = b.index_predict(keys)
    torch.cuda.synchronize()
    params, _ = _unpack(w.astype(np.float64), 1)
    xs = (u.cpu().numpy().astype(np.float64) - stats["feature_offset"]) * stats["feature_scale"]
    yo, _ = O.mlp_forward(params, xs[:, None])
    assert np.max(np.abs(y.cpu().numpy() - yo)) <= 1e-5 * max(1.0, np.abs(yo).max())
    # the network is non-decreasing in the key
    assert np.all(np.diff(yo) >= -1e-6)


@pytest.mark.parametrize("make", [L.square40, L.tri36_K], ids=["square40", "triangular36"])
def test_learned_full_size_equals_plain(S, make):
    """At benchmark sizes: the learned-index H.v equals the plain lookup's on
    every row (real sectors read x from the index's records, complex ones
    from x)."""
    torch = _torch()
    inst = make()
    _say("learned full size", inst.name)
    b = S.Basis.build(inst)
    st = b.train_index()
    _say("  max_err", st["max_err"], "mean window", round(st["mean_window"], 2))
    assert st["max_err"] <= 64                 # leaves with larger buckets are refined
    g = torch.Generator(device="cuda")
    g.manual_seed(12)
    dt = torch.complex128 if inst.is_complex else torch.float64
    x = torch.randn(b.dim, dtype=dt, device="cuda", generator=g)
    y0 = torch.zeros_like(x)
    b.apply_H(x, y0, mode=0)
    y1 = torch.zeros_like(x)
    b.apply_H(x, y1, mode=1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    del y0, y1, x
    b.free()
