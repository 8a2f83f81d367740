"""Learned index: gradients of the training kernels against the float64
oracle network, exact agreement of learned and plain lookups (every query,
found or absent), identical H.v and Lanczos results, the recorded windows
(every representative inside the window of its own cell), and the gain of
the trained network over an untrained one and over no network."""
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
    assert st["mean_window"] <= st["max_err"]
    assert 0.0 <= st["frac_exact"] <= 1.0 and st["mean_lines"] >= 1.0
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


@pytest.mark.parametrize("routing", [1, 2], ids=["untrained", "no-network"])
def test_every_routing_is_exact(S, routing):
    """The tables below the network are built for whatever picks the
    segment, so the untrained network and no network at all give exact
    lookups too (only slower ones)."""
    torch = _torch()
    inst = L.square32()
    b = S.Basis.build(inst)
    st = b.train_index(routing=routing)
    _say("  routing", routing, st)
    assert st["routing"] == routing
    reps, _ = b.export()
    _check_agreement(S, torch, b, reps, inst)
    x = torch.from_numpy(V.start_vector(len(reps), 6)).cuda()
    y0 = torch.zeros_like(x)
    y1 = torch.zeros_like(x)
    b.apply_H(x, y0, mode=0)
    b.apply_H(x, y1, mode=1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    b.free()


def test_trained_network_gains_over_untrained(S):
    """Same segment and cell tables behind three routings, built to the same
    window bound.  The trained network fills more segments than the untrained
    one, misplaces keys by far less, and so needs far fewer cells (the
    refinement makes up for bad routing with table size); every routing keeps
    its windows within the bound and beats the plain Limits window."""
    torch = _torch()
    inst = L.square32()
    b = S.Basis.build(inst)
    plain = b.info()["limits_mean_window"]
    none = b.train_index(routing=2, log2_segments=12)
    untrained = b.train_index(routing=1, log2_segments=12)
    trained = b.train_index(steps=1500, log2_segments=12)
    for name, st in (("plain", plain), ("none", none), ("untrained", untrained), ("trained", trained)):
        _say(name, st)
    for st in (none, untrained, trained):
        assert st["max_err"] <= 64
        assert st["mean_window"] < 0.2 * plain
    assert trained["mlp_max_err"] < 0.1 * untrained["mlp_max_err"]
    assert trained["used_segments"] > 2 * untrained["used_segments"]
    assert trained["table_bytes"] < 0.5 * untrained["table_bytes"]
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


def _time_apply(torch, b, x, y, mode, reps=2):
    b.apply_H(x, y, mode=mode)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.apply_H(x, y, mode=mode)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    return min(ts)


def test_trained_network_gains_at_square40(S):
    """At the 40-site benchmark sector (430,909,650 states), H.v through the
    trained network runs at more elements per second than through the
    untrained network, with the tables below built the same way, and the
    index (network, segments, cells) is smaller than the plain lookup's
    Limits table."""
    torch = _torch()
    inst = L.square40()
    b = S.Basis.build(inst)
    info = b.info()
    n_el = info["n_elements"]
    g = torch.Generator(device="cuda")
    g.manual_seed(21)
    x = torch.randn(b.dim, dtype=torch.float64, device="cuda", generator=g)
    y0 = torch.zeros_like(x)
    y1 = torch.zeros_like(x)
    rate = {}
    for name, routing in (("none", 2), ("untrained", 1), ("trained", 0)):
        st = b.train_index(routing=routing)
        t = _time_apply(torch, b, x, y1, 1)
        rate[name] = n_el / t
        _say(" ", name, "H.v", round(t, 3), "s", f"{rate[name]:.3e} el/s", {k: st[k] for k in (
            "mean_window", "max_err", "mean_abs_err", "frac_exact", "mean_lines", "n_cells", "table_bytes",
            "used_segments", "refined_segments")})
    assert st["table_bytes"] + st["mlp_bytes"] < info["limits_bytes"]
    assert rate["trained"] > rate["untrained"]
    b.apply_H(x, y0, mode=0)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    del x, y0, y1
    b.free()


def test_learned_index_requires_training(S):
    torch = _torch()
    b = S.Basis.build(L.chain16())
    x = torch.zeros(b.dim, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(S.EdError):
        b.apply_H(x, y, mode=1)


def test_large_segment_table_stays_in_bounds(S):
    """2^24 segments: the network output near 1 must map to the last segment
    (the float value of 2^24 - 0.5 rounds up to 2^24, so the segment index is
    clamped as an integer)."""
    torch = _torch()
    inst = L.square32()
    b = S.Basis.build(inst)
    st = b.train_index(steps=300, log2_segments=24)
    assert st["n_segments"] == 1 << 24
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
    assert st["max_err"] <= 64                 # segments with wider windows are refined
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
