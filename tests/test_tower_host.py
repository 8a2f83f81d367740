"""Host logic of the tower-of-states sweep: removal of spurious Lanczos Ritz
values (Cullum-Willoughby test) and the spin-S cut, on T-matrices from the
oracle's Lanczos (no reorthogonalization) over every sector of the 12-site
triangular cluster, against dense spectra."""
import numpy as np

from oracle import oracle as O
from workloads import lattices as L


def _distinct(w, k):
    return [e for i, e in enumerate(w) if i == 0 or e - w[i - 1] > 1e-8][:k]


def test_good_ritz_removes_spurious_values():
    from paper_2210_03511_amd import tower as T
    k, fixed = 4, 0
    for sz in (0, 1):
        for inst in L.triangular12_sectors(J2=0.0, n_up=6 + sz):
            reps, stabs = O.enumerate_basis(inst)
            if not len(reps):
                continue
            H = O.coo_matrix(inst, reps, stabs)
            exact = _distinct(np.linalg.eigvalsh(H.toarray()), k)
            for seed in range(3):
                rng = np.random.default_rng(seed)
                v0 = rng.standard_normal(len(reps))
                if inst.is_complex:
                    v0 = v0 + 1j * rng.standard_normal(len(reps))
                a, b = O.lanczos(lambda v: H @ v, v0, len(reps), hermitian_complex=inst.is_complex)
                bb = np.zeros(len(a))
                bb[:min(len(b), len(a))] = b[:len(a)]
                got = T.good_ritz(a, bb, k)
                assert len(got) == len(exact) and abs(got[0] - exact[0]) < 1e-10, inst.name
                assert np.allclose(got, exact, rtol=0, atol=1e-7), inst.name
                plain = _distinct(T.symed.eigenvalues(a, bb, len(a)), k)
                fixed += not np.allclose(plain, exact, rtol=0, atol=1e-7)
    assert fixed > 0        # the cases include T-matrices with a spurious value


def test_spin_levels_cut():
    from paper_2210_03511_amd import tower as T
    at_s = [("a", [-3.0, -1.0], 0.0, 10), ("b", [-2.5, -2.0], 0.0, 10)]
    at_s1 = [("a", [-1.5], 0.0, 8), ("b", [-0.5], 0.0, 8)]
    rows, cut = T.spin_levels(at_s, at_s1)
    assert cut == -1.5
    assert rows == [(-3.0, "a"), (-2.5, "b"), (-2.0, "b")]


def test_spin_levels_cut_lowered_by_drift():
    """A less converged copy of a higher-spin level at Sz = S + 1 (Ritz value
    above the level, drift 0.01) must not let that level pass as spin S."""
    from paper_2210_03511_amd import tower as T
    at_s = [("a", [-3.0, -2.0005], 0.0, 10)]           # -2.0005: a spin-(S+1) level, converged at Sz = S
    at_s1 = [("a", [-2.0], 0.01, 8)]                    # its copy at Sz = S + 1, not yet converged
    rows, cut = T.spin_levels(at_s, at_s1)
    assert cut == -2.01
    assert rows == [(-3.0, "a")]
    rows0, cut0 = T.spin_levels(at_s, at_s1, safety=0.0)
    assert rows0 == [(-3.0, "a"), (-2.0005, "a")]       # without the margin it would pass


def test_good_ritz_keeps_levels_with_small_start_weight():
    """A genuine level on which the start vector has little weight u lies
    about D u^2 from an eigenvalue of the reduced T-matrix (D ~ spectral
    width), as close as 1e-10 for u^2 ~ 1e-11 - the weight of a random start
    vector in a 10^8-state sector, now and then.  It must not be taken for a
    spurious value: a diagonal H with an isolated lowest level and a second
    level, each given such a weight."""
    from paper_2210_03511_amd import tower as T
    rng = np.random.default_rng(0)
    dim = 200_000
    ev = np.sort(rng.normal(0.0, 5.0, dim))
    ev[0] = ev[2] - 0.6
    ev[1] = ev[2] - 0.3
    v0 = np.random.default_rng(1).standard_normal(dim)
    v0[0] = 3e-6 * np.linalg.norm(v0)     # u^2 ~ 1e-11 on the lowest level
    v0[1] = 5e-6 * np.linalg.norm(v0)     # and on the second
    a, b = O.lanczos(lambda v: ev * v, v0, 100)
    lam = T.symed.eigenvalues(a, b, len(a))
    mu = T.symed.eigenvalues(a[1:], b[1:], len(a) - 1)
    scale = max(1.0, float(np.max(np.abs(lam))))
    # both levels converged and close to the reduced matrix's eigenvalues
    for e in ev[:2]:
        assert np.min(np.abs(lam - e)) < 1e-9
        assert np.min(np.abs(mu - e)) < 1e-10 * scale
    got = T.good_ritz(a, b, 3)
    assert abs(got[0] - ev[0]) < 1e-9 and abs(got[1] - ev[1]) < 1e-9
