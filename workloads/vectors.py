"""Seeded synthetic vectors.

* ``start_vector``: N(0,1) entries from numpy's PCG64 stream in canonical
  (ascending-representative) order; complex vectors take the real parts from
  the first `dim` draws and the imaginary parts from the next `dim`.
* ``state_vector``: a vector whose entry for representative s is a function
  of s alone (SplitMix64 of seed xor s, mapped to [-1, 1)), so that a value
  can be produced for any configuration without knowing its position in the
  basis.  SplitMix64 as published by Steele, Lea and Flood (2014).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    x = np.asarray(x, np.uint64)
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _unit(z):
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def state_vector(states, seed, is_complex=False):
    s = np.asarray(states, np.uint64)
    re = _unit(splitmix64(s ^ np.uint64(seed)))
    if not is_complex:
        return re
    im = _unit(splitmix64(s ^ np.uint64(seed + 0x5DEECE66D)))
    return re + 1j * im


def start_vector(dim, seed, is_complex=False):
    g = np.random.Generator(np.random.PCG64(seed))
    if not is_complex:
        return g.standard_normal(dim)
    d = g.standard_normal(2 * dim)
    return d[:dim] + 1j * d[dim:]


def random_sector_states(n_sites, n_up, count, seed):
    """Uniformly random configurations with n_up up spins."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros(count, np.uint64)
    for k in range(count):
        sites = g.choice(n_sites, size=n_up, replace=False)
        v = 0
        for q in sites:
            v |= 1 << (n_sites - 1 - int(q))
        out[k] = v
    return out


def random_color_states(n_sites, counts, count, seed):
    """Uniformly random configurations of an SU(d) color-count sector, two
    bits per site (site 0 in the most significant digit): a random
    permutation of the multiset of colors."""
    g = np.random.Generator(np.random.PCG64(seed))
    base = np.repeat(np.arange(len(counts)), counts)
    w = np.uint64(4) ** np.arange(n_sites - 1, -1, -1, dtype=np.uint64)
    out = np.zeros(count, np.uint64)
    for k in range(count):
        out[k] = np.sum(g.permutation(base).astype(np.uint64) * w, dtype=np.uint64)
    return out
