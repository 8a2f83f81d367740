"""SU(d) device code compiled for the host (colors_dev.h, represent.h and the
library's table builder) against the oracle: the enumeration of a color-count
sector chunk by chunk with prefix pruning gives the oracle's representatives
and stabilizers for every admissible pair of decompositions; rank/unrank and
the next-configuration step agree with brute force over the sector; the
sublattice-coded representative search agrees with brute force over the
group; and the moves built from the model act on each representative as the
oracle's non-branching pieces do (same targets, same summed amplitudes, same
diagonal).  Needs hipcc (host compilation only), no GPU."""
import os
import shutil
import struct
import subprocess
from collections import defaultdict

import numpy as np
import pytest

from oracle import oracle as O
from workloads import lattices as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "colors_check.cpp")
LIBDIR = os.path.join(ROOT, "paper_2210_03511_amd")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    objdir = os.path.join(LIBDIR, "_build")
    if not os.path.exists(os.path.join(objdir, "tables.cpp.o")):
        from paper_2210_03511_amd.build import build
        build()
    objs = sorted(os.path.join(objdir, f) for f in os.listdir(objdir) if f.endswith(".o"))
    out = str(tmp_path_factory.mktemp("cc") / "colors_check")
    cmd = [hipcc, "-x", "hip", "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(LIBDIR, "csrc"), SRC, "-x", "none"] + objs + ["-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _write(inst, path):
    counts = list(inst.counts) + [0] * (4 - len(inst.counts))
    with open(path, "wb") as f:
        f.write(struct.pack("9i", inst.n_sites, inst.local_dim, inst.n_elem, len(inst.bond_J), len(inst.tri_Jchi),
                            *counts))
        for a, t in ((inst.perms, np.int32), (inst.flips, np.uint8), (inst.chi.real, np.float64),
                     (inst.chi.imag, np.float64), (inst.bonds, np.int32), (inst.bond_J, np.float64),
                     (inst.tris, np.int32), (inst.tri_Jchi, np.float64)):
            f.write(np.ascontiguousarray(a, t).tobytes())


def _read(path):
    with open(path, "rb") as f:
        dim = struct.unpack("Q", f.read(8))[0]
        reps = np.frombuffer(f.read(8 * dim), np.uint64)
        stabs = np.frombuffer(f.read(4 * dim), np.uint32)
        rows = []
        for _ in range(dim):
            diag = struct.unpack("d", f.read(8))[0]
            k = struct.unpack("Q", f.read(8))[0]
            tg = np.frombuffer(f.read(8 * k), np.uint64)
            hr = np.frombuffer(f.read(8 * k), np.float64)
            hi = np.frombuffer(f.read(8 * k), np.float64)
            rows.append((diag, tg, hr + 1j * hi))
    return reps, stabs, rows


def _tri9(d, counts, K3, q=L.Q0):
    return L.sun_triangular((3, 0), (0, 3), d, counts, J=1.0, K3=K3, q=q, sublat_chain=[((1, 1), (2, -1))])


CASES = [
    L.sun_chain(6, 3, (2, 2, 2), k=1),
    L.sun_chain(6, 3, (2, 2, 2), K3=0.6, k=2),
    L.sun_chain(6, 3, (3, 2, 1), K3=-0.3, k=0, reflection=False),
    L.sun_chain(8, 4, (2, 2, 2, 2), k=3),
    L.sun_chain(8, 2, (4, 4), K3=0.3, k=4),
    L.sun_chain(6, 3, (6, 0, 0), k=0),
    L.sun_chain(6, 3, (6, 0, 0), k=1),
    L.sun_chain(8, 4, (3, 1, 0, 4), J=0.7, k=0, reflection=True),
    _tri9(3, (3, 3, 3), 0.4),
    _tri9(3, (3, 3, 3), 0.0, q=(L.Fraction(1, 3), L.Fraction(1, 3))),
]


def _oracle_rows(inst, reps):
    rows = [defaultdict(complex) for _ in reps]
    diag = np.zeros(len(reps), complex)
    for tgt, h in O.sun_terms(inst, reps):
        for r, (t, a) in enumerate(zip(tgt, h)):
            if t == reps[r]:
                diag[r] += a
            else:
                rows[r][int(t)] += a
    return diag, rows


@pytest.mark.parametrize("inst", CASES, ids=lambda i: f"{i.name}-{i.sector}")
def test_color_enumeration_and_moves_match_oracle(checker, inst, tmp_path):
    path, out = str(tmp_path / "inst.bin"), str(tmp_path / "out.bin")
    _write(inst, path)
    reps_o, stabs_o = O.sun_enumerate_basis(inst)
    diag_o, rows_o = _oracle_rows(inst, np.asarray(reps_o, np.uint64))
    N = 2 * inst.n_sites
    divisors = [d for d in range(1, N + 1) if N % d == 0]
    ran = 0
    for R in [0] + divisors:
        for A in [0] + divisors:
            if R and A and A % R:
                continue
            for ln in (1, 7, 256):
                r = subprocess.run([checker, path, str(R), str(A), str(ln), out], capture_output=True, text=True,
                                   timeout=120)
                if "build_color_tables failed" in r.stdout:
                    break
                assert r.returncode == 0, (R, A, ln, r.stdout[-500:])
                reps, stabs, rows = _read(out)
                assert np.array_equal(reps, np.asarray(reps_o, np.uint64)), (R, A, ln)
                assert np.array_equal(stabs, np.asarray(stabs_o)), (R, A, ln)
                ran += 1
    assert ran >= 1
    for k, (diag, tg, h) in enumerate(rows):
        got = defaultdict(complex)
        for t, a in zip(tg, h):
            got[int(t)] += a
        want = {t: a for t, a in rows_o[k].items() if abs(a) > 1e-15}
        got = {t: a for t, a in got.items() if abs(a) > 1e-15}
        assert got.keys() == want.keys()
        assert all(abs(got[t] - want[t]) < 1e-13 for t in want)
        assert abs(diag - diag_o[k]) < 1e-13


def test_color_build_rejects_bad_input(checker, tmp_path):
    path = str(tmp_path / "inst.bin")
    bad = []
    for field, val in (("counts", (2, 2, 1)), ("counts", (3, 4, -1)), ("flips", np.ones(6, np.uint8))):
        inst = L.sun_chain(6, 3, (2, 2, 2), k=0)
        setattr(inst, field, val)   # past the instance's own checks
        bad.append(inst)
    for inst in bad:
        _write(inst, path)
        r = subprocess.run([checker, path, "0", "0", "7", str(tmp_path / "o.bin")], capture_output=True, text=True,
                           timeout=60)
        assert "build_color_tables failed 1" in r.stdout, r.stdout
