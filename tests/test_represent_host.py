"""The sublattice-coded representative search of the H.v kernel (the
host-compiled copy of represent.h) against brute force over the group, for
every configuration of small instances and every admissible pair of
decompositions.  Needs hipcc (host compilation only), no GPU."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from workloads import lattices as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "represent_check.cpp")
LIBDIR = os.path.join(ROOT, "paper_2210_03511_amd")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    objdir = os.path.join(LIBDIR, "_build")
    # the library exports only its C ABI: link the table code from its objects
    if not os.path.exists(os.path.join(objdir, "tables.cpp.o")):
        from paper_2210_03511_amd.build import build
        build()
    objs = sorted(os.path.join(objdir, f) for f in os.listdir(objdir) if f.endswith(".o"))
    out = str(tmp_path_factory.mktemp("rc") / "represent_check")
    cmd = [hipcc, "-x", "hip", "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(LIBDIR, "csrc"), SRC, "-x", "none"] + objs + ["-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _write(inst, path):
    with open(path, "wb") as f:
        f.write(struct.pack("5i", inst.n_sites, inst.n_up, inst.n_elem, len(inst.bond_J), len(inst.tri_Jchi)))
        for a, t in ((inst.perms, np.int32), (inst.flips, np.uint8), (inst.chi.real, np.float64),
                     (inst.chi.imag, np.float64), (inst.bonds, np.int32), (inst.bond_J, np.float64),
                     (inst.tris, np.int32), (inst.tri_Jchi, np.float64)):
            f.write(np.ascontiguousarray(a, t).tobytes())


CASES = L.small_instances() + [L.chain16(), L.chain(6, sublat=(2,)), L.chain(6, sublat=(3,))] + L.kagome_instances()


@pytest.mark.parametrize("inst", CASES, ids=lambda i: f"{i.name}-{i.sector}")
def test_representative_search_matches_brute_force(checker, inst, tmp_path):
    path = str(tmp_path / "inst.bin")
    _write(inst, path)
    N = inst.n_sites
    divisors = [d for d in range(1, N + 1) if N % d == 0]
    ran = 0
    for R in [0] + divisors:
        for A in [0] + divisors:
            if R and A and A % R:
                continue
            r = subprocess.run([checker, path, str(R), str(A)], capture_output=True, text=True, timeout=120)
            if "build_host_tables failed" in r.stdout:
                continue
            assert r.returncode == 0, (R, A, r.stdout[-500:])
            ran += 1
    assert ran >= 1


def _large_cases():
    t36, c36 = L.TRI36_L, L.TRI36_CHAIN
    K = (L.F(1, 3), L.F(2, 3))
    return [
        ("triangular36 C6v Gamma.A1", L.triangular_j1j2chi(t36[0], t36[1], 1.0, 0.0, 0.0, L.Q0, irrep="A1", flip=1,
                                                           sublat_chain=c36)),
        ("triangular36 C6v K Sz=1", L.triangular_j1j2chi(t36[0], t36[1], 1.0, 0.0, 0.0, K, irrep="A1", flip=None,
                                                         sublat_chain=c36, n_up=19)),
        ("triangular36 {E, C2, mirrors}", L.triangular_j1j2chi(t36[0], t36[1], 1.0, 0.2, 0.0, L.Q0, irrep="A", flip=1,
                                                               sublat_chain=c36, pg_gens=[L.TRI_C2, L.TRI_MY])),
        ("triangular36 chiral C6", L.triangular_j1j2chi(t36[0], t36[1], 1.0, 0.1, 0.2, L.Q0, irrep="A", flip=1,
                                                        sublat_chain=c36)),
        ("triangular36 E2 sector", L.two_dim_sectors("triangular", t36, c36, J2=0.0, n_up=18)[2]),
        ("square32 E sector", L.two_dim_sectors("square", L.SQ32_L, L.SQ32_CHAIN, J2=0.5, n_up=16)[0]),
        ("square40", L.square40()),
        ("kagome27 C6v Sz=1/2", L.kagome27(J2=0.2, J3=0.1)),
        ("kagome27 chiral C6", L.kagome27(Jchi=0.3)),
    ]


@pytest.mark.parametrize("name,inst", _large_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_representative_search_sampled_large_groups(checker, name, inst, tmp_path):
    """The groups of the production-size sweeps and order parameters (36-site
    C6v, its subgroup that keeps a1's direction, the chiral C6, the sectors
    of 2-D irreps, the 40-site benchmark group), with the tables the library
    chooses by itself: 20000 random configurations each against brute force."""
    path = str(tmp_path / "inst.bin")
    _write(inst, path)
    r = subprocess.run([checker, path, "0", "0", "20000", "7"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (name, r.stdout[-500:])
    assert "checked 20000 bad 0" in r.stdout, r.stdout


def test_representative_search_sampled_all_decompositions_triangular36(checker, tmp_path):
    """Every admissible explicit pair (R, A) of the 36-site C6v group at Gamma
    (R sublattices for Rep/Sym, A for the action tables), 3000 random
    configurations each."""
    inst = L.triangular_j1j2chi(L.TRI36_L[0], L.TRI36_L[1], 1.0, 0.0, 0.0, L.Q0, irrep="A1", flip=1,
                                sublat_chain=L.TRI36_CHAIN)
    path = str(tmp_path / "inst.bin")
    _write(inst, path)
    ran = []
    for R in (1, 4, 12, 36):
        for A in (1, 4, 12, 36):
            if A % R:
                continue
            r = subprocess.run([checker, path, str(R), str(A), "3000", "11"], capture_output=True, text=True,
                               timeout=300)
            if "build_host_tables failed" in r.stdout:
                continue
            assert r.returncode == 0 and "bad 0" in r.stdout, (R, A, r.stdout[-300:])
            ran.append((R, A))
    assert ran == [(4, 4), (4, 12), (12, 12)], ran      # 1: tables too large; 36: not in the chain
