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


CASES = L.small_instances() + [L.chain16(), L.chain(6, sublat=(2,)), L.chain(6, sublat=(3,))]


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
