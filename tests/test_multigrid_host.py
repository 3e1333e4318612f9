"""Host-side multigrid identities behind the device's rearranged V-cycle
(prolongation inside post-smoothing, restriction inside the down-sweep,
Galerkin coarse operators), checked on the hierarchy of config 1's
potential matrix with the library's own host setup code (CPU only)."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_1309_5796_amd import binding, meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1309_5796_amd", "csrc")


def test_vcycle_rearrangements_are_identities(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "mg_identities")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "native", "mg_identities.cpp"),
                    os.path.join(CSRC, "amg.cpp"), "-o", exe, "-lpthread"], check=True)
    a = binding.assembly_export(meshgen.config1()["mesh"])
    path = str(tmp_path / "L.bin")
    with open(path, "wb") as f:
        np.array([a["Nt"], len(a["lci"])], np.int32).tofile(f)
        a["lrp"].astype(np.int32).tofile(f)
        a["lci"].astype(np.int32).tofile(f)
        a["L"].astype(np.float64).tofile(f)
    out = subprocess.run([exe, path], check=True, capture_output=True, text=True).stdout
    rows = re.findall(r"level (\d+) rows (\d+) rest (\S+) post (\S+) rap (\S+)", out)
    assert len(rows) >= 2, out   # at least two levels: a coarse level to restrict to and solve
    for lev, n, e_rest, e_post, e_rap in rows:
        assert float(e_rest) < 1e-12, out
        assert float(e_post) < 1e-12, out
        assert float(e_rap) < 1e-12, out
