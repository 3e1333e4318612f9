"""Host-side multigrid identities behind the device's rearranged V-cycle
(prolongation inside post-smoothing, restriction inside the down-sweep,
Galerkin coarse operators), the smoother's convergence on every level, and
the plain V(1,1) cycle being symmetric positive definite, checked on the
hierarchies of config 1's and of the 80 nm cube's potential matrices with
the library's own host setup code (CPU only)."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_1309_5796_amd import binding, meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1309_5796_amd", "csrc")


# config 1 (two levels) and the 80 nm cube (three levels; the smoother's
# Gershgorin cap binds on its coarsest)
MESHES = {"config1": lambda: meshgen.config1()["mesh"], "cube80": lambda: meshgen.config2()["mesh"]}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_vcycle_rearrangements_are_identities(tmp_path, name):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "mg_identities")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "native", "mg_identities.cpp"),
                    os.path.join(CSRC, "amg.cpp"), "-o", exe, "-lpthread"], check=True)
    a = binding.assembly_export(MESHES[name]())
    path = str(tmp_path / "L.bin")
    with open(path, "wb") as f:
        np.array([a["Nt"], len(a["lci"])], np.int32).tofile(f)
        a["lrp"].astype(np.int32).tofile(f)
        a["lci"].astype(np.int32).tofile(f)
        a["L"].astype(np.float64).tofile(f)
    out = subprocess.run([exe, path], check=True, capture_output=True, text=True).stdout
    rows = re.findall(r"level (\d+) rows (\d+) rest (\S+) post (\S+) rap (\S+) wg (\S+) wlam (\S+)", out)
    assert len(rows) >= 2, out   # at least two levels: a coarse level to restrict to and solve
    for lev, n, e_rest, e_post, e_rap, wg, wlam in rows:
        assert float(e_rest) < 1e-12, out
        assert float(e_post) < 1e-12, out
        assert float(e_rap) < 1e-12, out
        # Damped Jacobi with weight w on SPD A converges iff w lambda_max(D^-1 A) < 2.
        # w g <= 1.9 bounds it from above (lambda_max <= g, both Gershgorin forms);
        # the power-iteration estimate, a lower bound on w lambda_max, shows the
        # weight is not so small that the smoother stops damping high modes.
        assert float(wg) <= 1.9 + 1e-12, out
        assert 1.0 < float(wlam) < 2.0, out
    # The plain V(1,1) cycle is what the CG preconditions with: symmetric and
    # positive definite (W (2 W^-1 - A) W > 0 needs w lambda_max < 2; the
    # coarse correction needs R = P^T and a symmetric dense inverse that does
    # invert the coarsest Galerkin operator).
    cyc = re.findall(r"cycle coarse (\S+) sym (\S+) pd (\S+)", out)
    assert len(cyc) == 1, out
    e_coarse, asym, pd = map(float, cyc[0])
    assert e_coarse < 1e-12, out
    assert asym < 1e-12, out
    assert pd > 0, out


def write_mesh(path, mesh):
    with open(path, "wb") as f:
        d = getattr(mesh, "dirichlet", None)
        sh = getattr(mesh, "shell", None)
        np.array([mesh.xyz.shape[0], mesh.tets.shape[0], len(mesh.materials), d is not None, sh is not None],
                 np.int64).tofile(f)
        np.ascontiguousarray(mesh.xyz, np.float64).tofile(f)
        np.ascontiguousarray(mesh.tets, np.int32).tofile(f)
        np.ascontiguousarray(mesh.region, np.int32).tofile(f)
        (np.zeros(mesh.xyz.shape[0], np.uint8) if d is None else np.ascontiguousarray(d, np.uint8)).tofile(f)
        (np.zeros(9) if sh is None else np.ascontiguousarray(sh, np.float64)).tofile(f)
        for m in mesh.materials:
            np.array([m.region, m.Js, m.K1, m.A, *np.asarray(m.axis, float)], np.float64).tofile(f)


@pytest.mark.parametrize("name", ["two_regions", "delaunay", "no_air"])
def test_device_assembly_structure_matches_host_assembly(tmp_path, name):
    """The host half of the device-side assembly: the structure equals the
    full host assembly's, and the device kernels' per-row sums, replayed
    here on the CPU from it, give the host values (same terms, same order)."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    if name == "two_regions":
        mesh = meshgen.config1()["mesh"]
        region = mesh.region.copy()
        region[np.nonzero(region)[0][::3]] = 2
        mesh = meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets, region=region, dirichlet=mesh.dirichlet,
                            shell=mesh.shell, materials=mesh.materials + [
                                meshgen.Material(2, meshgen.JS_T, 1.3e6, 3e-12, np.array([0.3, -0.2, 0.9]))])
    elif name == "delaunay":
        mesh = meshgen.delaunay_box(5)
    else:
        mesh = meshgen.config1(air=False)["mesh"]
    exe = str(tmp_path / "structure_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "native", "structure_check.cpp"), os.path.join(CSRC, "assemble.cpp"),
                    os.path.join(CSRC, "amg.cpp"), "-o", exe, "-lpthread"], check=True)
    path = str(tmp_path / "mesh.bin")
    write_mesh(path, mesh)
    out = subprocess.run([exe, path], check=True, capture_output=True, text=True).stdout
    assert "structure equal" in out, out
    rel = dict(zip(["V", "K", "D1", "D2", "Q"], map(float, re.findall(
        r"rel V (\S+) K (\S+) D1 (\S+) D2 (\S+) Q (\S+)", out)[0])))
    for k, v in rel.items():
        assert v <= 1e-15, (k, out)
    if "potential columns missing" in out:
        assert "potential columns missing 0" in out, out
    else:
        assert name == "no_air", out
