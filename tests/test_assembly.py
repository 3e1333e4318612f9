"""The library's host assembly (C++) against the oracle's matrices (NumPy),
compared as data on the CPU: no device is used.  The library works in nm
and mu0 Ms^2 nm^3 units; the oracle in SI."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle.fem import MU0
from paper_1309_5796_amd import binding, meshgen

NM = 1e-9


@pytest.fixture(scope="module", params=["kuhn_two_regions", "delaunay"])
def both(request):
    if request.param == "delaunay":
        # irregular connectivity: potential rows of 4 to ~25 entries
        mesh = meshgen.delaunay_box(5)
    else:
        cfg = meshgen.config1()
        mesh = cfg["mesh"]
        # a second material region so per-region values are exercised
        region = mesh.region.copy()
        mag = np.nonzero(region)[0]
        region[mag[::3]] = 2
        mesh = meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets, region=region, dirichlet=mesh.dirichlet,
                            shell=mesh.shell, materials=mesh.materials + [
                                meshgen.Material(2, meshgen.JS_T, 1.3e6, 3e-12, np.array([0.3, -0.2, 0.9]))])
    return mesh, oracle.System(mesh), binding.assembly_export(mesh)


def csr(a, vals, n):
    return sp.csr_matrix((vals, a["mci"], a["mrp"]), shape=(n, n))


def test_sizes_and_volumes(both):
    mesh, s, a = both
    assert a["N"] == s.N and a["Nt"] == s.Nt
    np.testing.assert_allclose(a["V"] * NM ** 3, s.V, rtol=1e-13)
    assert abs(a["scalars"][1] * NM ** 3 - s.V.sum()) < 1e-13 * s.V.sum()
    assert abs(a["scalars"][0] * s.mu0Ms2 * NM ** 3 - s.anis_const) < 1e-13 * s.anis_const


def test_exchange_matrix(both):
    _, s, a = both
    Khat = csr(a, a["K"], s.N).toarray()
    ref = (2.0 / (s.mu0Ms2 * s.V[:, None])) * s.K.toarray()
    assert np.abs(Khat - ref).max() < 1e-12 * np.abs(ref).max()


def test_anisotropy_tensors(both):
    _, s, a = both
    c = 2.0 / (s.mu0Ms2 * s.V)
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for k, (i, j) in enumerate(idx):
        ref = c * s.Q[:, i, j]
        assert np.abs(a["Q"][k] - ref).max() <= 1e-12 * np.abs(c[:, None, None] * s.Q).max()


def test_potential_coupling_both_directions(both):
    _, s, a = both
    rng = np.random.default_rng(0)
    m = rng.normal(size=(s.N, 3))
    b_lib = sum(csr(a, a["D1"][c], s.N) @ m[:, c] for c in range(3)) * s.Ms * NM ** 2
    # oracle right-hand side on the free nodes; magnetic nodes come first in the library
    b_or = s.rhs(m)
    pos = s.fmap[a["pot_global"][: s.N]]
    np.testing.assert_allclose(b_lib, b_or[pos], rtol=0, atol=1e-12 * np.abs(b_or).max())
    assert np.abs(np.delete(b_or, pos)).max() == 0.0
    u = rng.normal(size=s.Nt)
    h_or = s.demag_field(u)
    u_lib = u[s.fmap[a["pot_global"]]] / (s.Ms * NM)
    h_lib = -np.stack([csr(a, a["D2"][c], s.N) @ u_lib[: s.N] for c in range(3)], axis=1)
    np.testing.assert_allclose(h_lib, h_or, rtol=0, atol=1e-12 * np.abs(h_or).max())


def test_transformed_laplacian(both):
    _, s, a = both
    Llib = sp.csr_matrix((a["L"], a["lci"], a["lrp"]), shape=(s.Nt, s.Nt)) * NM
    perm = s.fmap[a["pot_global"]]
    Lor = s.L.tocsr()[perm][:, perm]
    d = (Llib - Lor).tocoo()
    assert np.abs(d.data).max() < 1e-12 * np.abs(Lor.data).max()
    assert (Llib != 0).nnz <= Lor.nnz + s.Nt


def test_bad_meshes_are_rejected_on_the_host():
    cfg = meshgen.config1()
    mesh = cfg["mesh"]
    bad = meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets.copy(), region=mesh.region, dirichlet=mesh.dirichlet,
                       shell=mesh.shell, materials=mesh.materials)
    bad.tets[0, 0] = -1
    with pytest.raises(binding.MMSDError) as e:
        binding.assembly_export(bad)
    assert e.value.code == binding.E_MESH
    nomat = meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets, region=mesh.region * 7, dirichlet=mesh.dirichlet,
                         shell=mesh.shell, materials=mesh.materials)
    with pytest.raises(binding.MMSDError) as e:
        binding.assembly_export(nomat)
    assert e.value.code == binding.E_INVALID
    touching = meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets, region=np.ones_like(mesh.region),
                            dirichlet=mesh.dirichlet, shell=mesh.shell, materials=mesh.materials)
    with pytest.raises(binding.MMSDError) as e:
        binding.assembly_export(touching)
    assert e.value.code == binding.E_MESH


def test_sphere_experiment_mesh():
    """Staircase ball standing in for the paper's 20 nm sphere (80,000 tets,
    edge 0.76 nm): magnetic volume within 0.5% of the sphere's, about as many
    magnetic tets, and every magnetic tet inside the sphere's bounding box."""
    mesh = meshgen.kuhn_ball()
    mag = mesh.region > 0
    d = mesh.xyz[mesh.tets[mag][:, 1:]] - mesh.xyz[mesh.tets[mag][:, :1]]
    vol = np.abs(np.linalg.det(d)).sum() / 6.0
    r = 10e-9
    assert abs(vol - 4.0 / 3.0 * np.pi * r ** 3) < 5e-3 * 4.0 / 3.0 * np.pi * r ** 3
    assert 75_000 < int(mag.sum()) < 95_000
    assert np.abs(mesh.xyz[np.unique(mesh.tets[mag])]).max() <= r * (1 + 1e-12)
