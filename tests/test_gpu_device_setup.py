"""Problems whose operators are assembled on the device (mmsd_set_assembly
with MMSD_ASSEMBLE_DEVICE: device kernels, sliced potential matrix, row
sums and Jacobi factors formed on the device) against problems built from
the host assembly, through the C ABI: sizes, energies, fields, potentials,
a material change and a whole minimization, in FP64 and the mixed form;
and a server whose requests are set up that way."""
import sys
import time

import numpy as np
import pytest

from paper_1309_5796_amd import meshgen

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctxs():
    from paper_1309_5796_amd import binding
    say("contexts: host and device assembly")
    h = binding.Context(0)
    d = binding.Context(0)
    d.set_assembly(binding.ASSEMBLE_DEVICE)
    yield h, d
    d.close()
    h.close()


def two_regions():
    mesh = meshgen.config1()["mesh"]
    region = mesh.region.copy()
    mag = np.nonzero(region)[0]
    region[mag[::3]] = 2
    return meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets, region=region, dirichlet=mesh.dirichlet, shell=mesh.shell,
                        materials=mesh.materials + [
                            meshgen.Material(2, meshgen.JS_T, 1.3e6, 3e-12, np.array([0.3, -0.2, 0.9]))])


def grains():
    mesh = meshgen.kuhn_box((8e-9, 8e-9, 4e-9), (10, 10, 5), air=True)
    meshgen.assign_grains(mesh, 6, np.random.default_rng(11))
    return mesh


CASES = {
    "kuhn_two_regions": two_regions,
    "delaunay": lambda: meshgen.delaunay_box(5),
    "grains": grains,
    "no_air": lambda: meshgen.config1(air=False)["mesh"],
}
TERMS = ("energy_J", "e_exch_J", "e_anis_J", "e_zeem_J", "e_demag_J")


def energy_scale(r):
    return abs(r.e_exch_J) + abs(r.e_anis_J) + abs(r.e_zeem_J) + abs(r.e_demag_J)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_device_assembled_problem_matches_host_assembled(ctxs, name, prec):
    from paper_1309_5796_amd import binding
    h, d = ctxs
    precision = binding.FP64 if prec == "fp64" else binding.MIXED
    mesh = CASES[name]()
    say(f"problems {name} {prec}: {mesh.tets.shape[0]} tets")
    ph = binding.Problem(h, mesh, precision=precision)
    pd = binding.Problem(d, mesh, precision=precision)
    try:
        assert ph.sizes() == pd.sizes()
        t = pd.setup_times()
        assert all(v >= 0 for v in t.values()) and t["total"] >= t["assembly"], t
        rng = np.random.default_rng(7)
        m = rng.normal(size=(ph.N, 3))
        for p in (ph, pd):
            p.set_m(m)
            p.set_field([0.05, -0.1, 0.3])
        # FP64: the operators differ by fused multiply-add roundings only;
        # mixed: the same FP64 values rounded to FP32
        tol = 1e-12 if prec == "fp64" else 1e-6
        ftol = 1e-11 if prec == "fp64" else 1e-5
        # no potential problem without air: the stray field is left out
        terms = binding.ALL if ph.Nt else binding.EXCH | binding.ANIS | binding.ZEEM
        for stage in ("start", "material change"):
            rh, rd = ph.evaluate(terms=terms), pd.evaluate(terms=terms)
            s = energy_scale(rh)
            for k in TERMS:
                assert abs(getattr(rd, k) - getattr(rh, k)) <= tol * s, (stage, k, getattr(rd, k), getattr(rh, k))
            fh, fd = ph.get_field(), pd.get_field()
            assert np.abs(fd - fh).max() <= ftol * np.abs(fh).max(), stage
            if ph.Nt:
                uh, ud = ph.get_potential(), pd.get_potential()
                assert np.abs(ud - uh).max() <= ftol * np.abs(uh).max(), stage
            if stage == "start":
                mat = mesh.materials[0]
                new = meshgen.Material(mat.region, mat.Js, 0.7 * mat.K1, 1.4 * mat.A, np.array([0.4, 0.1, 0.9]))
                say(f"material change {name} {prec}")
                ph.set_material(new)
                pd.set_material(new)
        say(f"minimize {name} {prec}")
        m0 = meshgen.noisy_plus_z(ph.N, np.random.default_rng(5))
        for p in (ph, pd):
            p.set_m(m0)
            p.set_field(-0.8 * meshgen.U_H_1DEG)
        rh, rd = ph.minimize(terms=terms), pd.minimize(terms=terms)
        # the mixed form may stop at its precision floor (W_FLOOR)
        done = (binding.OK,) if prec == "fp64" else (binding.OK, binding.W_FLOOR)
        assert rh.status in done and rd.status in done, (rh.status, rd.status)
        s = energy_scale(rh)
        if prec == "fp64":
            assert abs(rd.energy_J - rh.energy_J) <= 1e-10 * s
            assert np.abs(rd.m_avg - rh.m_avg).max() <= 1e-6
        else:
            assert abs(rd.energy_J - rh.energy_J) <= 1e-6 * s
            assert np.abs(rd.m_avg - rh.m_avg).max() <= 1e-3
    finally:
        ph.close()
        pd.close()


def test_device_assembly_errors_reach_problem_creation(ctxs):
    from paper_1309_5796_amd import binding
    _, d = ctxs
    mesh = meshgen.config1()["mesh"]
    bad = meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets.copy(), region=mesh.region, dirichlet=mesh.dirichlet,
                       shell=mesh.shell, materials=mesh.materials)
    bad.tets[5, 3] = bad.tets[5, 2]
    say("device-assembled problem: degenerate tet")
    with pytest.raises(binding.MMSDError, match="degenerate tetrahedron 5") as e:
        binding.Problem(d, bad)
    assert e.value.code == binding.E_MESH
    with pytest.raises(binding.MMSDError, match="no material for region 1"):
        binding.Problem(d, mesh, materials=[])
    # the context still works after the failures
    p = binding.Problem(d, mesh)
    assert p.evaluate().status == binding.OK
    p.close()


def test_server_with_device_assembly_matches_direct_minimization(ctxs):
    from paper_1309_5796_amd import binding
    h, d = ctxs
    mesh = grains()
    n = meshgen.n_magnetic(mesh)
    m0 = meshgen.noisy_plus_z(n, np.random.default_rng(9))
    b = -0.9 * meshgen.U_H_1DEG
    say("direct minimization (host assembly)")
    p = binding.Problem(h, mesh)
    p.set_m(m0)
    p.set_field(b)
    ref = p.minimize()
    p.close()
    say("server on the device-assembly context")
    srv = binding.Server(d, hbm_budget=1 << 30, max_slots=2)
    try:
        t = srv.submit(mesh, b, m0=m0)
        out = None
        t0 = time.time()
        while out is None and time.time() - t0 < 60:
            out = srv.poll(t, n)
            time.sleep(0.01)
        assert out is not None
        r, m = out
        assert r.status == binding.OK
        assert abs(r.energy_J - ref.energy_J) <= 1e-10 * energy_scale(ref)
        assert np.abs(r.m_avg - ref.m_avg).max() <= 1e-6
    finally:
        srv.close()
