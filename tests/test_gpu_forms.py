"""GPU tests of the hysteresis, batched, checkpoint and serving forms, and of
the ABI's error handling, all through the C ABI."""
import math
import sys
import time

import numpy as np
import pytest

import oracle
from oracle.fem import ANIS, EXCH, MU0, ZEEM
from oracle.minimize import Options, bisect_switch
from paper_1309_5796_amd import meshgen

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1309_5796_amd import binding
    say("context create")
    c = binding.Context(0)
    yield c
    c.close()


def shared_launch_blocks(p, lanes=4, cap=512):
    """Blocks a problem gets inside a shared launch (batch or server): about
    four passes of a 512-thread block over its rows, a multiple of 8, capped
    by its own launch shape."""
    rows = max(p.N, p.Nt)
    g = -(-rows // (4 * (512 // lanes)))
    return max(8, min(-(-g // 8) * 8, cap))


def small_grain(edge_nm, seed, cells=None):
    rng = np.random.default_rng(seed)
    n = cells or meshgen.config4_cells(edge_nm * 1e-9)
    mesh = meshgen.kuhn_box((edge_nm * 0.5e-9,) * 3, (n, n, n), air=True)
    mesh.materials = [meshgen.Material(1, meshgen.JS_T, meshgen.K1_JM3, meshgen.A_JM, meshgen.cap_axis(rng))]
    nm = meshgen.n_magnetic(mesh)
    return mesh, meshgen.noisy_plus_z(nm, rng)


def test_hysteresis_sw_cube_switching_field_matches_oracle_bisection(ctx):
    """Demag-free SW cube: the library's bisected switching field equals the
    oracle's bisection and the astroid value."""
    from paper_1309_5796_amd import binding
    say("hysteresis SW cube with bisection")
    mesh = meshgen.kuhn_box((1e-9,) * 3, (2, 2, 2), air=False)
    s = oracle.System(mesh)
    u = meshgen.U_H_1DEG
    mu0HK = 2 * meshgen.K1_JM3 / (meshgen.JS_T / MU0)
    Bs = np.arange(-6.0, -7.41, -0.2)
    fields = Bs[:, None] * u[None, :]
    terms = EXCH | ANIS | ZEEM
    tol_T = 1e-4 * mu0HK
    p = binding.Problem(ctx, mesh)
    res, bsw = p.hysteresis(fields, terms=terms, tol=1e-9, refine_tol_T=tol_T)
    assert len(bsw) == 1
    psi = math.radians(1.0)
    exact = (math.cos(psi) ** (2 / 3) + math.sin(psi) ** (2 / 3)) ** (-1.5) * mu0HK
    # switching fields are projected on fields[0] / |fields[0]| = -u_H; near the
    # critical field the 0.1 rad first trial step crosses the vanishing barrier,
    # so the bisected value sits slightly below the astroid (the oracle agrees)
    assert abs(bsw[0] - exact) < 3e-3 * exact
    # oracle: same sweep, bisect in the bracket the library found
    recs, _ = oracle.hysteresis(s, np.tile([0.0, 0.0, 1.0], (s.N, 1)), fields, Options(terms=terms, tol=1e-9))
    k = [i for i in range(1, len(recs)) if np.sign(recs[i].m_avg @ u) != np.sign(recs[i - 1].m_avg @ u)][0]
    _, m_prev = oracle.hysteresis(s, np.tile([0.0, 0.0, 1.0], (s.N, 1)), fields[:k], Options(terms=terms, tol=1e-9))
    b_or = bisect_switch(s, m_prev, fields[k - 1], fields[k], u, tol_T, Options(terms=terms, tol=1e-9))
    assert abs(bsw[0] + b_or) < 2 * tol_T
    for r_gpu, r_or in zip(res, recs):
        assert abs(r_gpu.energy_J - r_or.E) < 1e-9 * abs(r_or.E)
    p.close()


def test_hysteresis_config1_short_sweep_matches_oracle(ctx, cfg1, cfg1_system):
    from paper_1309_5796_amd import binding
    say("hysteresis config1 short sweep")
    s = cfg1_system
    fields = np.array([-1.0, -2.0, -3.0])[:, None] * meshgen.U_H_1DEG[None, :]
    recs, _ = oracle.hysteresis(s, cfg1["m0"], fields, Options())
    p = binding.Problem(ctx, cfg1["mesh"])
    p.set_m(cfg1["m0"])
    res, _ = p.hysteresis(fields)
    for r_gpu, r_or in zip(res, recs):
        scale = abs(r_gpu.e_exch_J) + abs(r_gpu.e_anis_J) + abs(r_gpu.e_zeem_J) + abs(r_gpu.e_demag_J)
        assert r_gpu.status == 0
        assert abs(r_gpu.energy_J - r_or.E) < 1e-10 * scale
        np.testing.assert_allclose(r_gpu.m_avg, r_or.m_avg, atol=1e-7)
    p.close()


def test_batch_equals_one_by_one_bitwise(ctx):
    """A shared launch gives each problem min(its own block count, a count
    proportional to its rows); at a block count below the proportional one
    (16 here) both runs use the same decomposition and reduction order, so the
    results agree bit for bit."""
    from paper_1309_5796_amd import binding
    say("batch vs single")
    specs = [(10, 1), (14, 2), (12, 3), (16, 4)]
    single, probs = [], []
    for prec in (binding.FP64, binding.MIXED):
        for edge, seed in specs:
            mesh, m0 = small_grain(edge, seed)
            p = binding.Problem(ctx, mesh, precision=prec)
            p.set_launch(4, 16)
            p.set_m(m0)
            p.set_field(-1.0 * meshgen.U_H_1DEG)
            st = p.get_state()
            r = p.minimize()
            single.append((r.energy_J, r.evals, r.iterations, p.get_m().tobytes()))
            p.set_state(st)
            probs.append(p)
    say(f"batch of {len(probs)}")
    out = binding.minimize_batch(probs)
    for k, (p, r) in enumerate(zip(probs, out)):
        assert (r.energy_J, r.evals, r.iterations, p.get_m().tobytes()) == single[k], k
    # and every result is the oracle's minimum: FP64 to 1e-10, mixed to 1e-6
    # (relative to the sum of the term magnitudes)
    ref = {}
    for k, (p, r) in enumerate(zip(probs, out)):
        edge, seed = specs[k % len(specs)]
        if (edge, seed) not in ref:
            mesh, m0 = small_grain(edge, seed)
            ref[edge, seed] = oracle.minimize(oracle.System(mesh), m0, -1.0 * meshgen.U_H_1DEG, Options())
        ro = ref[edge, seed]
        tol = 1e-10 if p.precision == binding.FP64 else 1e-6
        assert ro.status == 0 and r.status in ((0,) if p.precision == binding.FP64 else (0, 2)), k
        assert abs(r.energy_J - ro.E) < tol * sum(abs(v) for v in ro.terms.values()), k
        np.testing.assert_allclose(p.get_m(), ro.m, atol=1e-5 if p.precision == binding.FP64 else 1e-3)
    for p in probs:
        p.close()


def test_checkpoint_resume_bitwise(ctx, cfg1):
    from paper_1309_5796_amd import binding
    say("checkpoint resume")
    fields = np.array([-1.0, -1.5, -2.0, -2.5])[:, None] * meshgen.U_H_1DEG[None, :]
    p = binding.Problem(ctx, cfg1["mesh"])
    p.set_m(cfg1["m0"])
    full, _ = p.hysteresis(fields)
    q = binding.Problem(ctx, cfg1["mesh"])
    q.set_m(cfg1["m0"])
    q.hysteresis(fields[:2])
    state = q.get_state()
    q.close()
    q2 = binding.Problem(ctx, cfg1["mesh"])
    q2.set_state(state)
    rest, _ = q2.hysteresis(fields[2:])
    for a, b in zip(full[2:], rest):
        assert a.energy_J == b.energy_J and a.evals == b.evals
    assert np.array_equal(p.get_m(), q2.get_m())
    p.close()
    q2.close()


def test_errors_are_reported_not_faulted(ctx, cfg1):
    from paper_1309_5796_amd import binding
    say("error paths")
    mesh = cfg1["mesh"]
    bad = meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets.copy(), region=mesh.region, dirichlet=mesh.dirichlet,
                       shell=mesh.shell, materials=mesh.materials)
    bad.tets[5, 2] = mesh.n_nodes + 7
    with pytest.raises(binding.MMSDError) as e:
        binding.Problem(ctx, bad)
    assert e.value.code == binding.E_MESH
    flat = meshgen.Mesh(xyz=mesh.xyz.copy(), tets=mesh.tets, region=mesh.region, dirichlet=mesh.dirichlet,
                        shell=mesh.shell, materials=mesh.materials)
    t = mesh.tets[np.nonzero(mesh.region)[0][0]]
    flat.xyz[t[3]] = flat.xyz[t[0]]
    with pytest.raises(binding.MMSDError) as e:
        binding.Problem(ctx, flat)
    assert e.value.code == binding.E_MESH
    p = binding.Problem(ctx, mesh)
    m = np.tile([0.0, 0.0, 1.0], (p.N, 1))
    m[3] = 0
    with pytest.raises(binding.MMSDError) as e:
        p.set_m(m)
    assert e.value.code == binding.E_INVALID
    r = p.minimize(max_evals=3)
    assert r.status == binding.W_MAXEVALS and r.evals == 3
    noair = meshgen.kuhn_box((1e-9,) * 3, (2, 2, 2), air=False)
    q = binding.Problem(ctx, noair)
    with pytest.raises(binding.MMSDError) as e:
        q.minimize()                       # stray field needs the outer boundary
    assert e.value.code == binding.E_INVALID
    p.close()
    q.close()


def test_server_results_equal_alone_and_in_the_mix(ctx):
    from paper_1309_5796_amd import binding
    say("server alone vs mix")
    reqs = [(10, 11, binding.FP64), (16, 12, binding.MIXED), (12, 13, binding.FP64),
            (20, 14, binding.FP64), (11, 15, binding.MIXED), (14, 16, binding.FP64)]
    alone = []
    for edge, seed, prec in reqs:
        mesh, m0 = small_grain(edge, seed)
        p = binding.Problem(ctx, mesh, precision=prec)
        p.set_launch(4, shared_launch_blocks(p))   # the shape the server gives the request
        p.set_m(m0)
        p.set_field(-1.5 * meshgen.U_H_1DEG)
        r = p.minimize()
        alone.append((r.energy_J, r.evals, p.get_m().tobytes()))
        p.close()
    srv = binding.Server(ctx, hbm_budget=2 << 30, max_slots=4)
    tickets = []
    for edge, seed, prec in reqs:
        mesh, m0 = small_grain(edge, seed)
        tickets.append((srv.submit(mesh, -1.5 * meshgen.U_H_1DEG, precision=prec, m0=m0),
                        meshgen.n_magnetic(mesh)))
    # a broken mesh in the queue: submit accepts it (sizing runs later, on a
    # setup worker), its poll reports the mesh error, and the others still finish
    bad, _ = small_grain(10, 17)
    bad.tets = bad.tets.copy()
    bad.tets[3, 2] = bad.xyz.shape[0] + 5
    bad_ticket = srv.submit(bad, -1.5 * meshgen.U_H_1DEG)
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < 120:
        for k, (t, n) in enumerate(tickets):
            if k in got:
                continue
            out = srv.poll(t, n)
            if out is not None:
                got[k] = out
        time.sleep(0.01)
    assert len(got) == len(tickets)
    for k in range(len(reqs)):
        r, m = got[k]
        assert (r.energy_J, r.evals, m.tobytes()) == alone[k], k
    # every served result is also the oracle's minimum (FP64 1e-10, mixed 1e-6)
    for k, (edge, seed, prec) in enumerate(reqs):
        r, m = got[k]
        mesh, m0 = small_grain(edge, seed)
        ro = oracle.minimize(oracle.System(mesh), m0, -1.5 * meshgen.U_H_1DEG, Options())
        tol = 1e-10 if prec == binding.FP64 else 1e-6
        assert ro.status == 0 and abs(r.energy_J - ro.E) < tol * sum(abs(v) for v in ro.terms.values()), k
        np.testing.assert_allclose(m, ro.m, atol=1e-5 if prec == binding.FP64 else 1e-3)
    t0 = time.time()
    with pytest.raises(binding.MMSDError, match="out of range") as e:
        while srv.poll(bad_ticket) is None and time.time() - t0 < 30:
            time.sleep(0.01)
    assert e.value.code == binding.E_MESH
    st = srv.stats()
    assert st["completed"] == len(reqs) + 1 and st["resident"] == 0
    srv.close()


def test_served_stream_under_load_finishes_every_request():
    """The first 48 requests of the seeded 200 req/s stream (grain boxes of
    1.2k-520k nodes, FP64/mixed), submitted at once to a 32-slot server with
    the device assembly: many problems share each launch while setup kernels
    run beside the step loop.  Every request must finish with a finite
    result.  Under this load a missing barrier in the V-cycle launches (a
    wavefront reading the cycle position after thread 0 had advanced it)
    once ended a few percent of requests non-finite."""
    from paper_1309_5796_amd import binding
    say("served stream under load: 48 requests, 32 slots, device assembly")
    reqs = meshgen.config5_requests(n_requests=48, rate_hz=200.0)
    built = [meshgen.request_mesh(r) for r in reqs]
    c = binding.Context(0)
    c.set_assembly(binding.ASSEMBLE_DEVICE)
    srv = binding.Server(c, hbm_budget=64 << 30, max_slots=32)
    tickets = {srv.submit(b["mesh"], b["b_ext"], precision=r.precision): k for k, (r, b) in enumerate(zip(reqs, built))}
    done, failed = {}, {}
    t0 = time.time()
    while len(done) + len(failed) < len(tickets) and time.time() - t0 < 240:
        for t, k in tickets.items():
            if k in done or k in failed:
                continue
            try:
                out = srv.poll(t)
            except binding.MMSDError as e:
                failed[k] = e.code
                continue
            if out is not None:
                done[k] = out[0]
        time.sleep(0.005)
    say(f"served {len(done)} failed {len(failed)} in {time.time() - t0:.1f} s")
    srv.close()
    c.close()
    assert not failed, failed
    assert len(done) == len(reqs)
    for k, r in done.items():
        assert r.status >= 0 and math.isfinite(r.energy_J) and math.isfinite(r.max_torque), (k, r.status)


def test_sphere_short_sweep_matches_oracle(ctx):
    """Coarse staircase ball (the paper's sphere experiment at 8 cells per
    diameter): field points 0, -1.5, -3 T at 45 degrees, warm-started, against
    the oracle's continuation."""
    from paper_1309_5796_amd import binding
    say("sphere short sweep")
    mesh = meshgen.kuhn_ball(cells=8)
    s = oracle.System(mesh)
    m0 = np.tile([0.0, 0.0, 1.0], (s.N, 1))
    fields = -np.array([0.0, 1.5, 3.0])[:, None] * meshgen.U_H_45DEG[None, :]
    recs, _ = oracle.hysteresis(s, m0, fields, Options())
    p = binding.Problem(ctx, mesh)
    p.set_m(m0)
    res, _ = p.hysteresis(fields)
    for r_gpu, r_or in zip(res, recs):
        scale = abs(r_gpu.e_exch_J) + abs(r_gpu.e_anis_J) + abs(r_gpu.e_zeem_J) + abs(r_gpu.e_demag_J)
        assert r_gpu.status == 0 and r_or.status == 0
        assert abs(r_gpu.energy_J - r_or.E) < 1e-10 * scale
        np.testing.assert_allclose(r_gpu.m_avg, r_or.m_avg, atol=1e-7)
    p.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_footprint_covers_the_device_memory_a_problem_holds(ctx, precision):
    """The admission estimate (first arena exact, multigrid hierarchy by an
    allowance) is at least what problem creation allocates through the
    context's allocator, on the 80 nm cube and on an irregular mesh."""
    from paper_1309_5796_amd import binding
    prec = binding.FP64 if precision == "fp64" else binding.MIXED
    for name, mesh in (("80 nm cube", meshgen.config2()["mesh"]), ("irregular", meshgen.delaunay_box(3))):
        say(f"footprint {name} {precision}")
        live = ctx._alloc.live
        before = sum(t.numel() for t in live.values())
        p = binding.Problem(ctx, mesh, precision=prec)
        used = sum(t.numel() for t in live.values()) - before
        est = binding.footprint(mesh, prec)
        say(f"  allocated {used / 1e6:.1f} MB, footprint {est / 1e6:.1f} MB")
        assert used > 0 and est >= used
        p.close()
