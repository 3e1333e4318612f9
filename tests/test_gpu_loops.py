"""Hysteresis loops through the C ABI against the FP64 oracle's loop
(Introduction: hysteresis as the path of successive local minima; Results,
comparison with the LLG solver: the switching field of a demagnetization
curve).

The workload is the 80 nm cube's sweep at the same cell size (2 nm) on a
16 nm cube (8^3 Kuhn cells, graded air and transformation shell): +8 -> -8
-> +8 T along z tilted by 1 degree, in 0.5 T steps, each point warm-started
from the previous minimum.  Parity bars: the FP64 path matches the oracle at
every point to 1e-10 relative energy (the sum of the term magnitudes as
denominator), switches at the same step on both branches and takes the same
number of energy-gradient evaluations; the mixed path matches to 1e-6
relative energy and its bisected switching fields lie within 1e-3 of the
oracle's bisection.  The loop also runs with every multigrid matrix in the
sliced layout and with the restriction in launches of its own, the code
paths that by default only meshes of about a million nodes take.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle.fem import MU0
from oracle.minimize import Options, bisect_switch
from paper_1309_5796_amd import meshgen

pytestmark = pytest.mark.gpu

U = meshgen.U_H_1DEG
MU0HK = 2 * meshgen.K1_JM3 / (meshgen.JS_T / MU0)
BISECT_T = 1e-4 * MU0HK


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _mesh():
    return meshgen.kuhn_box((8e-9,) * 3, (8, 8, 8), air=True)


def _switch_steps(m_avgs):
    s = np.sign([float(np.dot(m, U)) for m in m_avgs])
    return [k for k in range(1, len(s)) if s[k] != s[k - 1]]


@pytest.fixture(scope="module")
def loop_oracle():
    """The oracle's loop, with the minimum at every point kept (the bisection
    restarts from the last unswitched one)."""
    mesh = _mesh()
    s = oracle.System(mesh)
    fields = meshgen.sweep_fields(8.0, 0.5)
    say(f"oracle loop: {s.N} magnet / {s.Nt} potential nodes, {len(fields)} field points")
    m = np.tile([0.0, 0.0, 1.0], (s.N, 1))
    recs, ms = [], []
    for B in fields:
        r = oracle.minimize(s, m, B, Options())
        m = r.m
        recs.append(r)
        ms.append(m)
    sw = _switch_steps([s.mean_m(x) for x in ms])
    say(f"oracle switching steps {sw}, evals {sum(r.evals for r in recs)}")
    return dict(mesh=mesh, system=s, fields=fields, recs=recs, ms=ms, sw=sw)


def _gpu_loop(ctx, mesh, fields, precision, **opts):
    from paper_1309_5796_amd import binding
    p = binding.Problem(ctx, mesh, precision=precision)
    res, bsw = p.hysteresis(fields, **opts)
    p.close()
    return res, bsw


def _scale(r):
    return abs(r.e_exch_J) + abs(r.e_anis_J) + abs(r.e_zeem_J) + abs(r.e_demag_J)


@pytest.mark.parametrize("vcycle", ["default", "slice-all+separate-rest", "slice-all+fused"])
def test_fp64_loop_matches_oracle_point_by_point(loop_oracle, vcycle):
    from paper_1309_5796_amd import binding
    flags = {"default": None, "slice-all+separate-rest": binding.VC_SLICE_ALL,
             "slice-all+fused": binding.VC_SLICE_ALL | binding.VC_FUSE_REST | binding.VC_FOLD_SOLVE}[vcycle]
    say(f"fp64 loop, V-cycle {vcycle}")
    c = binding.Context(0)
    try:
        if flags is not None:
            c.set_vcycle(flags)
        res, _ = _gpu_loop(c, loop_oracle["mesh"], loop_oracle["fields"], binding.FP64)
    finally:
        c.close()
    recs = loop_oracle["recs"]
    assert _switch_steps([r.m_avg for r in res]) == loop_oracle["sw"] and len(loop_oracle["sw"]) == 2
    s = loop_oracle["system"]
    for k, (r, ro) in enumerate(zip(res, recs)):
        assert r.status == 0 and ro.status == 0, k
        assert abs(r.energy_J - ro.E) < 1e-10 * _scale(r), k
        np.testing.assert_allclose(r.m_avg, s.mean_m(ro.m), atol=1e-7)
        assert r.evals == ro.evals, (k, r.evals, ro.evals)
    say(f"  evals {sum(r.evals for r in res)}, pcg {sum(r.pcg_iters for r in res)}")


def test_mixed_loop_bisected_switching_fields_match_oracle(loop_oracle):
    """Mixed precision (FP32 storage and SpMV, FP64 reductions): energies at
    every point within 1e-6 of the oracle's, and both switching fields,
    bisected to 1e-4 of the anisotropy field from the last unswitched
    minimum, within 1e-3 of the oracle's bisection of the same bracket."""
    from paper_1309_5796_amd import binding
    say("mixed loop with bisection")
    c = binding.Context(0)
    try:
        res, bsw = _gpu_loop(c, loop_oracle["mesh"], loop_oracle["fields"], binding.MIXED, refine_tol_T=BISECT_T)
    finally:
        c.close()
    recs, s, fields = loop_oracle["recs"], loop_oracle["system"], loop_oracle["fields"]
    for k, (r, ro) in enumerate(zip(res, recs)):
        assert r.status in (0, 2), k
        assert abs(r.energy_J - ro.E) < 1e-6 * _scale(r), k
    sw_gpu = _switch_steps([r.m_avg for r in res])
    assert len(bsw) == 2 and len(sw_gpu) == 2
    for b_gpu, k in zip(bsw, sw_gpu):
        b_or = bisect_switch(s, loop_oracle["ms"][k - 1], fields[k - 1], fields[k], U, BISECT_T, Options())
        say(f"  switching field: library {b_gpu:.5f} T, oracle {b_or:.5f} T")
        assert abs(b_gpu - b_or) <= 1e-3 * abs(b_or)
