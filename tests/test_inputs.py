"""The seeded input generators (CPU only).  The request stream of the served
form: Poisson arrivals, log-uniform problem sizes, 2:2:1 boxes, the
FP64/mixed coin, the field range and the grain density, checked
statistically on the 2,000 requests, and the prefix property the bounded
runs rely on.  The easy axes, uniform on the 15 degree cap; the grains and
their boundary phase; the grain cubes' cell rule."""
import math

import numpy as np

from paper_1309_5796_amd import meshgen


def test_request_stream_recipe():
    rate = 200.0
    reqs = meshgen.config5_requests(n_requests=2000, rate_hz=rate)
    t = np.array([r.arrival_s for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    # exponential gaps: mean 1/rate (std of the mean 2.2% here) and
    # coefficient of variation 1
    assert abs(gaps.mean() * rate - 1.0) < 0.1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1
    n = np.array([r.cells[2] for r in reqs])
    assert all(r.cells == (2 * r.cells[2], 2 * r.cells[2], r.cells[2]) for r in reqs)
    # nodes of a 2n x 2n x n box of cells, about 4 n^3, log-uniform over
    # 1.2e3 .. 5.2e5: each decade-half of the log range holds half the requests
    nodes = (2 * n + 1) ** 2 * (n + 1)
    assert nodes.min() >= 0.5 * 1.2e3 and nodes.max() <= 2.0 * 5.2e5
    mid = math.sqrt(1.2e3 * 5.2e5)
    assert abs(np.mean(4.0 * n.astype(float) ** 3 < mid) - 0.5) < 0.05
    prec = np.array([r.precision for r in reqs])
    assert set(prec.tolist()) == {0, 1} and abs(prec.mean() - 0.5) < 0.05
    for r in reqs:
        b = np.asarray(r.b_ext)
        s = float(np.dot(b, meshgen.U_H_1DEG))
        np.testing.assert_allclose(b, s * meshgen.U_H_1DEG, atol=1e-15)
        assert -4.0 <= s <= 4.0
        # 64 grains per 200 x 200 x 100 nm, at least one
        vol = (2 * r.cells[2] * r.h) ** 2 * (r.cells[2] * r.h)
        assert r.n_grains == max(1, int(round(64 * vol / (200e-9 * 200e-9 * 100e-9))))
        assert r.h == 1.6e-9


def test_request_stream_is_seeded_and_prefix_stable():
    a = meshgen.config5_requests(n_requests=2000)
    b = meshgen.config5_requests(n_requests=48)
    for x, y in zip(a[:48], b):
        assert (x.arrival_s, x.cells, x.n_grains, x.precision, x.seed) == (y.arrival_s, y.cells, y.n_grains,
                                                                           y.precision, y.seed)
        np.testing.assert_array_equal(x.b_ext, y.b_ext)
    c = meshgen.config5_requests(n_requests=2000)
    assert [r.seed for r in a] == [r.seed for r in c]


def test_easy_axes_uniform_on_the_15_degree_cap():
    rng = np.random.default_rng(3)
    ax = np.array([meshgen.cap_axis(rng) for _ in range(4000)])
    np.testing.assert_allclose(np.linalg.norm(ax, axis=1), 1.0, atol=1e-15)
    c15 = math.cos(math.radians(15.0))
    assert ax[:, 2].min() >= c15 - 1e-15
    # uniform on the cap: cos(theta) uniform on [cos 15 deg, 1], azimuth uniform
    assert abs(ax[:, 2].mean() - (1 + c15) / 2) < 6 * (1 - c15) / math.sqrt(12 * len(ax))   # 6 standard errors
    phi = np.arctan2(ax[:, 1], ax[:, 0])
    assert abs(np.cos(phi).mean()) < 0.05 and abs(np.sin(phi).mean()) < 0.05


def test_grains_and_their_boundary_phase():
    mesh = meshgen.kuhn_box((20e-9, 20e-9, 10e-9), (20, 20, 10), air=True)
    meshgen.assign_grains(mesh, 8, np.random.default_rng(4))
    mag = mesh.region > 0
    regs = set(np.unique(mesh.region[mag]).tolist())
    assert regs <= set(range(1, 10)) and 9 in regs and len(regs) >= 6
    # grain boundaries: no anisotropy, reduced exchange; grains: the bulk
    # constants with easy axes on the 15 degree cap
    mats = {m.region: m for m in mesh.materials}
    assert mats[9].K1 == 0.0 and mats[9].A == meshgen.A_GB_JM == 2e-12
    c15 = math.cos(math.radians(15.0))
    for g in range(1, 9):
        assert mats[g].K1 == meshgen.K1_JM3 and mats[g].A == meshgen.A_JM
        assert float(mats[g].axis[2]) >= c15 - 1e-15
    # a thin layer: some, but a minority, of the magnet tets
    frac = np.mean(mesh.region[mag] == 9)
    assert 0.0 < frac < 0.5
    # air keeps region 0
    assert np.all(mesh.region[~mag] == 0)


def test_grain_cube_cells_rule():
    # n(L) = round(9 (L / 10 nm)^(ln 4 / ln 6)): 9 cells at 10 nm and, six
    # times the edge giving four times the cells, 36 at 60 nm
    assert meshgen.config4_cells(10e-9) == 9
    assert meshgen.config4_cells(60e-9) == 36
    Ls = np.exp(np.linspace(np.log(10e-9), np.log(60e-9), 50))
    n = [meshgen.config4_cells(L) for L in Ls]
    assert all(b >= a for a, b in zip(n, n[1:]))
