"""The seeded request stream of the served form (CPU only): Poisson
arrivals, log-uniform problem sizes, 2:2:1 boxes, the FP64/mixed coin, the
field range and the grain density, checked statistically on the 2,000
requests, and the prefix property the bounded runs rely on."""
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
