"""Pins of the oracle's finite-element model against closed forms and exact
identities (no GPU).  Each test names the property of the discretization or
of the paper's Method section that it fixes."""
import numpy as np
import pytest

import oracle
from oracle.fem import ANIS, DEMAG, EXCH, MU0, ZEEM
from paper_1309_5796_amd import meshgen


def _box(cells=(4, 4, 4), half=(4e-9, 4e-9, 4e-9), air=False, jitter=0.0, seed=0):
    return meshgen.kuhn_box(half, cells, air=air, jitter=jitter, rng=np.random.default_rng(seed))


def test_p1_gradients_reproduce_affine_functions():
    mesh = _box(jitter=0.1)
    V, grad = oracle.tet_geometry(mesh.xyz, mesh.tets)
    rng = np.random.default_rng(1)
    w, c0 = rng.normal(size=3) * 1e9, rng.normal()
    f = mesh.xyz @ w + c0
    g = np.einsum("ea,eac->ec", f[mesh.tets], grad)
    assert np.allclose(g, w[None, :], rtol=0, atol=1e-9 * np.abs(w).max())
    assert np.abs(grad.sum(axis=1)).max() < 1e-6 * np.abs(grad).max()
    assert np.all(V > 0)


def test_volumes_sum_to_box_exactly_under_jitter():
    mesh = _box(jitter=0.1)
    s = oracle.System(mesh)
    vol = 8e-9 ** 3
    assert abs(s.V_e.sum() - vol) < 1e-13 * vol
    assert abs(s.V.sum() - vol) < 1e-13 * vol


def test_exchange_stiffness_symmetric_psd_with_constant_kernel():
    s = oracle.System(_box(cells=(3, 3, 3), jitter=0.1))
    K = s.K.toarray()
    assert np.abs(K - K.T).max() < 1e-14 * np.abs(K).max()
    assert np.abs(K.sum(axis=1)).max() < 1e-12 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-12 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 1        # only the constants


def test_exchange_energy_exact_for_linear_fields():
    """For m(x) = M x + c (not normalized) P1 is exact: E_ex = A |M|_F^2 Vol."""
    mesh = _box(jitter=0.1)
    s = oracle.System(mesh)
    rng = np.random.default_rng(2)
    M = rng.normal(size=(3, 3)) * 1e8
    c = rng.normal(size=3)
    m = mesh.xyz[s.nodes] @ M.T + c
    E = s.evaluate(m, np.zeros(3), EXCH)["E_ex"]
    exact = meshgen.A_JM * np.sum(M * M) * 8e-9 ** 3
    assert abs(E - exact) < 1e-12 * exact


def test_unjittered_kuhn_stiffness_is_seven_point_stencil():
    """On an unjittered Kuhn grid P1 stiffness equals h times the 7-point
    Laplacian stencil; an interior row has 15 structural nonzeros."""
    h = 2e-9
    s = oracle.System(_box(cells=(4, 4, 4)))
    K = s.K.tocsr() / (meshgen.A_JM * h)
    centre = 2 + 5 * (2 + 5 * 2)
    row = K.getrow(centre)
    assert row.nnz == 15
    vals = dict(zip(row.indices, row.data))
    assert abs(vals[centre] - 6.0) < 1e-12
    for off in (1, 5, 25):
        assert abs(vals[centre + off] + 1.0) < 1e-12 and abs(vals[centre - off] + 1.0) < 1e-12
    others = [v for j, v in vals.items() if abs(j - centre) not in (0, 1, 5, 25)]
    assert len(others) == 8 and max(abs(v) for v in others) < 1e-12


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, np.pi / 2, 2.5])
def test_uniform_state_anisotropy_and_zeeman_closed_form(theta):
    mesh = _box(jitter=0.1)
    s = oracle.System(mesh)
    m = np.tile([np.sin(theta) * 0.6, np.sin(theta) * 0.8, np.cos(theta)], (s.N, 1))
    b = np.array([0.3, -1.2, 0.7])
    ev = s.evaluate(m, b, ANIS | ZEEM | EXCH)
    vol = 8e-9 ** 3
    assert abs(ev["E_an"] - meshgen.K1_JM3 * vol * np.sin(theta) ** 2) < 1e-12 * meshgen.K1_JM3 * vol
    Ms = meshgen.JS_T / MU0
    assert abs(ev["E_Z"] + Ms * vol * (b @ m[0])) < 1e-12 * Ms * vol * np.linalg.norm(b)
    assert abs(ev["E_ex"]) < 1e-25


def test_uniform_magnetization_rhs_vanishes_inside_and_sums_to_zero():
    mesh = meshgen.kuhn_box((4e-9,) * 3, (4, 4, 4), air=True, jitter=0.1, rng=np.random.default_rng(3))
    s = oracle.System(mesh)
    m = np.tile([0.2, -0.5, 0.84], (s.N, 1))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    b = s.rhs(m)
    scale = np.abs(b).max()
    assert abs(b.sum()) < 1e-12 * scale
    x = mesh.xyz[s.free]
    inner = np.all(np.abs(x) < 4e-9 * (1 - 1e-9), axis=1)
    assert inner.sum() == 27
    assert np.abs(b[inner]).max() < 1e-12 * scale


def test_galerkin_identity_and_energy_formulas_agree():
    """b.u (from the potential) equals -Ms^2 sum_i V_i m_i . h_d,i (from the
    field), and the two total-energy formulas agree."""
    c = meshgen.config1()
    s = oracle.System(c["mesh"])
    rng = np.random.default_rng(4)
    m = rng.normal(size=(s.N, 3))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    ev = s.evaluate(m, c["b_ext"], DEMAG)
    from_field = -0.5 * s.mu0Ms2 * float(np.sum(s.V[:, None] * m * ev["h"]))
    assert abs(ev["E_d"] - from_field) < 1e-12 * abs(ev["E_d"])
    L = s.L
    assert abs(L - L.T).max() < 1e-14 * abs(L).max()
    ev = s.evaluate(m, c["b_ext"])
    e2 = s.reduced_energy_from_field(m, ev["h"], c["b_ext"])
    scale = sum(abs(ev[k]) for k in ("E_ex", "E_an", "E_Z", "E_d")) / s.mu0Ms2
    assert abs(ev["e"] - e2) < 1e-13 * scale


def _demag_factor(cells, half, axis=0):
    mesh = meshgen.kuhn_box(half, cells, air=True)
    s = oracle.System(mesh)
    m = np.zeros((s.N, 3))
    m[:, axis] = 1.0
    E = s.evaluate(m, np.zeros(3), DEMAG)["E_d"]
    vol = 8 * np.prod(half)
    return 2 * E / (s.mu0Ms2 * vol)


def test_cube_demag_factor_symmetric_and_approaches_one_third_from_below():
    n4 = [_demag_factor((4, 4, 4), (4e-9,) * 3, ax) for ax in range(3)]
    assert max(n4) - min(n4) < 1e-10
    n8 = _demag_factor((8, 8, 8), (4e-9,) * 3, 0)
    assert 0.28 < n4[0] < n8 < 1 / 3


def aharoni_z(a, b, c):
    """Demagnetizing factor along z of a 2a x 2b x 2c prism (Aharoni, J. Appl.
    Phys. 83, 3432 (1998), eq. (1)), written from the published formula."""
    r = np.sqrt(a * a + b * b + c * c)
    ab, bc, ac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    t = ((b * b - c * c) / (2 * b * c)) * np.log((r - a) / (r + a)) \
        + ((a * a - c * c) / (2 * a * c)) * np.log((r - b) / (r + b)) \
        + (b / (2 * c)) * np.log((ab + a) / (ab - a)) + (a / (2 * c)) * np.log((ab + b) / (ab - b)) \
        + (c / (2 * a)) * np.log((bc - b) / (bc + b)) + (c / (2 * b)) * np.log((ac - a) / (ac + a)) \
        + 2 * np.arctan(a * b / (c * r)) + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c) \
        + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r + (c / (a * b)) * (ac + bc) \
        - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c)
    return t / np.pi


def test_aharoni_formula_self_consistent():
    assert abs(aharoni_z(1, 1, 1) - 1 / 3) < 1e-14
    assert abs(aharoni_z(2, 3, 1) + aharoni_z(3, 1, 2) + aharoni_z(1, 2, 3) - 1) < 1e-13


def test_flat_prism_demag_factor_extrapolates_to_aharoni():
    """2:2:1 prism: N_x = N_y by symmetry, N_z rises monotonically with
    refinement, and the Richardson limit of three levels is Aharoni's value."""
    half = (4e-9, 4e-9, 2e-9)
    Nz = [_demag_factor((2 * k, 2 * k, k), half, 2) for k in (2, 4, 8)]
    nx, ny = (_demag_factor((8, 8, 4), half, ax) for ax in (0, 1))
    assert abs(nx - ny) < 1e-10
    assert Nz[0] < Nz[1] < Nz[2] < aharoni_z(2, 2, 1)
    d1, d2 = Nz[1] - Nz[0], Nz[2] - Nz[1]
    p = np.log2(d1 / d2)
    limit = Nz[2] + d2 / (2 ** p - 1)
    assert 0.8 < p < 2.2
    assert abs(limit - aharoni_z(2, 2, 1)) < 5e-3 * aharoni_z(2, 2, 1)


def test_elementwise_terms_equal_the_assembled_ones():
    """The element-wise evaluation used at full size (no assembled matrices)
    gives the same exchange, anisotropy and Zeeman energies and fields as the
    assembled operators, on a two-material mesh."""
    from oracle.fem import local_terms
    cfg = meshgen.config1()
    mesh = cfg["mesh"]
    region = mesh.region.copy()
    region[np.nonzero(region)[0][::4]] = 2
    mesh = meshgen.Mesh(xyz=mesh.xyz, tets=mesh.tets, region=region, dirichlet=mesh.dirichlet, shell=mesh.shell,
                        materials=mesh.materials + [meshgen.Material(2, meshgen.JS_T, 2.1e6, 5e-12,
                                                                     np.array([0.2, 0.5, 0.8]))])
    s = oracle.System(mesh)
    rng = np.random.default_rng(4)
    m = rng.normal(size=(s.N, 3))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    terms = oracle.fem.EXCH | oracle.fem.ANIS | oracle.fem.ZEEM
    ev = s.evaluate(m, cfg["b_ext"], terms)
    smp = rng.choice(s.N, 60, replace=False)
    lt = local_terms(mesh, m, smp, cfg["b_ext"], terms)
    for k in ("E_ex", "E_an", "E_Z"):
        assert abs(lt[k] - ev[k]) <= 1e-13 * abs(ev[k])
    assert np.abs(lt["h"] - ev["h"][smp]).max() <= 1e-13 * np.abs(ev["h"]).max()


def test_shell_metric_is_the_transformed_laplacians_metric():
    """The shell metric against its definition: per axis the open-boundary
    transformation maps the distance s = |t - c| to itself inside the inner
    box and to a (b - a) / (b - s) in the shell a <= s < b.  Its Jacobian J
    is taken here by central differences of that map and the metric
    |det J| J^-1 J^-T by generic 3x3 linear algebra; the oracle's closed
    form (derivative and diagonal simplification) must agree, off-diagonal
    entries included."""
    c = np.array([1.0, -2.0, 0.5])
    a = np.array([3.0, 2.0, 4.0])
    b = np.array([5.0, 4.5, 5.5])

    def F(x):
        d = x - c
        s = np.abs(d)
        g = np.where(s <= a, s, a * (b - a) / (b - np.minimum(s, b - 1e-300)))
        return c + np.sign(d) * g

    rng = np.random.default_rng(11)
    pts = []
    while len(pts) < 60:
        # per axis: inside, or in the shell, away from the kink at s = a
        x = np.empty(3)
        for k in range(3):
            if rng.random() < 0.5:
                s = rng.uniform(0.0, 0.95 * a[k])
            else:
                s = rng.uniform(a[k] + 0.02 * (b[k] - a[k]), b[k] - 0.05 * (b[k] - a[k]))
            x[k] = c[k] + (1 if rng.random() < 0.5 else -1) * s
        pts.append(x)
    pts = np.array(pts)
    shell = np.concatenate([c, a, b])
    got = oracle.fem.shell_metric(pts, shell)
    h = 1e-6
    for x, gdiag in zip(pts, got):
        J = np.empty((3, 3))
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            J[:, j] = (F(x + e) - F(x - e)) / (2 * h)
        Ji = np.linalg.inv(J)
        G = abs(np.linalg.det(J)) * Ji @ Ji.T
        np.testing.assert_allclose(np.diag(G), gdiag, rtol=1e-6)
        assert np.max(np.abs(G - np.diag(np.diag(G)))) <= 1e-12 * np.max(np.abs(G))
    # no shell: the identity metric
    np.testing.assert_array_equal(oracle.fem.shell_metric(pts, None), np.ones((len(pts), 3)))
