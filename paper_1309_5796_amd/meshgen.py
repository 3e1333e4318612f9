"""Seeded synthetic inputs for the curvilinear steepest-descent minimizer.

This module only *generates inputs*: node coordinates, Kuhn-split tetrahedra,
region ids, Dirichlet flags, the geometry of the open-boundary shell, material
tables, initial magnetizations, applied-field lists and request streams.  It
holds none of the method's arithmetic (no finite-element matrices, no shell
metric, no energies); both the CPU oracle and the HIP library consume what it
produces and each computes everything else on its own.

Mesh recipe (the paper's workload is a tetrahedral P1 mesh of a small
Nd2Fe14B particle, Results section; its own mesh is not available, so these
boxes stand in for it):

* Tensor-product grid; every hexahedral cell is split into the 6 Kuhn
  tetrahedra that share the cell's main diagonal, so neighbouring cells are
  conforming.
* Magnet box of half-extent ``a`` per axis, ``n`` cells of spacing ``h``.
* Optional air layer from ``a`` to ``2a`` per side, geometrically graded from
  ``h`` with ratio <= 1.25 (the smallest cell count that reaches ``2a`` at
  ratio 1.25, then the ratio is solved so the layer ends exactly at ``2a``),
  followed by 4 uniform cells of transformation shell out to ``3a``.  The outer
  box faces are Dirichlet (potential 0).
* Optional jitter of interior magnet nodes by U(-0.1h, 0.1h) per coordinate;
  surface and air nodes stay on the grid, so the magnet box is exact.

All lengths are metres.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 1309579600
# field direction: z tilted by 1 degree towards x
U_H_1DEG = np.array([math.sin(math.radians(1.0)), 0.0, math.cos(math.radians(1.0))])

# Nd2Fe14B-like material used by every workload
JS_T = 1.61
K1_JM3 = 4.9e6
A_JM = 8e-12
A_GB_JM = 2e-12


@dataclass
class Material:
    region: int
    Js: float
    K1: float
    A: float
    axis: np.ndarray


@dataclass
class Mesh:
    xyz: np.ndarray            # (n_nodes, 3) float64, metres
    tets: np.ndarray           # (n_tets, 4) int32
    region: np.ndarray         # (n_tets,) int32; 0 = non-magnetic (air/shell)
    dirichlet: np.ndarray      # (n_nodes,) uint8; 1 = potential fixed to 0
    shell: Optional[np.ndarray] = None   # (9,) centre(3), a_air(3), b(3)
    shape: tuple = ()          # grid node counts (nx, ny, nz)
    magnet_cells: tuple = ()   # magnet cells per axis
    h: float = 0.0             # magnet cell size
    materials: List[Material] = field(default_factory=list)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


def _graded_layer(h: float, thickness: float, max_ratio: float = 1.25) -> np.ndarray:
    """Cell sizes of a layer that starts next to a cell of size h and grows by a
    constant ratio <= max_ratio, ending exactly at `thickness`."""
    n, acc, c = 0, 0.0, h
    while acc < thickness * (1 - 1e-12):
        n += 1
        c *= max_ratio
        acc += c
    lo, hi = 1.0, max_ratio          # sum_{k=1..n} h r^k == thickness
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = h * sum(mid ** k for k in range(1, n + 1))
        if s < thickness:
            lo = mid
        else:
            hi = mid
    r = 0.5 * (lo + hi)
    sizes = np.array([h * r ** k for k in range(1, n + 1)])
    sizes *= thickness / sizes.sum()
    return sizes


def axis_coords(a: float, n_cells: int, air: bool, shell_cells: int = 4):
    """Node coordinates along one axis; returns (coords, i0, i1, a_air, b)
    where nodes i0..i1 are the magnet's."""
    h = 2 * a / n_cells
    mag = np.linspace(-a, a, n_cells + 1)
    if not air:
        return mag, 0, n_cells, a, a
    a_air, b = 2 * a, 3 * a
    layer = _graded_layer(h, a_air - a)
    out = a + np.cumsum(layer)
    out[-1] = a_air
    sh = a_air + (b - a_air) * np.arange(1, shell_cells + 1) / shell_cells
    pos = np.concatenate([out, sh])
    coords = np.concatenate([-pos[::-1], mag, pos])
    i0 = len(pos)
    return coords, i0, i0 + n_cells, a_air, b


# The 6 Kuhn tetrahedra of a unit cell: one per ordering of the axes, walking
# from corner (0,0,0) to (1,1,1) one unit step per axis.
_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def kuhn_box(half_extent: Sequence[float], cells: Sequence[int], *, air: bool = True,
             jitter: float = 0.0, rng: Optional[np.random.Generator] = None) -> Mesh:
    """Kuhn-split box magnet, optionally surrounded by graded air and the
    transformation shell.  Region 1 for every magnet tet (override later)."""
    axes = [axis_coords(float(a), int(n), air) for a, n in zip(half_extent, cells)]
    X, Y, Z = (ax[0] for ax in axes)
    nx, ny, nz = len(X), len(Y), len(Z)
    gi, gj, gk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # node id = i + nx*(j + ny*k): lexicographic with x fastest
    gi, gj, gk = (g.transpose(2, 1, 0).ravel() for g in (gi, gj, gk))
    xyz = np.stack([X[gi], Y[gj], Z[gk]], axis=1).astype(np.float64)

    def nid(i, j, k):
        return i + nx * (j + ny * k)

    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    ci, cj, ck = (c.transpose(2, 1, 0).ravel() for c in (ci, cj, ck))
    tets = []
    for p in _PERMS:
        cur = [ci.copy(), cj.copy(), ck.copy()]
        verts = [nid(*cur)]
        for ax in p:
            cur[ax] = cur[ax] + 1
            verts.append(nid(*cur))
        tets.append(np.stack(verts, axis=1))
    # order tets cell-major: the 6 tets of one cell are adjacent
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    cell_of_tet = np.repeat(np.arange(ci.size), 6)

    (i0, i1), (j0, j1), (k0, k1) = ((ax[1], ax[2]) for ax in axes)
    cin = ((ci >= i0) & (ci < i1) & (cj >= j0) & (cj < j1) & (ck >= k0) & (ck < k1))
    region = cin[cell_of_tet].astype(np.int32)

    dirichlet = np.zeros(nx * ny * nz, dtype=np.uint8)
    if air:
        bnd = (gi == 0) | (gi == nx - 1) | (gj == 0) | (gj == ny - 1) | (gk == 0) | (gk == nz - 1)
        dirichlet[bnd] = 1

    h = 2 * float(half_extent[0]) / int(cells[0])
    if jitter > 0:
        assert rng is not None
        inner = ((gi > i0) & (gi < i1) & (gj > j0) & (gj < j1) & (gk > k0) & (gk < k1))
        idx = np.nonzero(inner)[0]
        xyz[idx] += rng.uniform(-jitter * h, jitter * h, size=(idx.size, 3))

    shell = None
    if air:
        shell = np.array([0.0, 0.0, 0.0] + [ax[3] for ax in axes] + [ax[4] for ax in axes])
    return Mesh(xyz=xyz, tets=tets, region=region, dirichlet=dirichlet, shell=shell,
                shape=(nx, ny, nz), magnet_cells=tuple(int(c) for c in cells), h=h,
                materials=[Material(1, JS_T, K1_JM3, A_JM, np.array([0.0, 0.0, 1.0]))])


def cap_axis(rng: np.random.Generator, half_angle_deg: float = 15.0) -> np.ndarray:
    """Unit vector uniform on the spherical cap of the given half-angle about z."""
    ct = rng.uniform(math.cos(math.radians(half_angle_deg)), 1.0)
    ph = rng.uniform(0.0, 2 * math.pi)
    st = math.sqrt(max(0.0, 1 - ct * ct))
    return np.array([st * math.cos(ph), st * math.sin(ph), ct])


def tet_centroids(mesh: Mesh) -> np.ndarray:
    return mesh.xyz[mesh.tets].mean(axis=1)


def assign_grains(mesh: Mesh, n_grains: int, rng: np.random.Generator,
                  gb_half_width: float = 1e-9) -> None:
    """Voronoi grains from n_grains centres uniform in the magnet box; magnet
    tets within gb_half_width of a Voronoi face form the grain-boundary phase
    (K1 = 0, A = 2 pJ/m).  Regions: grain g -> g+1, boundary -> n_grains+1."""
    mag = mesh.region > 0
    xyz = mesh.xyz
    mt = mesh.tets[mag]
    on_magnet = np.zeros(xyz.shape[0], dtype=bool)
    on_magnet[mt.ravel()] = True
    lo = xyz[on_magnet].min(axis=0)
    hi = xyz[on_magnet].max(axis=0)
    centres = rng.uniform(lo, hi, size=(n_grains, 3))
    axes = [cap_axis(rng) for _ in range(n_grains)]
    cen = xyz[mt].mean(axis=1)
    if n_grains == 1:
        reg = np.ones(cen.shape[0], dtype=np.int32)
    else:
        from scipy.spatial import cKDTree
        dist, idx = cKDTree(centres).query(cen, k=2)
        c1, c2 = idx[:, 0], idx[:, 1]
        d1, dd = dist[:, 0] ** 2, dist[:, 1] ** 2
        sep = np.linalg.norm(centres[c2] - centres[c1], axis=1)
        dist_face = (dd - d1) / (2 * sep)
        reg = (c1 + 1).astype(np.int32)
        reg[dist_face < gb_half_width] = n_grains + 1
    region = mesh.region.copy()
    region[mag] = reg
    mesh.region = region
    mesh.materials = [Material(g + 1, JS_T, K1_JM3, A_JM, axes[g]) for g in range(n_grains)]
    if n_grains > 1:
        mesh.materials.append(Material(n_grains + 1, JS_T, 0.0, A_GB_JM, np.array([0.0, 0.0, 1.0])))


def noisy_plus_z(n: int, rng: Optional[np.random.Generator], sigma: float = 0.01) -> np.ndarray:
    """+z plus N(0, sigma) per component, renormalized; rng None gives exact +z."""
    m = np.zeros((n, 3))
    m[:, 2] = 1.0
    if rng is not None and sigma > 0:
        m += rng.normal(0.0, sigma, size=(n, 3))
        m /= np.linalg.norm(m, axis=1, keepdims=True)
    return m


def streams(cfg: int):
    """Independent generators [jitter, m-noise, grains, requests] of a workload."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(SEED_BASE + cfg).spawn(4)]


def n_magnetic(mesh: Mesh) -> int:
    return int(np.unique(mesh.tets[mesh.region > 0]).size)


# ---------------------------------------------------------------------------
# Workloads.  cfg 1: 20 nm cube, 10^3 cells, jitter, noisy +z, -2 T.
# cfg 2: 80 nm cube, 40^3 cells, hysteresis +8 -> -8 -> +8 T in 0.1 T steps.
# cfg 3: 200x200x100 nm box, 126x126x63 cells, 64 grains, -2 T, noisy +z.
# cfg 4: 256 cubes of edge log-uniform 10-60 nm, one grain each, -1 T.
# cfg 5: request stream of 2:2:1 boxes (h = 1.6 nm), 1.2k-520k nodes.
# ---------------------------------------------------------------------------

def config1(air: bool = True) -> dict:
    rj, rm, _, _ = streams(1)
    mesh = kuhn_box((10e-9, 10e-9, 10e-9), (10, 10, 10), air=air, jitter=0.1, rng=rj)
    n = n_magnetic(mesh)
    return dict(mesh=mesh, m0=noisy_plus_z(n, rm), b_ext=-2.0 * U_H_1DEG, tol=1e-6)


# ---------------------------------------------------------------------------
# The paper's own experiment (Results, comparison with the LLG solver): a
# 20 nm Nd2Fe14B sphere, field ramped 0 -> -6 T in 0.01 T steps at 45 degrees
# to the easy axis.  The paper's mesh (80,000 tets, edge 0.76 nm) is not
# available; a staircase ball of Kuhn cells of the same tet count stands in.
# ---------------------------------------------------------------------------

U_H_45DEG = np.array([np.sin(np.pi / 4), 0.0, np.cos(np.pi / 4)])


def kuhn_ball(diameter: float = 20e-9, cells: int = 30, air: bool = True) -> Mesh:
    """Kuhn-split cube of `cells`^3 cells spanning the sphere's bounding box
    (plus graded air and the transformation shell); tets whose centroid lies
    in the sphere are magnetic (region 1), the rest of the box is air.  30
    cells give ~85,000 magnetic tets with edges 0.67-1.15 nm."""
    r = 0.5 * diameter
    mesh = kuhn_box((r, r, r), (cells, cells, cells), air=air)
    cen = mesh.xyz[mesh.tets].mean(axis=1)
    region = (np.linalg.norm(cen, axis=1) < r).astype(np.int32)
    return Mesh(xyz=mesh.xyz, tets=mesh.tets, region=region, dirichlet=mesh.dirichlet, shell=mesh.shell,
                shape=mesh.shape, magnet_cells=mesh.magnet_cells, h=mesh.h,
                materials=[Material(1, JS_T, K1_JM3, A_JM, np.array([0.0, 0.0, 1.0]))])


def sphere_experiment(cells: int = 30, step: float = 0.01, bmax: float = 6.0) -> dict:
    """m0 = +z (the easy axis); fields 0, -step, ..., -bmax tesla along the
    45-degree direction."""
    mesh = kuhn_ball(cells=cells)
    n = n_magnetic(mesh)
    k = int(round(bmax / step))
    fields = -(np.arange(k + 1) * step)[:, None] * U_H_45DEG[None, :]
    return dict(mesh=mesh, m0=np.tile([0.0, 0.0, 1.0], (n, 1)), fields=fields, tol=1e-6)


def delaunay_box(seed: int, outer: float = 30e-9, inner: float = 12e-9, n: int = 16) -> Mesh:
    """Irregular test mesh: Delaunay tetrahedra of a jittered (n+1)^3 point
    grid over [-outer, outer]^3 (interior points moved by up to 0.3 of the
    spacing, boundary points kept on their faces); tets whose centroid lies in
    [-inner, inner]^3 are magnetic (region 1); the outer faces are Dirichlet;
    no transformation shell.  Node degrees vary (about 8 to 30)."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    t = np.linspace(-outer, outer, n + 1)
    g = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    on_face = np.abs(np.abs(g) - outer) < 1e-6 * (t[1] - t[0])
    jit = rng.uniform(-0.3, 0.3, size=g.shape) * (t[1] - t[0])
    xyz = np.where(on_face, g, g + jit)
    tets = Delaunay(xyz).simplices.astype(np.int32)
    d = xyz[tets[:, 1:]] - xyz[tets[:, :1]]
    vol = np.abs(np.linalg.det(d)) / 6.0
    tets = tets[vol > 1e-6 * (t[1] - t[0]) ** 3]          # drop flat boundary slivers
    cen = xyz[tets].mean(axis=1)
    region = np.all(np.abs(cen) < inner, axis=1).astype(np.int32)
    dirichlet = np.any(on_face, axis=1).astype(np.uint8)
    return Mesh(xyz=xyz, tets=tets, region=region, dirichlet=dirichlet,
                materials=[Material(1, JS_T, K1_JM3, A_JM, np.array([0.0, 0.0, 1.0]))])


def sweep_fields(bmax: float = 8.0, step: float = 0.1) -> np.ndarray:
    """+bmax -> -bmax -> +bmax in `step` T steps along the 1-degree direction."""
    k = int(round(bmax / step))
    down = np.arange(k, -k - 1, -1) * step
    up = np.arange(-k + 1, k + 1) * step
    B = np.concatenate([down, up])
    return B[:, None] * U_H_1DEG[None, :]


def config2(cells: int = 40, edge: float = 80e-9) -> dict:
    mesh = kuhn_box((edge / 2,) * 3, (cells,) * 3, air=True)
    n = n_magnetic(mesh)
    return dict(mesh=mesh, m0=noisy_plus_z(n, None), fields=sweep_fields(), tol=1e-6)


def config3(scale: float = 1.0) -> dict:
    """scale < 1 shrinks the box and cell counts (same h) for quick runs."""
    rj, rm, rg, _ = streams(3)
    cx, cz = int(round(126 * scale)), int(round(63 * scale))
    h = 200e-9 / 126
    mesh = kuhn_box((cx * h / 2, cx * h / 2, cz * h / 2), (cx, cx, cz), air=True)
    assign_grains(mesh, 64 if scale == 1.0 else max(1, int(round(64 * scale ** 3))), rg)
    n = n_magnetic(mesh)
    return dict(mesh=mesh, m0=noisy_plus_z(n, rm), b_ext=-2.0 * U_H_1DEG, tol=1e-6)


def config4_cells(edge_m: float) -> int:
    return int(round(9 * (edge_m / 10e-9) ** (math.log(4) / math.log(6))))


def config4(n_problems: int = 256, edge_range=(10e-9, 60e-9)) -> List[dict]:
    _, rm, rg, _ = streams(4)
    out = []
    for _ in range(n_problems):
        L = math.exp(rg.uniform(math.log(edge_range[0]), math.log(edge_range[1])))
        n = config4_cells(L)
        mesh = kuhn_box((L / 2,) * 3, (n,) * 3, air=True)
        ax = cap_axis(rg)
        mesh.materials = [Material(1, JS_T, K1_JM3, A_JM, ax)]
        nm = n_magnetic(mesh)
        out.append(dict(mesh=mesh, m0=noisy_plus_z(nm, rm), b_ext=-1.0 * U_H_1DEG, tol=1e-6, edge=L))
    return out


@dataclass
class Request:
    arrival_s: float
    cells: tuple
    h: float
    n_grains: int
    b_ext: np.ndarray
    precision: int          # 0 = FP64, 1 = mixed
    seed: int


def config5_requests(n_requests: int = 2000, rate_hz: float = 200.0,
                     node_range=(1.2e3, 5.2e5), h: float = 1.6e-9) -> List[Request]:
    _, _, _, rr = streams(5)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rr.exponential(1.0 / rate_hz)
        target = math.exp(rr.uniform(math.log(node_range[0]), math.log(node_range[1])))
        n = max(1, int(round((target / 4.0) ** (1.0 / 3.0))))
        cells = (2 * n, 2 * n, n)
        vol = (2 * n * h) * (2 * n * h) * (n * h)
        ng = max(1, int(round(64 * vol / (200e-9 * 200e-9 * 100e-9))))
        B = rr.uniform(-4.0, 4.0)
        prec = int(rr.integers(0, 2))
        out.append(Request(t, cells, h, ng, B * U_H_1DEG, prec, int(rr.integers(0, 2**31 - 1))))
    return out


def request_mesh(req: Request) -> dict:
    nx, ny, nz = req.cells
    mesh = kuhn_box((nx * req.h / 2, ny * req.h / 2, nz * req.h / 2), req.cells, air=True)
    assign_grains(mesh, req.n_grains, np.random.default_rng(req.seed))
    n = n_magnetic(mesh)
    return dict(mesh=mesh, m0=noisy_plus_z(n, None), b_ext=req.b_ext, tol=1e-6)
