"""FP64 finite-element model of the micromagnetic energy -- oracle (test
infrastructure only; see the package docstring).

The paper minimizes the total Gibbs free energy (stray field + exchange +
anisotropy + external, Method section, eq. (1)) discretized with standard
linear tetrahedral elements (Abstract).  It does not write the discrete
energy down; this module uses the reading:

* exchange: consistent P1 stiffness, E_ex = sum_c m_c^T K m_c,
  K_ij = sum_e A_e V_e grad(phi_i).grad(phi_j);
* anisotropy: nodal (lumped) uniaxial, E_an = sum_e V_e K1_e - sum_i m_i^T Q_i m_i,
  Q_i = sum_{e ni i} V_e/4 K1_e u_e u_e^T (zero for m along the easy axis);
* Zeeman: E_Z = -Ms sum_i V_i b.m_i with b = mu0 H_ext in tesla;
* stray field from a magnetic scalar potential (Results, comparison
  section): L u = b, b_j = Ms int_magnet m . grad(phi_j), E_d = mu0/2 b.u,
  with the open boundary handled by a space transformation (Brunotte 1992,
  cited there): a per-axis map of the shell [a, b) onto [a, inf) and the
  metric tensor evaluated at each tetrahedron's centroid;
* effective field (variational, lumped; the paper defines h_eff = -dphi/dm
  below eq. (9)): h_i = -1/(mu0 Ms^2 V_i) dE/dm_i, in units of Ms.

All lengths are metres and all energies joules; the reduced energy used by
the minimizer is e = E/(mu0 Ms^2) (cubic metres).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

MU0 = 4e-7 * np.pi

EXCH, ANIS, ZEEM, DEMAG = 1, 2, 4, 8
ALL_TERMS = 15


def tet_geometry(xyz: np.ndarray, tets: np.ndarray):
    """Volumes and P1 basis-function gradients of every tetrahedron.

    With D the 3x3 matrix whose rows are x_k - x_0 (k = 1..3), the barycentric
    coordinate lambda_k (k >= 1) has gradient equal to column k of D^{-1}, and
    grad(lambda_0) = -sum_k grad(lambda_k).  V = |det D| / 6.
    Returns (V[E], grad[E,4,3]).  Raises ValueError on a degenerate tet.
    """
    x = xyz[tets]                                   # (E, 4, 3)
    D = x[:, 1:, :] - x[:, :1, :]                   # (E, 3, 3), row k-1 = x_k - x_0
    det = np.linalg.det(D)
    scale = np.abs(D).max(axis=(1, 2)) ** 3
    if np.any(np.abs(det) <= 1e-10 * scale):
        raise ValueError("degenerate tetrahedron")
    Dinv = np.linalg.inv(D)
    grad = np.empty((tets.shape[0], 4, 3))
    grad[:, 1:, :] = np.transpose(Dinv, (0, 2, 1))  # grad[e, k] = Dinv[e, :, k-1]
    grad[:, 0, :] = -grad[:, 1:, :].sum(axis=1)
    return np.abs(det) / 6.0, grad


def shell_metric(centroids: np.ndarray, shell) -> np.ndarray:
    """Diagonal metric tensor of the open-boundary space transformation.

    Per axis, the map f(t) = a (b - a) / (b - |t - c|) sends the shell
    a <= |t - c| < b onto [a, inf) and is the identity inside; its derivative
    is f'(t) = a (b - a) / (b - |t - c|)^2 in the shell and 1 inside.  With
    J = diag(f'_x, f'_y, f'_z) the transformed Laplacian has the metric
    |det J| J^{-1} J^{-T} = diag(f'_y f'_z / f'_x, f'_x f'_z / f'_y,
    f'_x f'_y / f'_z), evaluated at the centroid.  Returns (E, 3) diagonals.
    Pinned against its definition (the map's Jacobian by central differences,
    the metric by generic 3x3 algebra) and through the demagnetizing factors.
    """
    E = centroids.shape[0]
    if shell is None:
        return np.ones((E, 3))
    c, a, b = np.asarray(shell[0:3]), np.asarray(shell[3:6]), np.asarray(shell[6:9])
    fp = np.ones((E, 3))
    for k in range(3):
        t = np.abs(centroids[:, k] - c[k])
        out = t > a[k]
        fp[out, k] = a[k] * (b[k] - a[k]) / (b[k] - t[out]) ** 2
    return np.stack([fp[:, 1] * fp[:, 2] / fp[:, 0],
                     fp[:, 0] * fp[:, 2] / fp[:, 1],
                     fp[:, 0] * fp[:, 1] / fp[:, 2]], axis=1)


class System:
    """Assembled FE operators of one mesh with its materials.

    mesh: object with xyz (n,3), tets (E,4), region (E,), dirichlet (n,),
    shell (9,) or None, materials [objects with region, Js, K1, A, axis].
    Magnetic nodes are the nodes of region >= 1 tets, in ascending global
    index; arrays indexed by magnetic node use that order.
    """

    def __init__(self, mesh, direct_max: int = 60000):
        self.mesh = mesh
        xyz, tets = np.asarray(mesh.xyz, float), np.asarray(mesh.tets, np.int64)
        region = np.asarray(mesh.region)
        self.V_e, self.grad = tet_geometry(xyz, tets)
        mats = {int(m.region): m for m in mesh.materials}
        mag = region > 0
        self.mag_tets = np.nonzero(mag)[0]
        Js = {mats[int(r)].Js for r in np.unique(region[mag])}
        if len(Js) != 1:
            raise ValueError("one saturation polarization for all magnetic regions")
        self.Js = Js.pop()
        self.Ms = self.Js / MU0
        self.mu0Ms2 = MU0 * self.Ms ** 2

        self.nodes = np.unique(tets[mag])                       # global ids, ascending
        self.N = self.nodes.size
        gmap = -np.ones(xyz.shape[0], dtype=np.int64)
        gmap[self.nodes] = np.arange(self.N)
        self.gmap = gmap
        mt = tets[mag]
        self.loc = gmap[mt]                                      # (Em, 4) magnetic indices
        Vm = self.V_e[mag]
        self.Vm = Vm
        gm = self.grad[mag]
        self.gm = gm
        reg = region[mag]
        A_e = np.array([mats[int(r)].A for r in reg])
        K1_e = np.array([mats[int(r)].K1 for r in reg])
        u_e = np.array([np.asarray(mats[int(r)].axis, float) / np.linalg.norm(mats[int(r)].axis)
                        for r in reg])

        # lumped nodal volumes: every vertex of a tet carries a quarter of it
        self.V = np.zeros(self.N)
        np.add.at(self.V, self.loc.ravel(), np.repeat(Vm / 4.0, 4))

        # exchange stiffness K_ij = sum_e A_e V_e grad_i . grad_j
        rows = np.repeat(self.loc, 4, axis=1).ravel()
        cols = np.tile(self.loc, (1, 4)).ravel()
        vals = (A_e * Vm)[:, None, None] * np.einsum("eac,ebc->eab", gm, gm)
        self.K = sp.csr_matrix((vals.ravel(), (rows, cols)), shape=(self.N, self.N))
        self.K.sum_duplicates()

        # lumped anisotropy tensors Q_i = sum_e V_e/4 K1_e u_e u_e^T
        self.Q = np.zeros((self.N, 3, 3))
        uu = (Vm / 4.0 * K1_e)[:, None, None] * np.einsum("ei,ej->eij", u_e, u_e)
        for a in range(4):
            np.add.at(self.Q, self.loc[:, a], uu)
        self.anis_const = float(np.sum(Vm * K1_e))

        # scalar potential: all nodes, Dirichlet rows/cols eliminated
        self.has_potential = bool(np.any(np.asarray(mesh.dirichlet) > 0))
        if self.has_potential:
            cen = xyz[tets].mean(axis=1)
            T = shell_metric(cen, mesh.shell)
            Tg = self.grad * T[:, None, :]
            rows = np.repeat(tets, 4, axis=1).ravel()
            cols = np.tile(tets, (1, 4)).ravel()
            vals = self.V_e[:, None, None] * np.einsum("eac,ebc->eab", Tg, self.grad)
            n = xyz.shape[0]
            Lfull = sp.csr_matrix((vals.ravel(), (rows, cols)), shape=(n, n))
            Lfull.sum_duplicates()
            self.free = np.nonzero(np.asarray(mesh.dirichlet) == 0)[0]
            self.L = Lfull[self.free][:, self.free].tocsc()
            fmap = -np.ones(n, dtype=np.int64)
            fmap[self.free] = np.arange(self.free.size)
            self.fmap = fmap
            self.Nt = self.free.size
            self._solve = spla.factorized(self.L) if self.Nt <= direct_max else None
        else:
            self.Nt = 0

    # -- stray field ------------------------------------------------------
    def rhs(self, m: np.ndarray) -> np.ndarray:
        """b_j = Ms sum_{e magnetic, e ni j} V_e/4 sum_{a in e} m_a . grad(phi_j)|_e
        on the free potential nodes."""
        msum = m[self.loc].sum(axis=1)                           # (Em, 3)
        contrib = self.Ms * (self.Vm / 4.0)[:, None] * np.einsum("ec,eac->ea", msum, self.gm)
        b = np.zeros(self.mesh.xyz.shape[0])
        np.add.at(b, np.asarray(self.mesh.tets)[self.mag_tets].ravel(), contrib.ravel())
        return b[self.free]

    def solve_potential(self, b: np.ndarray) -> np.ndarray:
        """L u = b: sparse LU where it fits (the paper's CPU path factorizes
        at setup), else CG to a relative residual of 1e-13."""
        if self._solve is not None:
            return self._solve(b)
        d = self.L.diagonal()
        M = spla.LinearOperator(self.L.shape, matvec=lambda x: x / d)
        u, info = spla.cg(self.L, b, rtol=1e-13, atol=0.0, maxiter=20000, M=M)
        if info != 0:
            raise RuntimeError("oracle CG did not converge")
        return u

    def demag_field(self, u_free: np.ndarray) -> np.ndarray:
        """h_d,i = -1/(Ms V_i) sum_{e ni i} V_e/4 grad(u)|_e (units of Ms)."""
        u = np.zeros(self.mesh.xyz.shape[0])
        u[self.free] = u_free
        ut = u[np.asarray(self.mesh.tets)[self.mag_tets]]        # (Em, 4)
        gu = np.einsum("ea,eac->ec", ut, self.gm)                # grad u per tet
        acc = np.zeros((self.N, 3))
        w = (self.Vm / 4.0)[:, None] * gu
        for a in range(4):
            np.add.at(acc, self.loc[:, a], w)
        return -acc / (self.Ms * self.V[:, None])

    # -- energy and field -------------------------------------------------
    def evaluate(self, m: np.ndarray, b_ext, terms: int = ALL_TERMS) -> dict:
        """Energy terms (J), reduced energy e = E/(mu0 Ms^2), and the
        effective field h (units of Ms) at the nodal field m (N, 3)."""
        b_ext = np.asarray(b_ext, float)
        h = np.zeros((self.N, 3))
        out = dict(E_ex=0.0, E_an=0.0, E_Z=0.0, E_d=0.0, u=None)
        c = 1.0 / (self.mu0Ms2 * self.V[:, None])
        if terms & EXCH:
            Km = self.K @ m
            out["E_ex"] = float(np.sum(m * Km))
            h += -2.0 * c * Km
        if terms & ANIS:
            Qm = np.einsum("nij,nj->ni", self.Q, m)
            out["E_an"] = self.anis_const - float(np.sum(m * Qm))
            h += 2.0 * c * Qm
        if terms & ZEEM:
            out["E_Z"] = -self.Ms * float(np.sum(self.V * (m @ b_ext)))
            h += b_ext[None, :] / self.Js
        if terms & DEMAG:
            if not self.has_potential:
                raise ValueError("stray field needs a mesh with air and Dirichlet nodes")
            b = self.rhs(m)
            u = self.solve_potential(b)
            out["E_d"] = 0.5 * MU0 * float(b @ u)
            out["u"] = u
            h += self.demag_field(u)
        E = out["E_ex"] + out["E_an"] + out["E_Z"] + out["E_d"]
        out["E"] = E
        out["e"] = E / self.mu0Ms2
        out["h"] = h
        return out

    def reduced_energy_from_field(self, m, h, b_ext, terms: int = ALL_TERMS) -> float:
        """Second energy formula: for this quadratic-plus-linear energy,
        e = -1/2 sum_i V_i m_i.(h_i + h_Z) + sum_e V_e K1_e / (mu0 Ms^2)."""
        hz = np.asarray(b_ext, float) / self.Js if terms & ZEEM else np.zeros(3)
        e = -0.5 * float(np.sum(self.V[:, None] * m * (h + hz[None, :])))
        if terms & ANIS:
            e += self.anis_const / self.mu0Ms2
        return e

    def mean_m(self, m: np.ndarray) -> np.ndarray:
        return (self.V[:, None] * m).sum(axis=0) / self.V.sum()


# -- element-wise evaluation at full size (no assembled matrices) -----------

def local_terms(mesh, m: np.ndarray, sample: np.ndarray, b_ext, terms: int = EXCH | ANIS | ZEEM) -> dict:
    """Exchange, anisotropy and Zeeman parts of the energy (J), summed tet by
    tet, and of the effective field (units of Ms) at the sampled magnetic
    nodes, each from the tets around that node only: the same energy and
    field as System.evaluate (module docstring) without assembling K, Q or
    the potential matrix, so meshes of millions of nodes fit.

    m: (N, 3) at the magnetic nodes (ascending global index); sample:
    magnetic-node indices.  Returns E_ex, E_an, E_Z and h (len(sample), 3).
    """
    xyz, tets = np.asarray(mesh.xyz, float), np.asarray(mesh.tets, np.int64)
    region = np.asarray(mesh.region)
    mats = {int(mt.region): mt for mt in mesh.materials}
    mag = np.nonzero(region > 0)[0]
    mt = tets[mag]
    nodes = np.unique(mt)
    gmap = -np.ones(xyz.shape[0], dtype=np.int64)
    gmap[nodes] = np.arange(nodes.size)
    loc = gmap[mt]                                               # (Em, 4)
    Js = mats[int(region[mag[0]])].Js
    Ms = Js / MU0
    mu0Ms2 = MU0 * Ms * Ms
    b_ext = np.asarray(b_ext, float)
    out = dict(E_ex=0.0, E_an=0.0, E_Z=0.0)
    # energies, in chunks of tets
    V_all = np.zeros(nodes.size)
    for s0 in range(0, mag.size, 1 << 20):
        sl = slice(s0, min(mag.size, s0 + (1 << 20)))
        V_e, grad = tet_geometry(xyz, mt[sl])
        reg = region[mag[sl]]
        A_e = np.array([mats[int(r)].A for r in reg])
        K1_e = np.array([mats[int(r)].K1 for r in reg])
        ax = np.array([np.asarray(mats[int(r)].axis, float) / np.linalg.norm(mats[int(r)].axis) for r in reg])
        me = m[loc[sl]]                                          # (e, 4, 3)
        np.add.at(V_all, loc[sl].ravel(), np.repeat(V_e / 4.0, 4))
        if terms & EXCH:
            G = np.einsum("eac,ebc->eab", grad, grad)             # grad_a . grad_b
            MM = np.einsum("eac,ebc->eab", me, me)                # m_a . m_b
            out["E_ex"] += float(np.sum(A_e * V_e * np.einsum("eab,eab->e", G, MM)))
        if terms & ANIS:
            um = np.einsum("ec,eac->ea", ax, me)                  # u . m_a
            out["E_an"] += float(np.sum(V_e * K1_e * (1.0 - 0.25 * np.sum(um * um, axis=1))))
        if terms & ZEEM:
            out["E_Z"] -= Ms * float(np.sum(V_e / 4.0 * np.einsum("eac,c->e", me, b_ext)))
    # fields at the sampled nodes from their own tets
    sample = np.asarray(sample, np.int64)
    order = np.argsort(loc.ravel(), kind="stable")
    first = np.searchsorted(loc.ravel()[order], sample, side="left")
    last = np.searchsorted(loc.ravel()[order], sample, side="right")
    h = np.zeros((sample.size, 3))
    for k, i in enumerate(sample):
        slots = order[first[k]:last[k]]
        et, vert = slots // 4, slots % 4                          # incident tets, i's vertex in each
        V_e, grad = tet_geometry(xyz, mt[et])
        reg = region[mag[et]]
        Vi = float(np.sum(V_e / 4.0))
        c = 1.0 / (mu0Ms2 * Vi)
        me = m[loc[et]]
        if terms & EXCH:
            A_e = np.array([mats[int(r)].A for r in reg])
            gi = grad[np.arange(et.size), vert]                   # grad(phi_i) in each tet
            Km = np.einsum("e,ec,ebc,ebd->d", A_e * V_e, gi, grad, me)
            h[k] += -2.0 * c * Km
        if terms & ANIS:
            K1_e = np.array([mats[int(r)].K1 for r in reg])
            ax = np.array([np.asarray(mats[int(r)].axis, float) / np.linalg.norm(mats[int(r)].axis) for r in reg])
            Qm = np.einsum("e,ec,ed,d->c", V_e / 4.0 * K1_e, ax, ax, m[i])
            h[k] += 2.0 * c * Qm
        if terms & ZEEM:
            h[k] += b_ext / Js
    out["h"] = h
    return out
