// Host-side P1 tetrahedral assembly (Abstract: standard linear tetrahedral
// finite elements) of the exchange stiffness, the potential-coupling
// matrices, the lumped anisotropy tensors and volumes, and the transformed
// Laplacian of the scalar-potential problem (Results, comparison section:
// scalar potential with a space transformation for the open boundary).
//
// Rows are assembled one at a time from a node -> tetrahedron adjacency, so
// the work splits over host threads without atomics and the sums are
// deterministic.
#include "assemble.h"

#include "amg.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

namespace mmsd {
namespace {

// Sum of many same-signed terms (millions of tets) with a running error term
// (Neumaier): plain accumulation loses ~1e-10 relative at 6M terms, which the
// anisotropy energy's constant part would carry into E_an.
struct CompensatedSum {
  double s = 0, c = 0;
  void add(double x) {
    const double t = s + x;
    c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};


constexpr double kNm = 1e-9;

// Node -> incident (tet, vertex) lists, for the tets selected by `keep`.
void node_tets(int64_t n_nodes, const int32_t* tets, int64_t n_tets, const std::vector<char>& keep,
               std::vector<int>& ptr, std::vector<int>& lst) {
  ptr.assign(n_nodes + 1, 0);
  for (int64_t e = 0; e < n_tets; ++e)
    if (keep[e])
      for (int a = 0; a < 4; ++a) ptr[tets[4 * e + a] + 1]++;
  for (int64_t i = 0; i < n_nodes; ++i) ptr[i + 1] += ptr[i];
  lst.resize(ptr[n_nodes]);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t e = 0; e < n_tets; ++e)
    if (keep[e])
      for (int a = 0; a < 4; ++a) lst[fill[tets[4 * e + a]]++] = (int)(4 * e + a);
}

// Sorted unique neighbour columns of every row.  row_node[r] is the global
// node of row r; col_of[g] maps a global node to its column (-1 = excluded).
// Each thread fills a flat buffer for its contiguous range of rows; the
// ranges are laid end to end after.
void build_pattern(const int32_t* tets, const std::vector<int>& row_node,
                   const std::vector<int>& tptr, const std::vector<int>& tlst,
                   const std::vector<int>& col_of, std::vector<int>& rp, std::vector<int>& ci) {
  const int64_t R = (int64_t)row_node.size();
  rp.assign(R + 1, 0);
  std::mutex mu;
  std::map<int64_t, std::vector<int>> parts;   // by first row of the range
  parallel_for(R, [&](int64_t a, int64_t b) {
    std::vector<int> part, tmp;
    for (int64_t r = a; r < b; ++r) {
      int g = row_node[r];
      tmp.clear();
      for (int k = tptr[g]; k < tptr[g + 1]; ++k) {
        int e = tlst[k] >> 2;
        for (int v = 0; v < 4; ++v) {
          int c = col_of[tets[4 * e + v]];
          if (c >= 0) tmp.push_back(c);
        }
      }
      std::sort(tmp.begin(), tmp.end());
      tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
      part.insert(part.end(), tmp.begin(), tmp.end());
      rp[r + 1] = (int)tmp.size();
    }
    std::lock_guard<std::mutex> g(mu);
    parts[a] = std::move(part);
  });
  for (int64_t r = 0; r < R; ++r) rp[r + 1] += rp[r];
  ci.resize(rp[R]);
  for (auto& kv : parts) std::copy(kv.second.begin(), kv.second.end(), ci.begin() + rp[kv.first]);
}

inline int find_col(const std::vector<int>& ci, int a, int b, int c) {
  auto it = std::lower_bound(ci.begin() + a, ci.begin() + b, c);
  return (int)(it - ci.begin());
}

// Volume and P1 gradients of one tet (nm units).  With D the matrix whose
// rows are x_k - x_0, grad(lambda_k) is column k of D^-1 (k = 1..3) and
// grad(lambda_0) = -sum of the others.  Returns false when degenerate.
bool tet_geo(const double* xyz, const int32_t* t, double* V, double g[4][3]) {
  double D[3][3];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) D[k][c] = (xyz[3 * t[k + 1] + c] - xyz[3 * t[0] + c]) / kNm;
  double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  double sc = 0;
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) sc = std::max(sc, std::fabs(D[k][c]));
  if (!(std::fabs(det) > 1e-10 * sc * sc * sc)) return false;
  // inverse: Dinv[c][k] = cofactor[k][c] / det
  double inv[3][3];
  inv[0][0] = c00 / det;
  inv[1][0] = c01 / det;
  inv[2][0] = c02 / det;
  inv[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) / det;
  inv[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) / det;
  inv[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) / det;
  inv[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) / det;
  inv[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) / det;
  inv[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) / det;
  for (int k = 1; k < 4; ++k)
    for (int c = 0; c < 3; ++c) g[k][c] = inv[c][k - 1];
  for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
  *V = std::fabs(det) / 6.0;
  return true;
}

// Diagonal metric of the per-axis shell map x = a (b - a) / (b - |t - c|)
// (identity for |t - c| <= a): with f' its derivative and J = diag(f'),
// the transformed Laplacian carries |det J| J^-1 J^-T.  Evaluated at the
// centroid (nm).  Returns false when the centroid lies outside the shell.
bool shell_diag(const double* shell, const double cen[3], double T[3]) {
  double fp[3] = {1, 1, 1};
  if (shell) {
    for (int k = 0; k < 3; ++k) {
      double c = shell[k] / kNm, a = shell[3 + k] / kNm, b = shell[6 + k] / kNm;
      double t = std::fabs(cen[k] - c);
      if (t > a) {
        if (!(t < b)) return false;
        fp[k] = a * (b - a) / ((b - t) * (b - t));
      }
    }
  }
  T[0] = fp[1] * fp[2] / fp[0];
  T[1] = fp[0] * fp[2] / fp[1];
  T[2] = fp[0] * fp[1] / fp[2];
  return true;
}

int check_mesh(const mmsd_mesh* m, std::string* err) {
  if (!m || m->n_nodes <= 0 || m->n_tets <= 0 || !m->xyz || !m->tets || !m->tet_region) {
    *err = "mesh: missing arrays or empty mesh";
    return MMSD_E_INVALID;
  }
  if (m->n_nodes > (int64_t)INT32_MAX / 2 || m->n_tets > (int64_t)INT32_MAX / 4) {
    *err = "mesh: too large for 32-bit indices";
    return MMSD_E_INVALID;
  }
  for (int64_t i = 0; i < 4 * m->n_tets; ++i)
    if (m->tets[i] < 0 || m->tets[i] >= m->n_nodes) {
      *err = "mesh: node index out of range in tet " + std::to_string(i / 4);
      return MMSD_E_MESH;
    }
  for (int64_t i = 0; i < 3 * m->n_nodes; ++i)
    if (!std::isfinite(m->xyz[i])) {
      *err = "mesh: non-finite coordinate";
      return MMSD_E_MESH;
    }
  bool any = false;
  for (int64_t e = 0; e < m->n_tets; ++e) {
    if (m->tet_region[e] < 0) {
      *err = "mesh: negative region id";
      return MMSD_E_MESH;
    }
    any |= m->tet_region[e] > 0;
  }
  if (!any) {
    *err = "mesh: no magnetic tetrahedra";
    return MMSD_E_MESH;
  }
  return MMSD_OK;
}

struct Numbering {
  std::vector<int> mag_global, mag_of;     // magnetic ids
  std::vector<int> pot_global, pot_of;     // potential ids (magnetic first)
};

int number_nodes(const mmsd_mesh* m, Numbering* nb, std::string* err) {
  const int64_t n = m->n_nodes;
  std::vector<char> ismag(n, 0);
  for (int64_t e = 0; e < m->n_tets; ++e)
    if (m->tet_region[e] > 0)
      for (int a = 0; a < 4; ++a) ismag[m->tets[4 * e + a]] = 1;
  nb->mag_of.assign(n, -1);
  nb->mag_global.clear();
  for (int64_t g = 0; g < n; ++g)
    if (ismag[g]) {
      nb->mag_of[g] = (int)nb->mag_global.size();
      nb->mag_global.push_back((int)g);
    }
  nb->pot_of.assign(n, -1);
  nb->pot_global.clear();
  if (m->dirichlet) {
    bool anyd = false;
    for (int64_t g = 0; g < n; ++g) {
      if (m->dirichlet[g] && ismag[g]) {
        *err = "mesh: magnetic node on the Dirichlet boundary";
        return MMSD_E_MESH;
      }
      anyd |= m->dirichlet[g] != 0;
    }
    if (anyd) {
      std::vector<char> used(n, 0);
      for (int64_t i = 0; i < 4 * m->n_tets; ++i) used[m->tets[i]] = 1;
      for (int g : nb->mag_global) {
        nb->pot_of[g] = (int)nb->pot_global.size();
        nb->pot_global.push_back(g);
      }
      for (int64_t g = 0; g < n; ++g)
        if (!ismag[g] && !m->dirichlet[g] && used[g]) {
          nb->pot_of[g] = (int)nb->pot_global.size();
          nb->pot_global.push_back((int)g);
        }
    }
  }
  return MMSD_OK;
}

}  // namespace

int pattern_sizes(const mmsd_mesh* mesh, PatternSizes* out, std::string* err) {
  int st = check_mesh(mesh, err);
  if (st) return st;
  Numbering nb;
  if ((st = number_nodes(mesh, &nb, err))) return st;
  const int64_t E = mesh->n_tets;
  std::vector<char> keep(E);
  for (int64_t e = 0; e < E; ++e) keep[e] = mesh->tet_region[e] > 0;
  std::vector<int> tptr, tlst, rp, ci;
  node_tets(mesh->n_nodes, mesh->tets, E, keep, tptr, tlst);
  build_pattern(mesh->tets, nb.mag_global, tptr, tlst, nb.mag_of, rp, ci);
  out->N = (int64_t)nb.mag_global.size();
  out->nnzM = (int64_t)ci.size();
  out->Nt = (int64_t)nb.pot_global.size();
  out->nnzL = 0;
  if (out->Nt) {
    std::fill(keep.begin(), keep.end(), 1);
    node_tets(mesh->n_nodes, mesh->tets, E, keep, tptr, tlst);
    build_pattern(mesh->tets, nb.pot_global, tptr, tlst, nb.pot_of, rp, ci);
    out->nnzL = (int64_t)ci.size();
  }
  out->nnzLs = out->Nt ? sliced_entries(rp) : 0;
  return MMSD_OK;
}

int64_t sliced_entries(const std::vector<int>& rp) {
  const int64_t n = (int64_t)rp.size() - 1;
  int64_t total = 0;
  for (int64_t s0 = 0; s0 < n; s0 += 64) {
    int w = 0;
    for (int64_t i = s0; i < std::min<int64_t>(n, s0 + 64); ++i) w = std::max(w, rp[i + 1] - rp[i]);
    total += 64LL * w;
  }
  return total;
}

int assemble_material_values(Assembly* A, std::string* err, bool operators) {
  const int N = A->N;
  const int64_t Em = (int64_t)A->mregion.size();
  // every region used needs a material with a common Js; the regions'
  // lines are looked up once, into a table by region id
  double Js = -1;
  int max_region = 0;
  for (int64_t e = 0; e < Em; ++e) max_region = std::max(max_region, (int)A->mregion[e]);
  std::vector<const MatLine*> line(max_region + 1, nullptr);
  for (int64_t e = 0; e < Em; ++e) {
    const int r = A->mregion[e];
    if (line[r]) continue;
    auto it = A->mats.find(r);
    if (it == A->mats.end()) {
      *err = "no material for region " + std::to_string(r);
      return MMSD_E_INVALID;
    }
    line[r] = &it->second;
    if (Js < 0) Js = it->second.Js;
    if (it->second.Js != Js) {
      *err = "all magnetic regions must share one Js";
      return MMSD_E_INVALID;
    }
  }
  if (!(Js > 0)) {
    *err = "Js must be positive";
    return MMSD_E_INVALID;
  }
  A->Js = Js;
  A->Ms = Js / kMu0;
  A->mu0Ms2 = kMu0 * A->Ms * A->Ms;
  const double mu0Ms2 = A->mu0Ms2;
  // per-tet coefficients
  std::vector<double> kex(Em), kan(Em), uu(Em * 6);
  CompensatedSum c_an;
  for (int64_t e = 0; e < Em; ++e) {
    const MatLine& M = *line[A->mregion[e]];
    double Ve = A->mgeo[13 * e];
    kex[e] = M.A / (mu0Ms2 * kNm * kNm) * Ve;
    double un = std::sqrt(M.u[0] * M.u[0] + M.u[1] * M.u[1] + M.u[2] * M.u[2]);
    double u[3] = {M.u[0] / un, M.u[1] / un, M.u[2] / un};
    kan[e] = 0.25 * Ve * M.K1 / mu0Ms2;
    uu[6 * e + 0] = u[0] * u[0];
    uu[6 * e + 1] = u[1] * u[1];
    uu[6 * e + 2] = u[2] * u[2];
    uu[6 * e + 3] = u[0] * u[1];
    uu[6 * e + 4] = u[0] * u[2];
    uu[6 * e + 5] = u[1] * u[2];
    c_an.add(Ve * M.K1 / mu0Ms2);
  }
  A->c_an = c_an.value();
  if (!operators) return MMSD_OK;
  A->K.assign(A->mci.size(), 0.0);
  for (int k = 0; k < 6; ++k) A->Q[k].assign(N, 0.0);
  parallel_for(N, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      const int r0 = A->mrp[i], r1 = A->mrp[i + 1];
      double q[6] = {0, 0, 0, 0, 0, 0};
      for (int k = A->mnode_tets_ptr[i]; k < A->mnode_tets_ptr[i + 1]; ++k) {
        const int e = A->mnode_tets[k] >> 2, va = A->mnode_tets[k] & 3;
        const double* g = &A->mgeo[13 * (int64_t)e + 1];
        for (int vb = 0; vb < 4; ++vb) {
          int j = A->mtet[4 * (int64_t)e + vb];
          int pos = find_col(A->mci, r0, r1, j);
          double dot = g[3 * va] * g[3 * vb] + g[3 * va + 1] * g[3 * vb + 1] + g[3 * va + 2] * g[3 * vb + 2];
          A->K[pos] += kex[e] * dot;
        }
        for (int c = 0; c < 6; ++c) q[c] += kan[e] * uu[6 * (int64_t)e + c];
      }
      const double s = 2.0 / A->V[i];
      for (int k = r0; k < r1; ++k) A->K[k] *= s;
      for (int c = 0; c < 6; ++c) A->Q[c][i] = q[c] * s;
    }
  });
  return MMSD_OK;
}

int assemble(const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, Assembly* A,
             std::string* err) {
  int st = check_mesh(mesh, err);
  if (st) return st;
  Numbering nb;
  if ((st = number_nodes(mesh, &nb, err))) return st;
  const int64_t E = mesh->n_tets;
  const int32_t* tets = mesh->tets;
  A->n_nodes = mesh->n_nodes;
  A->N = (int)nb.mag_global.size();
  A->Nt = (int)nb.pot_global.size();
  A->mag_global = nb.mag_global;
  A->pot_global = nb.pot_global;
  A->mats.clear();
  for (int k = 0; k < n_mats; ++k) {
    const mmsd_material& m = mats[k];
    double un = std::sqrt(m.easy_axis[0] * m.easy_axis[0] + m.easy_axis[1] * m.easy_axis[1] +
                          m.easy_axis[2] * m.easy_axis[2]);
    if (m.region < 1 || !(un > 0) || !(m.Js_T > 0) || !(m.A_Jm >= 0) || !std::isfinite(m.K1_Jm3)) {
      *err = "invalid material for region " + std::to_string(m.region);
      return MMSD_E_INVALID;
    }
    A->mats[m.region] = MatLine{m.Js_T, m.K1_Jm3, m.A_Jm, {m.easy_axis[0], m.easy_axis[1], m.easy_axis[2]}};
  }

  // geometry of every tet (needed for L) -- validated here
  std::unique_ptr<double[]> geo(new double[13 * E]);   // every entry written below (or the mesh rejected)
  std::vector<char> bad(E, 0);
  parallel_for(E, [&](int64_t a, int64_t b) {
    for (int64_t e = a; e < b; ++e) {
      double g[4][3], V;
      if (!tet_geo(mesh->xyz, tets + 4 * e, &V, g)) {
        bad[e] = 1;
        continue;
      }
      geo[13 * e] = V;
      for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 3; ++c) geo[13 * e + 1 + 3 * k + c] = g[k][c];
    }
  });
  for (int64_t e = 0; e < E; ++e)
    if (bad[e]) {
      *err = "mesh: degenerate tetrahedron " + std::to_string(e);
      return MMSD_E_MESH;
    }

  // magnetic tets
  std::vector<char> keep(E);
  int64_t Em = 0;
  for (int64_t e = 0; e < E; ++e) Em += (keep[e] = mesh->tet_region[e] > 0);
  A->mtet.resize(4 * Em);
  A->mgeo.resize(13 * Em);
  A->mregion.resize(Em);
  std::vector<int> mag_tet_ids(Em);
  for (int64_t e = 0, k = 0; e < E; ++e)
    if (keep[e]) mag_tet_ids[k++] = (int)e;
  parallel_for(Em, [&](int64_t k0, int64_t k1) {
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t e = mag_tet_ids[k];
      for (int a = 0; a < 4; ++a) A->mtet[4 * k + a] = nb.mag_of[tets[4 * e + a]];
      std::copy(&geo[13 * e], &geo[13 * e] + 13, &A->mgeo[13 * k]);
      A->mregion[k] = mesh->tet_region[e];
    }
  });
  // magnetic node -> (magnetic tet, vertex)
  {
    std::vector<int> lt(4 * Em);
    for (int64_t i = 0; i < 4 * Em; ++i) lt[i] = A->mtet[i];
    std::vector<char> all(Em, 1);
    node_tets(A->N, lt.data(), Em, all, A->mnode_tets_ptr, A->mnode_tets);
  }
  // magnet pattern
  {
    std::vector<int> tptr, tlst;
    node_tets(mesh->n_nodes, tets, E, keep, tptr, tlst);
    build_pattern(tets, nb.mag_global, tptr, tlst, nb.mag_of, A->mrp, A->mci);
  }
  const int N = A->N;
  const int64_t nnzM = (int64_t)A->mci.size();
  // lumped volumes
  A->V.assign(N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int k = A->mnode_tets_ptr[i]; k < A->mnode_tets_ptr[i + 1]; ++k)
      A->V[i] += 0.25 * A->mgeo[13 * (int64_t)(A->mnode_tets[k] >> 2)];
  CompensatedSum vol;
  for (int i = 0; i < N; ++i) vol.add(A->V[i]);
  A->vol = vol.value();
  // potential coupling: D1 (b = D1 m) and D2 (h_d = -D2 u)
  for (int c = 0; c < 3; ++c) {
    A->D1[c].assign(nnzM, 0.0);
    A->D2[c].assign(nnzM, 0.0);
  }
  parallel_for(N, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      const int r0 = A->mrp[i], r1 = A->mrp[i + 1];
      for (int k = A->mnode_tets_ptr[i]; k < A->mnode_tets_ptr[i + 1]; ++k) {
        const int e = A->mnode_tets[k] >> 2, va = A->mnode_tets[k] & 3;
        const double q = 0.25 * A->mgeo[13 * (int64_t)e];
        const double* g = &A->mgeo[13 * (int64_t)e + 1];
        for (int vb = 0; vb < 4; ++vb) {
          int pos = find_col(A->mci, r0, r1, A->mtet[4 * (int64_t)e + vb]);
          for (int c = 0; c < 3; ++c) {
            A->D1[c][pos] += q * g[3 * va + c];
            A->D2[c][pos] += q * g[3 * vb + c];
          }
        }
      }
      const double s = 1.0 / A->V[i];
      for (int c = 0; c < 3; ++c)
        for (int k = r0; k < r1; ++k) A->D2[c][k] *= s;
    }
  });
  if ((st = assemble_material_values(A, err))) return st;

  // transformed Laplacian on the free nodes
  if (A->Nt > 0) {
    std::vector<double> T(3 * E);
    parallel_for(E, [&](int64_t a, int64_t b) {
      for (int64_t e = a; e < b; ++e) {
        double cen[3] = {0, 0, 0};
        for (int v = 0; v < 4; ++v)
          for (int c = 0; c < 3; ++c) cen[c] += 0.25 * mesh->xyz[3 * tets[4 * e + v] + c] / kNm;
        if (!shell_diag(mesh->shell, cen, &T[3 * e])) bad[e] = 1;
      }
    });
    for (int64_t e = 0; e < E; ++e)
      if (bad[e]) {
        *err = "mesh: tetrahedron outside the transformation shell";
        return MMSD_E_MESH;
      }
    std::vector<char> all(E, 1);
    std::vector<int> tptr, tlst;
    node_tets(mesh->n_nodes, tets, E, all, tptr, tlst);
    build_pattern(tets, nb.pot_global, tptr, tlst, nb.pot_of, A->lrp, A->lci);
    A->L.assign(A->lci.size(), 0.0);
    A->invd.assign(A->Nt, 0.0);
    bool badrow = false;
    parallel_for(A->Nt, [&](int64_t a, int64_t b) {
      for (int64_t r = a; r < b; ++r) {
        const int g = nb.pot_global[r];
        const int r0 = A->lrp[r], r1 = A->lrp[r + 1];
        for (int k = tptr[g]; k < tptr[g + 1]; ++k) {
          const int e = tlst[k] >> 2, va = tlst[k] & 3;
          const double Ve = geo[13 * (int64_t)e];
          const double* gr = &geo[13 * (int64_t)e + 1];
          const double* Te = &T[3 * (int64_t)e];
          for (int vb = 0; vb < 4; ++vb) {
            int col = nb.pot_of[tets[4 * (int64_t)e + vb]];
            if (col < 0) continue;
            int pos = find_col(A->lci, r0, r1, col);
            A->L[pos] += Ve * (gr[3 * va] * Te[0] * gr[3 * vb] + gr[3 * va + 1] * Te[1] * gr[3 * vb + 1] +
                               gr[3 * va + 2] * Te[2] * gr[3 * vb + 2]);
          }
        }
        int pd = find_col(A->lci, r0, r1, (int)r);
        if (pd >= r1 || A->lci[pd] != r || !(A->L[pd] > 0)) badrow = true;
        else A->invd[r] = 1.0 / A->L[pd];
      }
    });
    if (badrow) {
      *err = "mesh: potential matrix has a non-positive diagonal";
      return MMSD_E_MESH;
    }
  }
  return MMSD_OK;
}

int assemble_host_side(const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, AssemblyStructure* S,
                       std::vector<double>&& V, Assembly* A, std::string* err) {
  A->n_nodes = mesh->n_nodes;
  A->N = S->N;
  A->Nt = S->Nt;
  A->mag_global = std::move(S->mag_global);
  A->pot_global = std::move(S->pot_global);
  A->mats.clear();
  for (int k = 0; k < n_mats; ++k) {
    const mmsd_material& m = mats[k];
    A->mats[m.region] = MatLine{m.Js_T, m.K1_Jm3, m.A_Jm, {m.easy_axis[0], m.easy_axis[1], m.easy_axis[2]}};
  }
  A->mtet = std::move(S->mtet);
  A->mregion = std::move(S->mregion);
  const int64_t Em = (int64_t)A->mregion.size();
  A->mgeo.resize(13 * Em);
  std::atomic<int> bad{0};
  parallel_for(Em, [&](int64_t k0, int64_t k1) {
    for (int64_t k = k0; k < k1; ++k) {
      double g[4][3], Ve;
      if (!tet_geo(mesh->xyz, mesh->tets + 4 * (int64_t)S->mtet_mesh[k], &Ve, g)) {
        bad.store(1);
        continue;
      }
      A->mgeo[13 * k] = Ve;
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) A->mgeo[13 * k + 1 + 3 * a + c] = g[a][c];
    }
  });
  if (bad) {
    *err = "mesh: degenerate tetrahedron";
    return MMSD_E_MESH;
  }
  A->V = std::move(V);
  CompensatedSum vol;
  for (int i = 0; i < A->N; ++i) vol.add(A->V[i]);
  A->vol = vol.value();
  A->mnode_tets_ptr.clear();
  A->mnode_tets.clear();
  return assemble_material_values(A, err, /*operators=*/false);
}

void ensure_magnet_adjacency(Assembly* A) {
  if (!A->mnode_tets_ptr.empty()) return;
  const int64_t Em = (int64_t)A->mregion.size();
  std::vector<char> all(Em, 1);
  node_tets(A->N, A->mtet.data(), Em, all, A->mnode_tets_ptr, A->mnode_tets);
}

int assemble_structure(const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, AssemblyStructure* S,
                       std::string* err, bool with_patterns) {
  int st = check_mesh(mesh, err);
  if (st) return st;
  Numbering nb;
  if ((st = number_nodes(mesh, &nb, err))) return st;
  const int64_t E = mesh->n_tets;
  const int32_t* tets = mesh->tets;
  S->E = E;
  S->N = (int)nb.mag_global.size();
  S->Nt = (int)nb.pot_global.size();
  S->mag_global = std::move(nb.mag_global);
  S->pot_global = std::move(nb.pot_global);
  S->pot_of = std::move(nb.pot_of);
  std::map<int, MatLine> lines;
  for (int k = 0; k < n_mats; ++k) {
    const mmsd_material& m = mats[k];
    double un = std::sqrt(m.easy_axis[0] * m.easy_axis[0] + m.easy_axis[1] * m.easy_axis[1] +
                          m.easy_axis[2] * m.easy_axis[2]);
    if (m.region < 1 || !(un > 0) || !(m.Js_T > 0) || !(m.A_Jm >= 0) || !std::isfinite(m.K1_Jm3)) {
      *err = "invalid material for region " + std::to_string(m.region);
      return MMSD_E_INVALID;
    }
    lines[m.region] = MatLine{m.Js_T, m.K1_Jm3, m.A_Jm, {m.easy_axis[0], m.easy_axis[1], m.easy_axis[2]}};
  }
  // magnetic tets
  std::vector<char> keep(E);
  int64_t Em = 0;
  int max_region = 0;
  for (int64_t e = 0; e < E; ++e) {
    Em += (keep[e] = mesh->tet_region[e] > 0);
    max_region = std::max(max_region, (int)mesh->tet_region[e]);
  }
  S->mtet.resize(4 * Em);
  S->mtet_mesh.resize(Em);
  S->mregion.resize(Em);
  for (int64_t e = 0, k = 0; e < E; ++e)
    if (keep[e]) S->mtet_mesh[k++] = (int)e;
  parallel_for(Em, [&](int64_t k0, int64_t k1) {
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t e = S->mtet_mesh[k];
      for (int a = 0; a < 4; ++a) S->mtet[4 * k + a] = nb.mag_of[tets[4 * e + a]];
      S->mregion[k] = mesh->tet_region[e];
    }
  });
  // materials of the regions in use: one Js, factors as assemble_material_values forms them
  std::vector<char> used(max_region + 1, 0);
  for (int64_t k = 0; k < Em; ++k) used[S->mregion[k]] = 1;
  double Js = -1;
  for (int r = 1; r <= max_region; ++r) {
    if (!used[r]) continue;
    auto it = lines.find(r);
    if (it == lines.end()) {
      *err = "no material for region " + std::to_string(r);
      return MMSD_E_INVALID;
    }
    if (Js < 0) Js = it->second.Js;
    if (it->second.Js != Js) {
      *err = "all magnetic regions must share one Js";
      return MMSD_E_INVALID;
    }
  }
  S->Js = Js;
  const double Ms = Js / kMu0;
  S->mu0Ms2 = kMu0 * Ms * Ms;
  S->reg.assign(8 * (size_t)(max_region + 1), 0.0);
  for (int r = 1; r <= max_region; ++r) {
    if (!used[r]) continue;
    const MatLine& M = lines[r];
    double* t = &S->reg[8 * (size_t)r];
    t[0] = M.A / (S->mu0Ms2 * kNm * kNm);
    t[1] = M.K1;
    double un = std::sqrt(M.u[0] * M.u[0] + M.u[1] * M.u[1] + M.u[2] * M.u[2]);
    double u[3] = {M.u[0] / un, M.u[1] / un, M.u[2] / un};
    t[2] = u[0] * u[0];
    t[3] = u[1] * u[1];
    t[4] = u[2] * u[2];
    t[5] = u[0] * u[1];
    t[6] = u[0] * u[2];
    t[7] = u[1] * u[2];
  }
  if (!with_patterns) return MMSD_OK;
  {
    std::vector<char> all(Em, 1);
    node_tets(S->N, S->mtet.data(), Em, all, S->mnode_tets_ptr, S->mnode_tets);
  }
  {
    std::vector<int> tptr, tlst;
    node_tets(mesh->n_nodes, tets, E, keep, tptr, tlst);
    build_pattern(tets, S->mag_global, tptr, tlst, nb.mag_of, S->mrp, S->mci);
  }
  if (S->Nt > 0) {
    std::vector<char> all(E, 1);
    node_tets(mesh->n_nodes, tets, E, all, S->tptr, S->tlst);
    build_pattern(tets, S->pot_global, S->tptr, S->tlst, S->pot_of, S->lrp, S->lci);
  }
  return MMSD_OK;
}

}  // namespace mmsd
