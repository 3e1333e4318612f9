// CPU check of the host half of the device-side assembly: the structure
// (numbering, adjacency, patterns, per-region material table) equals what
// the full host assembly builds, and the per-row sums the device kernels
// form from it (same terms, same order, written out here in plain loops)
// reproduce the host assembly's values.  Reads a mesh written by the test.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "assemble.h"

using namespace mmsd;

static double max_rel(const std::vector<double>& a, const std::vector<double>& b) {
  double m = 0, s = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    m = std::max(m, std::fabs(a[i] - b[i]));
    s = std::max(s, std::fabs(b[i]));
  }
  return s > 0 ? m / s : m;
}

static int find(const std::vector<int>& ci, int r0, int r1, int c) {
  int lo = r0, hi = r1;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (ci[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t h[5];
  if (fread(h, 8, 5, f) != 5) return 2;
  std::vector<double> xyz(3 * h[0]), shell(9);
  std::vector<int32_t> tets(4 * h[1]), region(h[1]);
  std::vector<uint8_t> dir(h[0]);
  std::vector<double> mt(7 * h[2]);
  bool ok = fread(xyz.data(), 8, xyz.size(), f) == xyz.size() && fread(tets.data(), 4, tets.size(), f) == tets.size() &&
            fread(region.data(), 4, region.size(), f) == region.size() &&
            fread(dir.data(), 1, dir.size(), f) == dir.size() && fread(shell.data(), 8, 9, f) == 9 &&
            fread(mt.data(), 8, mt.size(), f) == mt.size();
  fclose(f);
  if (!ok) return 2;
  std::vector<mmsd_material> mats(h[2]);
  for (int64_t k = 0; k < h[2]; ++k) {
    mats[k].region = (int32_t)mt[7 * k];
    mats[k].Js_T = mt[7 * k + 1];
    mats[k].K1_Jm3 = mt[7 * k + 2];
    mats[k].A_Jm = mt[7 * k + 3];
    for (int c = 0; c < 3; ++c) mats[k].easy_axis[c] = mt[7 * k + 4 + c];
  }
  mmsd_mesh mesh{h[0], xyz.data(), h[1], tets.data(), region.data(), h[3] ? dir.data() : nullptr,
                 h[4] ? shell.data() : nullptr};
  std::string err;
  Assembly A;
  AssemblyStructure S;
  if (assemble(&mesh, mats.data(), (int)mats.size(), &A, &err) ||
      assemble_structure(&mesh, mats.data(), (int)mats.size(), &S, &err)) {
    printf("error %s\n", err.c_str());
    return 1;
  }
  const bool same = S.N == A.N && S.Nt == A.Nt && S.mag_global == A.mag_global && S.pot_global == A.pot_global &&
                    S.mrp == A.mrp && S.mci == A.mci && S.lrp == A.lrp && S.lci == A.lci && S.mtet == A.mtet &&
                    S.mregion == A.mregion && S.mnode_tets_ptr == A.mnode_tets_ptr &&
                    S.mnode_tets == A.mnode_tets && S.mu0Ms2 == A.mu0Ms2;
  printf("structure %s\n", same ? "equal" : "DIFFERENT");
  if (!same) return 1;

  // geometry as the device computes it: the host's per-tet records
  const int N = S.N;
  const int64_t nnz = (int64_t)S.mci.size(), Em = (int64_t)S.mtet_mesh.size();
  std::vector<double> Ve(Em);
  for (int64_t e = 0; e < Em; ++e) Ve[e] = A.mgeo[13 * e];
  std::vector<double> V(N, 0.0), K(nnz, 0.0), Q(6 * (size_t)N, 0.0), D1(3 * nnz, 0.0), D2(3 * nnz, 0.0);
  for (int i = 0; i < N; ++i) {
    const int r0 = S.mrp[i], r1 = S.mrp[i + 1];
    for (int k = S.mnode_tets_ptr[i]; k < S.mnode_tets_ptr[i + 1]; ++k) V[i] += 0.25 * Ve[S.mnode_tets[k] >> 2];
    double q[6] = {0, 0, 0, 0, 0, 0};
    for (int k = S.mnode_tets_ptr[i]; k < S.mnode_tets_ptr[i + 1]; ++k) {
      const int e = S.mnode_tets[k] >> 2, va = S.mnode_tets[k] & 3;
      const double* g = &A.mgeo[13 * (int64_t)e + 1];
      const double* R = &S.reg[8 * (size_t)S.mregion[e]];
      const double qv = 0.25 * Ve[e], kex = R[0] * Ve[e], kan = 0.25 * Ve[e] * R[1] / S.mu0Ms2;
      for (int vb = 0; vb < 4; ++vb) {
        const int p = find(S.mci, r0, r1, S.mtet[4 * (int64_t)e + vb]);
        for (int c = 0; c < 3; ++c) {
          D1[c * nnz + p] += qv * g[3 * va + c];
          D2[c * nnz + p] += qv * g[3 * vb + c];
        }
        const double dot = g[3 * va] * g[3 * vb] + g[3 * va + 1] * g[3 * vb + 1] + g[3 * va + 2] * g[3 * vb + 2];
        K[p] += kex * dot;
      }
      for (int c = 0; c < 6; ++c) q[c] += kan * R[2 + c];
    }
    const double s1 = 1.0 / V[i], s2 = 2.0 / V[i];
    for (int p = r0; p < r1; ++p) {
      for (int c = 0; c < 3; ++c) D2[c * nnz + p] *= s1;
      K[p] *= s2;
    }
    for (int c = 0; c < 6; ++c) Q[c * (size_t)N + i] = q[c] * s2;
  }
  std::vector<double> hD1, hD2, hQ;
  for (int c = 0; c < 3; ++c) {
    hD1.insert(hD1.end(), A.D1[c].begin(), A.D1[c].end());
    hD2.insert(hD2.end(), A.D2[c].begin(), A.D2[c].end());
  }
  for (int c = 0; c < 6; ++c) hQ.insert(hQ.end(), A.Q[c].begin(), A.Q[c].end());
  printf("rel V %.3e K %.3e D1 %.3e D2 %.3e Q %.3e\n", max_rel(V, A.V), max_rel(K, A.K), max_rel(D1, hD1),
         max_rel(D2, hD2), max_rel(Q, hQ));
  // the potential rows read the mesh's node adjacency and pot_of
  if (S.Nt > 0) {
    int64_t missing = 0;
    for (int r = 0; r < S.Nt; ++r) {
      const int g = S.pot_global[r];
      for (int k = S.tptr[g]; k < S.tptr[g + 1]; ++k) {
        const int e = S.tlst[k] >> 2;
        for (int vb = 0; vb < 4; ++vb) {
          const int col = S.pot_of[tets[4 * (int64_t)e + vb]];
          if (col < 0) continue;
          const int p = find(S.lci, S.lrp[r], S.lrp[r + 1], col);
          missing += p >= S.lrp[r + 1] || S.lci[p] != col;
        }
      }
    }
    printf("potential columns missing %lld\n", (long long)missing);
  }
  return 0;
}
