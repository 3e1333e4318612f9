// Host check of the multigrid hierarchy's algebraic identities, on which
// the device's rearranged V(1,1) cycle rests.  Reads a CSR matrix (int32 n,
// int32 nnz, rp, ci, values) from argv[1], builds the hierarchy and prints
// one line per level with the largest relative deviations:
//   rest  |R (b - A W b) - M b|, M = residual_restriction (W = wsmooth D^-1)
//   post  |xa + W (b - A xa) - (xa + W (res - (A P) x))|, xa = W b + P x,
//         res = b - A W b (the fused post-smoothing)
//   rap   |R A P - A_next| (Galerkin product against the stored next level)
// for seeded random b and x.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "amg.h"

using namespace mmsd;

static std::vector<double> spmv(const Csr& A, const std::vector<double>& x) {
  std::vector<double> y(A.nrows, 0.0);
  for (int i = 0; i < A.nrows; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) y[i] += A.v[k] * x[A.ci[k]];
  return y;
}

static double rel(const std::vector<double>& a, const std::vector<double>& b) {
  double d = 0, m = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    d = std::fmax(d, std::fabs(a[i] - b[i]));
    m = std::fmax(m, std::fabs(a[i]));
  }
  return m > 0 ? d / m : d;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int n = 0, nnz = 0;
  Csr A;
  bool ok = std::fread(&n, 4, 1, f) == 1 && std::fread(&nnz, 4, 1, f) == 1;
  if (ok) {
    A.nrows = A.ncols = n;
    A.rp.resize(n + 1);
    A.ci.resize(nnz);
    A.v.resize(nnz);
    ok = std::fread(A.rp.data(), 4, n + 1, f) == (size_t)n + 1 && std::fread(A.ci.data(), 4, nnz, f) == (size_t)nnz &&
         std::fread(A.v.data(), 8, nnz, f) == (size_t)nnz;
  }
  std::fclose(f);
  if (!ok) return 2;
  AmgHierarchy h;
  if (!amg_setup(A, AmgParams{}, &h)) return 3;
  std::mt19937_64 g(7);
  std::normal_distribution<double> N01;
  for (size_t l = 0; l < h.lv.size(); ++l) {
    const AmgLevel& L = h.lv[l];
    const int nl = L.A.nrows, nn = L.P.ncols;
    std::vector<double> b(nl), x(nn), wb(nl), res(nl), xa(nl);
    for (auto& v : b) v = N01(g);
    for (auto& v : x) v = N01(g);
    for (int i = 0; i < nl; ++i) wb[i] = L.wsmooth * L.dinv[i] * b[i];
    const std::vector<double> Awb = spmv(L.A, wb);
    for (int i = 0; i < nl; ++i) res[i] = b[i] - Awb[i];
    // restriction of the pre-smoothed residual
    const double e_rest = rel(spmv(L.R, res), spmv(residual_restriction(L), b));
    // post-smoothing, separate and fused
    const std::vector<double> Px = spmv(L.P, x), APx = spmv(L.AP, x);
    for (int i = 0; i < nl; ++i) xa[i] = wb[i] + Px[i];
    const std::vector<double> Axa = spmv(L.A, xa);
    std::vector<double> z1(nl), z2(nl);
    for (int i = 0; i < nl; ++i) {
      const double w = L.wsmooth * L.dinv[i];
      z1[i] = xa[i] + w * (b[i] - Axa[i]);
      z2[i] = xa[i] + w * (res[i] - APx[i]);
    }
    const double e_post = rel(z1, z2);
    // Galerkin product against the next level's operator
    double e_rap = 0;
    if (l + 1 < h.lv.size()) {
      const Csr& An = h.lv[l + 1].A;
      std::vector<double> y(nn);
      for (auto& v : y) v = N01(g);
      e_rap = rel(spmv(L.R, spmv(L.A, spmv(L.P, y))), spmv(An, y));
    }
    std::printf("level %zu rows %d rest %.3e post %.3e rap %.3e\n", l, nl, e_rest, e_post, e_rap);
  }
  return 0;
}
