// Host check of the multigrid hierarchy's algebraic identities, on which
// the device's rearranged V(1,1) cycle rests.  Reads a CSR matrix (int32 n,
// int32 nnz, rp, ci, values) from argv[1], builds the hierarchy and prints
// one line per level with the largest relative deviations:
//   rest  |R (b - A W b) - M b|, M = residual_restriction (W = wsmooth D^-1)
//   post  |xa + W (b - A xa) - (xa + W (res - (A P) x))|, xa = W b + P x,
//         res = b - A W b (the fused post-smoothing)
//   rap   |R A P - A_next| (Galerkin product against the stored next level)
// for seeded random b and x, and the smoother's damping on that level:
//   wg    w g, g the Gershgorin bound of D^-1 A or of D^-1/2 A D^-1/2,
//         whichever is smaller, recomputed here from A's own diagonal
//   wlam  w lambda_max(D^-1 A), lambda from 300 power iterations on the
//         symmetric scaling D^-1/2 A D^-1/2 (its Rayleigh quotient)
// with w = wsmooth; damped Jacobi on an SPD matrix converges iff w lambda < 2.
// Then one line for the whole cycle, V(1,1) from zero written out plainly
// (damped Jacobi before and after, Galerkin coarse correction, the dense
// inverse on the coarsest level), which the CG needs symmetric positive
// definite:
//   coarse  |Ainv (R A P) y - y| / |y| on the last level
//   sym     largest |y.V x - x.V y| / |y| |V x| over seeded pairs
//   pd      smallest x.V x / x.x over seeded x (must be > 0)
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

// Largest eigenvalue of D^-1 A for SPD A, by power iteration on the
// similar symmetric matrix D^-1/2 A D^-1/2.
static double lambda_max(const Csr& A, std::mt19937_64& g) {
  const int n = A.nrows;
  std::vector<double> s(n, 0.0), x(n), y(n);
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) s[i] = 1.0 / std::sqrt(A.v[k]);
  std::normal_distribution<double> N01;
  for (auto& v : x) v = N01(g);
  double lam = 0;
  for (int it = 0; it < 300; ++it) {
    double nx = 0;
    for (double v : x) nx += v * v;
    nx = std::sqrt(nx);
    for (auto& v : x) v /= nx;
    for (int i = 0; i < n; ++i) {
      double acc = 0;
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) acc += A.v[k] * s[A.ci[k]] * x[A.ci[k]];
      y[i] = s[i] * acc;
    }
    lam = 0;
    for (int i = 0; i < n; ++i) lam += x[i] * y[i];
    x.swap(y);
  }
  return lam;
}

// Smaller of the Gershgorin bounds of D^-1 A (row sums of |a_ij| / a_ii) and
// of D^-1/2 A D^-1/2 (row sums of |a_ij| / sqrt(a_ii a_jj)).
static double gershgorin_bound(const Csr& A) {
  const int n = A.nrows;
  std::vector<double> d(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) d[i] = A.v[k];
  double g1 = 0, g2 = 0;
  for (int i = 0; i < n; ++i) {
    double r1 = 0, r2 = 0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      r1 += std::fabs(A.v[k]) / d[i];
      r2 += std::fabs(A.v[k]) / std::sqrt(d[i] * d[A.ci[k]]);
    }
    g1 = std::fmax(g1, r1);
    g2 = std::fmax(g2, r2);
  }
  return std::fmin(g1, g2);
}

// One V(1,1) cycle from zero on level l.
static std::vector<double> vcycle(const AmgHierarchy& h, size_t l, const std::vector<double>& b) {
  const AmgLevel& L = h.lv[l];
  const int n = L.A.nrows;
  std::vector<double> x(n), r(n);
  for (int i = 0; i < n; ++i) x[i] = L.wsmooth * L.dinv[i] * b[i];
  std::vector<double> Ax = spmv(L.A, x);
  for (int i = 0; i < n; ++i) r[i] = b[i] - Ax[i];
  const std::vector<double> bc = spmv(L.R, r);
  std::vector<double> xc;
  if (l + 1 < h.lv.size()) {
    xc = vcycle(h, l + 1, bc);
  } else {
    xc.assign(h.nc, 0.0);
    for (int I = 0; I < h.nc; ++I)
      for (int K = 0; K < h.nc; ++K) xc[I] += h.Ainv[(size_t)I * h.nc + K] * bc[K];
  }
  const std::vector<double> Pxc = spmv(L.P, xc);
  for (int i = 0; i < n; ++i) x[i] += Pxc[i];
  Ax = spmv(L.A, x);
  for (int i = 0; i < n; ++i) x[i] += L.wsmooth * L.dinv[i] * (b[i] - Ax[i]);
  return x;
}

static double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
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
    const double wg = L.wsmooth * gershgorin_bound(L.A), wlam = L.wsmooth * lambda_max(L.A, g);
    std::printf("level %zu rows %d rest %.3e post %.3e rap %.3e wg %.6f wlam %.6f\n", l, nl, e_rest, e_post, e_rap,
                wg, wlam);
  }
  {
    // the dense inverse against the coarsest Galerkin operator
    const AmgLevel& Ll = h.lv.back();
    std::vector<double> y(h.nc), z(h.nc, 0.0);
    for (auto& v : y) v = N01(g);
    const std::vector<double> Ay = spmv(Ll.R, spmv(Ll.A, spmv(Ll.P, y)));
    for (int I = 0; I < h.nc; ++I)
      for (int K = 0; K < h.nc; ++K) z[I] += h.Ainv[(size_t)I * h.nc + K] * Ay[K];
    const double e_coarse = rel(z, y);
    // the whole cycle: symmetric, positive definite
    const int n0 = h.lv[0].A.nrows;
    double asym = 0, pd = 1e300;
    for (int t = 0; t < 4; ++t) {
      std::vector<double> x(n0), y0(n0);
      for (auto& v : x) v = N01(g);
      for (auto& v : y0) v = N01(g);
      const std::vector<double> Vx = vcycle(h, 0, x), Vy = vcycle(h, 0, y0);
      asym = std::fmax(asym, std::fabs(dot(y0, Vx) - dot(x, Vy)) / std::sqrt(dot(y0, y0) * dot(Vx, Vx)));
      pd = std::fmin(pd, dot(x, Vx) / dot(x, x));
    }
    std::printf("cycle coarse %.3e sym %.3e pd %.6e\n", e_coarse, asym, pd);
  }
  return 0;
}
