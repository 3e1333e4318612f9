// Smoothed-aggregation AMG setup (host, C++17).
//
// Level l -> l + 1:
//   strength:   j is a strong neighbour of i if |a_ij| >= theta sqrt(|a_ii a_jj|)
//   aggregates: pass 1 takes every node whose strong neighbours are all free,
//               with those neighbours; pass 2 joins leftover nodes to a
//               neighbouring aggregate; pass 3 groups what is still left
//   tentative:  T_i,agg(i) = 1 (the constants, the Laplacian's near-kernel)
//   smoothing:  P = (I - omega D^-1 A) T on the first `smooth_levels` levels
//               (all by default), P = T below; entries of a smoothed row
//               below p_drop x its largest are dropped and the rest rescaled
//               to the row's sum.  On the 80 nm cube (p_drop 0.1): P from 7
//               to 3.0 and the next operator from 75 to 39 entries per row;
//               with the drop, smoothing every level keeps the operator
//               complexity at 1.45 and takes 56 -> 34 PCG iterations from
//               zero (polycrystal: 84 -> 34, complexity 1.46)
//   Galerkin:   A_{l+1} = P^T A P
// The coarsest operator is inverted densely (Cholesky, then the inverse).
#include "amg.h"

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <functional>
#include <map>
#include <mutex>
#include <random>
#include <thread>

namespace mmsd {

namespace {
thread_local const std::atomic<int>* t_sharing = nullptr;
}  // namespace

void share_cores(const std::atomic<int>* active) { t_sharing = active; }

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::max<unsigned>(1, std::min<unsigned>(hw ? hw : 4, 16));
  if (t_sharing) nt = std::max(1, std::min(nt, (int)(hw ? hw : 4) / std::max(1, t_sharing->load())));
  if (n < 2048) nt = 1;
  if (nt == 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t c = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t a = t * c, b = std::min(n, a + c);
    if (a < b) th.emplace_back(f, a, b);
  }
  for (auto& x : th) x.join();
}

namespace {

std::vector<double> diagonal(const Csr& A) {
  std::vector<double> d(A.nrows, 0.0);
  for (int i = 0; i < A.nrows; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) d[i] = A.v[k];
  return d;
}

// Largest eigenvalue of D^-1 A by power iteration (fixed seed).
double spectral_radius(const Csr& A, const std::vector<double>& dinv) {
  const int n = A.nrows;
  std::vector<double> x(n), y(n);
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (auto& v : x) v = U(rng);
  double lam = 1.0;
  for (int it = 0; it < 20; ++it) {
    parallel_for(n, [&](int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) {
        double s = 0;
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) s += A.v[k] * x[A.ci[k]];
        y[i] = dinv[i] * s;
      }
    });
    double nrm = 0, nx = 0;
    for (int i = 0; i < n; ++i) {
      nrm += y[i] * y[i];
      nx += x[i] * x[i];
    }
    lam = std::sqrt(nrm / nx);
    const double s = 1.0 / std::sqrt(nrm);
    for (int i = 0; i < n; ++i) x[i] = y[i] * s;
  }
  return lam;
}

// Upper bound of rho(D^-1 A) (a_ii > 0): the smaller of the Gershgorin
// bounds of D^-1 A, max_i sum_j |a_ij| / a_ii, and of the similar matrix
// D^-1/2 A D^-1/2, max_i sum_j |a_ij| / sqrt(a_ii a_jj).
double gershgorin(const Csr& A, const std::vector<double>& dinv) {
  double g1 = 0, g2 = 0;
  for (int i = 0; i < A.nrows; ++i) {
    double s1 = 0, s2 = 0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      s1 += std::fabs(A.v[k]);
      s2 += std::fabs(A.v[k]) * std::sqrt(dinv[A.ci[k]]);
    }
    g1 = std::max(g1, s1 * dinv[i]);
    g2 = std::max(g2, s2 * std::sqrt(dinv[i]));
  }
  return std::min(g1, g2);
}

int aggregate(const Csr& A, const std::vector<double>& d, double theta, std::vector<int>& agg) {
  const int n = A.nrows;
  // strength graph
  std::vector<int> sp(n + 1, 0), sc;
  sc.reserve(A.ci.size());
  for (int i = 0; i < n; ++i) {
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j != i && std::fabs(A.v[k]) >= theta * std::sqrt(std::fabs(d[i] * d[j]))) sc.push_back(j);
    }
    sp[i + 1] = (int)sc.size();
  }
  agg.assign(n, -1);
  int na = 0;
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free_nb = true;
    for (int k = sp[i]; k < sp[i + 1] && free_nb; ++k) free_nb = agg[sc[k]] < 0;
    if (!free_nb) continue;
    agg[i] = na;
    for (int k = sp[i]; k < sp[i + 1]; ++k) agg[sc[k]] = na;
    ++na;
  }
  std::vector<int> pass2(n, -1);
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    for (int k = sp[i]; k < sp[i + 1]; ++k)
      if (agg[sc[k]] >= 0) {
        pass2[i] = agg[sc[k]];
        break;
      }
  }
  for (int i = 0; i < n; ++i)
    if (agg[i] < 0 && pass2[i] >= 0) agg[i] = pass2[i];
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int k = sp[i]; k < sp[i + 1]; ++k)
      if (agg[sc[k]] < 0) agg[sc[k]] = na;
    ++na;
  }
  return na;
}

Csr transpose(const Csr& M) {
  Csr T;
  T.nrows = M.ncols;
  T.ncols = M.nrows;
  T.rp.assign(T.nrows + 1, 0);
  for (int c : M.ci) T.rp[c + 1]++;
  for (int i = 0; i < T.nrows; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(M.ci.size());
  T.v.resize(M.v.size());
  std::vector<int> fill(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < M.nrows; ++i)
    for (int k = M.rp[i]; k < M.rp[i + 1]; ++k) {
      const int pos = fill[M.ci[k]]++;
      T.ci[pos] = i;
      T.v[pos] = M.v[k];
    }
  return T;   // rows come out with ascending columns
}

// C = A B (Gustavson, rows in parallel, sorted columns).  Each thread fills
// flat buffers for its contiguous range of rows; the ranges are then laid
// end to end.
Csr spgemm(const Csr& A, const Csr& B) {
  Csr C;
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  C.rp.assign(C.nrows + 1, 0);
  struct Part {
    std::vector<int> ci;
    std::vector<double> v;
  };
  std::mutex mu;
  std::map<int64_t, Part> parts;   // by first row of the range
  parallel_for(A.nrows, [&](int64_t a, int64_t b) {
    Part part;
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int> mark(B.ncols, -1), list;
    for (int64_t i = a; i < b; ++i) {
      list.clear();
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int kk = A.ci[k];
        const double av = A.v[k];
        for (int m = B.rp[kk]; m < B.rp[kk + 1]; ++m) {
          const int j = B.ci[m];
          if (mark[j] != (int)i) {
            mark[j] = (int)i;
            acc[j] = 0.0;
            list.push_back(j);
          }
          acc[j] += av * B.v[m];
        }
      }
      std::sort(list.begin(), list.end());
      for (int j : list) {
        part.ci.push_back(j);
        part.v.push_back(acc[j]);
      }
      C.rp[i + 1] = (int)list.size();
    }
    std::lock_guard<std::mutex> g(mu);
    parts[a] = std::move(part);
  });
  for (int i = 0; i < C.nrows; ++i) C.rp[i + 1] += C.rp[i];
  C.ci.resize(C.rp.back());
  C.v.resize(C.rp.back());
  std::vector<std::thread> th;   // one copy per range (at most 16)
  for (auto& kv : parts)
    th.emplace_back([&C, &kv] {
      std::copy(kv.second.ci.begin(), kv.second.ci.end(), C.ci.begin() + C.rp[kv.first]);
      std::copy(kv.second.v.begin(), kv.second.v.end(), C.v.begin() + C.rp[kv.first]);
    });
  for (auto& t : th) t.join();
  return C;
}

// Dense SPD inverse by Cholesky (n is small).
bool dense_inverse(const Csr& A, std::vector<double>& inv) {
  const int n = A.nrows;
  std::vector<double> L((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) L[(size_t)i * n + A.ci[k]] = A.v[k];
  for (int j = 0; j < n; ++j) {
    double s = L[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0)) return false;
    const double ljj = std::sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = L[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / ljj;
    }
    for (int i = 0; i < j; ++i) L[(size_t)i * n + j] = 0.0;
  }
  // inverse column by column: L L^T x = e_c
  inv.assign((size_t)n * n, 0.0);
  std::vector<double> y(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * y[k];
      y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * inv[(size_t)k * n + c];
      inv[(size_t)i * n + c] = t / L[(size_t)i * n + i];
    }
  }
  // symmetrize against rounding
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double m = 0.5 * (inv[(size_t)i * n + j] + inv[(size_t)j * n + i]);
      inv[(size_t)i * n + j] = inv[(size_t)j * n + i] = m;
    }
  return true;
}

}  // namespace

Csr residual_restriction(const AmgLevel& L) {
  const Csr T = transpose(L.AP);   // (A P)^T: n_next x n
  const Csr& R = L.R;
  Csr M;
  M.nrows = T.nrows;
  M.ncols = T.ncols;
  M.rp.assign(M.nrows + 1, 0);
  // rows are the sorted unions of T's and R's rows: count, then fill
  auto merge = [&](int I, int* ci, double* v) {
    int a = T.rp[I], b = R.rp[I], o = 0;
    const int ae = T.rp[I + 1], be = R.rp[I + 1];
    while (a < ae || b < be) {
      const int ca = a < ae ? T.ci[a] : INT32_MAX, cb = b < be ? R.ci[b] : INT32_MAX;
      const int c = std::min(ca, cb);
      double x = 0;
      if (cb == c) x += R.v[b++];
      if (ca == c) x -= T.v[a++] * L.wsmooth * L.dinv[c];
      if (ci) {
        ci[o] = c;
        v[o] = x;
      }
      ++o;
    }
    return o;
  };
  parallel_for(M.nrows, [&](int64_t a, int64_t b) {
    for (int64_t I = a; I < b; ++I) M.rp[I + 1] = merge((int)I, nullptr, nullptr);
  });
  for (int I = 0; I < M.nrows; ++I) M.rp[I + 1] += M.rp[I];
  M.ci.resize(M.rp[M.nrows]);
  M.v.resize(M.rp[M.nrows]);
  parallel_for(M.nrows, [&](int64_t a, int64_t b) {
    for (int64_t I = a; I < b; ++I) merge((int)I, &M.ci[M.rp[I]], &M.v[M.rp[I]]);
  });
  return M;
}

bool amg_setup(Csr A0, const AmgParams& prm, AmgHierarchy* h) {
  h->lv.clear();
  const double nnz0 = (double)A0.ci.size();
  Csr A = std::move(A0);
  double nnz_total = nnz0;
  while (A.nrows > prm.coarse_max && (int)h->lv.size() < prm.max_levels) {
    AmgLevel L;
    std::vector<double> d = diagonal(A);
    L.dinv.resize(A.nrows);
    for (int i = 0; i < A.nrows; ++i) L.dinv[i] = 1.0 / d[i];
    const double rho = spectral_radius(A, L.dinv);
    L.omega = 4.0 / (3.0 * rho);
    L.wsmooth = std::min(prm.smooth_scale * L.omega, 1.9 / gershgorin(A, L.dinv));
    std::vector<int> agg;
    const int na = aggregate(A, d, prm.theta, agg);
    if (na >= (int)(0.8 * A.nrows) || na < 1) break;   // no useful coarsening
    Csr T;
    T.nrows = A.nrows;
    T.ncols = na;
    T.rp.resize(A.nrows + 1);
    T.ci.resize(A.nrows);
    T.v.assign(A.nrows, 1.0);
    for (int i = 0; i <= A.nrows; ++i) T.rp[i] = i;
    for (int i = 0; i < A.nrows; ++i) T.ci[i] = agg[i];
    if ((int)h->lv.size() < prm.smooth_levels) {
      // P = T - omega D^-1 A T
      Csr AT = spgemm(A, T);
      for (int i = 0; i < AT.nrows; ++i)
        for (int k = AT.rp[i]; k < AT.rp[i + 1]; ++k) AT.v[k] *= -L.omega * L.dinv[i];
      // add T (one entry per row, column agg[i]); each thread fills flat
      // buffers for its contiguous range of rows, laid end to end after
      Csr P;
      P.nrows = A.nrows;
      P.ncols = na;
      P.rp.assign(A.nrows + 1, 0);
      struct Part {
        std::vector<int> ci;
        std::vector<double> v;
      };
      std::mutex mu;
      std::map<int64_t, Part> parts;
      parallel_for(A.nrows, [&](int64_t a, int64_t b) {
        Part part;
        std::vector<std::pair<int, double>> r, kept;
        for (int64_t i = a; i < b; ++i) {
          r.clear();
          bool found = false;
          for (int k = AT.rp[i]; k < AT.rp[i + 1]; ++k) {
            double v = AT.v[k];
            if (AT.ci[k] == agg[i]) {
              v += 1.0;
              found = true;
            }
            r.emplace_back(AT.ci[k], v);
          }
          if (!found) {
            r.emplace_back(agg[i], 1.0);
            std::sort(r.begin(), r.end());
          }
          if (prm.p_drop > 0 && r.size() > 1) {
            // drop small entries, rescale the rest to keep the row sum (the
            // constants stay in the range of P)
            double mx = 0, sum = 0;
            for (auto& e : r) {
              mx = std::max(mx, std::fabs(e.second));
              sum += e.second;
            }
            kept.clear();
            double ksum = 0;
            for (auto& e : r)
              if (std::fabs(e.second) >= prm.p_drop * mx) {
                kept.push_back(e);
                ksum += e.second;
              }
            if (ksum != 0) {
              for (auto& e : kept) e.second *= sum / ksum;
              r.swap(kept);
            }
          }
          for (auto& e : r) {
            part.ci.push_back(e.first);
            part.v.push_back(e.second);
          }
          P.rp[i + 1] = (int)r.size();
        }
        std::lock_guard<std::mutex> g(mu);
        parts[a] = std::move(part);
      });
      for (int i = 0; i < A.nrows; ++i) P.rp[i + 1] += P.rp[i];
      P.ci.resize(P.rp.back());
      P.v.resize(P.rp.back());
      for (auto& kv : parts) {
        std::copy(kv.second.ci.begin(), kv.second.ci.end(), P.ci.begin() + P.rp[kv.first]);
        std::copy(kv.second.v.begin(), kv.second.v.end(), P.v.begin() + P.rp[kv.first]);
      }
      L.P = std::move(P);
    } else {
      L.P = std::move(T);
    }
    L.R = transpose(L.P);
    L.AP = spgemm(A, L.P);
    Csr Ac = spgemm(L.R, L.AP);
    L.A = std::move(A);
    h->lv.push_back(std::move(L));
    A = std::move(Ac);
    nnz_total += (double)A.ci.size();
  }
  if (h->lv.empty() || A.nrows > 4 * prm.coarse_max + 2000) {
    h->lv.clear();
    return false;
  }
  h->nc = A.nrows;
  if (!dense_inverse(A, h->Ainv)) {
    h->lv.clear();
    return false;
  }
  h->complexity = nnz_total / nnz0;
  return true;
}

}  // namespace mmsd
