// C ABI of the minimizer: contexts, problem upload, device-driven
// minimization runs, hysteresis continuation, batched runs, checkpoints and
// kernel timing.  All device work goes through the step kernel; the host
// only arms a run and polls a small control block (one batch of launches of
// lookahead), so no host round trip sits between phases.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "runtime.h"

using namespace mmsd;

namespace mmsd {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? MMSD_E_NOMEM : MMSD_E_HIP;
}

namespace {

constexpr double kNmCube = 1e-27;

int invalid(const std::string& m) {
  set_error(m);
  return MMSD_E_INVALID;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Layout of one problem's device arena.
struct Layout {
  size_t mrp, mci, K, D1[3], D2[3], Q[6], V, m[2][3], H[2][3], h[3], mh[2];
  size_t lso, lsc, lsv, lsum, u[3], p, rec[2];
  size_t part, ctrl, prob, blk, btab;
  size_t snap[2][2];
  size_t total;
};

int blocks_for(int64_t rows, int lpr, int max_blocks) {
  const int64_t rpp = kBlock / lpr;
  int64_t g = (rows + rpp - 1) / rpp;
  g = std::max<int64_t>(8, std::min<int64_t>(g, max_blocks));
  return (int)((g + 7) / 8 * 8);
}

Layout make_layout(int64_t N, int64_t nnzM, int64_t Nt, int64_t nnzLs, size_t s) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.mrp = take(4 * (N + 1));
  L.mci = take(4 * nnzM);
  L.K = take(s * nnzM);
  for (int c = 0; c < 3; ++c) L.D1[c] = take(s * nnzM);
  for (int c = 0; c < 3; ++c) L.D2[c] = take(s * nnzM);
  for (int c = 0; c < 6; ++c) L.Q[c] = take(s * N);
  L.V = take(s * N);
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < 3; ++c) L.m[k][c] = take(s * N);
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < 3; ++c) L.H[k][c] = take(s * N);
  for (int c = 0; c < 3; ++c) L.h[c] = take(s * N);
  for (int k = 0; k < 2; ++k) L.mh[k] = take(s * N);
  L.lso = take(4 * ((Nt + 63) / 64 + 1));
  L.lsc = take(4 * nnzLs);
  L.lsv = take(s * nnzLs);
  L.lsum = take(s * Nt);
  for (int k = 0; k < 3; ++k) L.u[k] = take(s * Nt);
  L.p = take(s * Nt);
  for (int k = 0; k < 2; ++k) L.rec[k] = take(4 * s * Nt);
  L.part = take(8 * 2 * (size_t)kMaxBlocks * kNPart);   // G may change between runs
  L.ctrl = take(2 * sizeof(Ctrl));
  L.prob = take(sizeof(Prob<double>));
  L.blk = take(8);
  L.btab = take(8 * kByteSlots);
  for (int k = 0; k < 2; ++k) {
    L.snap[k][0] = take(s * 3 * N);
    L.snap[k][1] = take(s * std::max<int64_t>(Nt, 1));
  }
  L.total = o;
  return L;
}

template <typename real>
int upload_vec(hipStream_t st, char* dst, const std::vector<double>& v) {
  if (v.empty()) return MMSD_OK;
  if constexpr (sizeof(real) == sizeof(double)) {
    MMSD_HIP(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st));
    MMSD_HIP(hipStreamSynchronize(st));
  } else {
    std::vector<float> f(v.begin(), v.end());
    MMSD_HIP(hipMemcpyAsync(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, st));
    MMSD_HIP(hipStreamSynchronize(st));
  }
  return MMSD_OK;
}

int upload_int(hipStream_t st, char* dst, const std::vector<int>& v) {
  if (v.empty()) return MMSD_OK;
  MMSD_HIP(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, st));
  MMSD_HIP(hipStreamSynchronize(st));
  return MMSD_OK;
}

template <typename real>
Prob<real>& desc_of(mmsd_problem p) {
  return *reinterpret_cast<Prob<real>*>(p->desc);
}

// Lanes per row W (4, 8, 16 or 32) for a multigrid matrix swept in CSR.  A
// block pass covers 512 / W rows; a lane loads 8 entries per batch (4 with
// 4 lanes).  Rows of more than 16 entries on average take 8 lanes (64
// entries per batch), more than 64 take 16, shorter ones 4.  A small matrix
// whose rows all fit one pass of the 512 blocks of a full-GPU launch at 32
// lanes (at most 8192 rows) takes 32 lanes when its rows are long: that
// spreads its few rows over many more blocks, and a row of up to 256
// entries is one batch.  The coarse levels are latency-bound (each sweep a
// chain of dependent loads): measured 1-1.5 us faster per sweep than 8
// lanes.
constexpr int64_t kSmallRows = 512 * (kBlock / 32);
int row_lanes(const Csr& M) {
  const double avg = M.nrows ? (double)M.ci.size() / M.nrows : 0.0;
  if (avg > 16 && M.nrows <= kSmallRows) return 32;
  return avg > 64 ? 16 : avg > 16 ? 8 : 4;
}
// Block passes of a CSR sweep of n rows at W lanes per row over g blocks.
static int64_t sweep_passes(int64_t n, int64_t g, int W) {
  const int64_t rpp = kBlock / W, c = (n + g - 1) / g;
  return (c + rpp - 1) / rpp;
}

// Latency cost of a sweep of matrix M (rows of avg entries) at W lanes per
// row (W = 1: sliced, one thread per row) over g blocks, in units of one
// dependent round trip: each block pass loads the row start, then per batch
// the entries and their gathers (8 entries per lane per batch at 8 or more
// lanes, 4 otherwise), then stores.
static int64_t sweep_cost(int64_t n, double avg, int64_t g, int W) {
  const double per_batch = W == 1 ? 4.0 : W == 4 ? 16.0 : 8.0 * W;
  const int64_t batches = std::max<int64_t>(1, (int64_t)std::ceil(avg / per_batch));
  return sweep_passes(n, g, W) * (batches + 1);
}

// Lanes per row of a CSR sweep: the default's (row_lanes) unless 4 or 8
// lanes cost fewer round trips over a full launch's 512 blocks (the 39k-row
// level of the 80 nm cube, rows of ~20 entries: one block pass at 4 lanes
// against two at 8).
static int model_lanes(const Csr& R) {
  const double avg = R.nrows ? (double)R.ci.size() / R.nrows : 0.0;
  int best = row_lanes(R);
  int64_t cost = sweep_cost(R.nrows, avg, 512, best);
  for (int W : {4, 8}) {
    const int64_t c = sweep_cost(R.nrows, avg, 512, W);
    if (c < cost) {
      cost = c;
      best = W;
    }
  }
  return best;
}

// Shape of a DOWN launch that also restricts (levels >= 1), for the 512
// blocks of a full-GPU launch: the split of the blocks between A's rows (nA
// rows of avgA entries at wa lanes) and M's, and M's lanes per row, that
// minimize the slower part's cost (on ties: the most blocks for M, then
// the cheapest M sweep; measured 1-1.5 us faster on the coarse levels than
// the fewest).  The fusion is kept (m_blocks > 0) when
// that cost is below the two separate sweeps' plus one launch (counted as
// 2 round trips): on coarse, latency-bound levels it removes a launch; on a
// large level, M (about 5x R's entries) would cost more than it saves.
static void fused_shape(int64_t nA, double avgA, int wa, int64_t nR, double avgR, int wr, const Csr& M, int& wm,
                        int& m_blocks) {
  const double avgM = M.nrows ? (double)M.ci.size() / M.nrows : 0.0;
  const int64_t separate = sweep_cost(nA, avgA, 512, wa) + sweep_cost(nR, avgR, 512, wr) + 2;
  int64_t best = INT64_MAX;
  wm = 4;
  m_blocks = 0;
  int64_t best_m = INT64_MAX;
  for (int64_t gd = 8; gd <= 504; gd += 8) {   // ties: the largest share for M, then M's cheapest lanes
    const int64_t ca = sweep_cost(nA, avgA, gd, wa);
    for (int W : {4, 8, 16, 32}) {
      const int64_t cm = sweep_cost(M.nrows, avgM, 512 - gd, W), c = std::max(ca, cm);
      if (c < best || (c == best && 512 - gd > m_blocks) || (c == best && 512 - gd == m_blocks && cm < best_m)) {
        best = c;
        best_m = cm;
        wm = W;
        m_blocks = (int)(512 - gd);
      }
    }
  }
  if (best >= separate) m_blocks = 0;
}

// Shape of the last DOWN when it also forms the coarsest solution (Ainv M
// folded in): the dense rows of Ainv M take one block each per pass (the
// whole block streams a row), so the split of the 512 blocks and A's lanes
// per row are chosen together for the fewest round trips of the slower
// part (on ties: the most blocks for the dense rows).  On the 80 nm cube
// this gives each of the 384 dense rows a block of its own, A at 16 lanes.
static void folded_shape(int64_t nA, double avgA, int64_t nc, int& wa, int& m_blocks) {
  int64_t best = INT64_MAX;
  for (int64_t gd = 8; gd <= 504; gd += 8) {
    const int64_t gm = 512 - gd, cm = 2 * ((nc + gm - 1) / gm);
    for (int W : {4, 8, 16, 32}) {
      const int64_t c = std::max(sweep_cost(nA, avgA, gd, W), cm);
      if (c < best || (c == best && gm > m_blocks)) {
        best = c;
        wa = W;
        m_blocks = (int)gm;
      }
    }
  }
}

// Largest dense Ainv M (coarsest size x last level's rows) folded into the
// last DOWN.
constexpr double kMaxFoldedBytes = 64.0 * (1 << 20);

// Average row length up to which a matrix with many rows is sliced.
constexpr size_t kWideRow = 24;
// Rows from which a multigrid matrix with short rows (at most kWideRow on
// average) is held in the sliced layout (no CSR copy) and swept one row per
// thread (enough wavefronts to fill the GPU); long rows keep their lanes per
// row (row_lanes), which measured faster.
constexpr int kSlicedRows = 65536;

// 64-row sliced layout of a CSR matrix: slice s holds rows 64s..64s+63,
// entry k of row i at so[s] + 64 k + (i mod 64); short rows are padded with
// their own column (clamped to the column range) and a zero value.  Entry
// k's value is v[stride k + off] (one value of an interleaved array).
// Slices are built in parallel.
struct Sliced {
  std::vector<int> so, sc;
  std::vector<double> sv;
  std::vector<int> order;   // row at each position (empty: position = row)
};

// Rows sorted by length, longest first, inside windows of kOrderWindow rows
// (8 slices): a slice is as wide as its longest row, and the multigrid's
// matrices mix row lengths (aggregates of 5-47 fine nodes, rows of A P next
// to aggregate boundaries), so that sorting cuts the padding (polycrystal:
// R_0 1.34x -> 1.06x its entries, A P 1.16x -> 1.03x) while rows stay
// inside their neighbourhood for the gathers and the XCD chunks.
constexpr int kOrderWindow = 512;
std::vector<int> window_order(const std::vector<int>& len) {
  const int64_t n = (int64_t)len.size();
  std::vector<int> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int)i;
  parallel_for((n + kOrderWindow - 1) / kOrderWindow, [&](int64_t a, int64_t b) {
    for (int64_t w = a; w < b; ++w) {
      auto first = order.begin() + w * kOrderWindow;
      auto last = order.begin() + std::min<int64_t>(n, (w + 1) * kOrderWindow);
      std::stable_sort(first, last, [&](int x, int y) { return len[x] > len[y]; });
    }
  });
  return order;
}
// Offsets of the 64-row slices of a CSR pattern: slice s starts at so[s]
// and holds 64 x (its longest row) entries.
std::vector<int> slice_offsets(const std::vector<int>& rp) {
  const int64_t n = (int64_t)rp.size() - 1, ns = (n + 63) / 64;
  std::vector<int> so(ns + 1, 0);
  parallel_for(ns, [&](int64_t a, int64_t b) {
    for (int64_t sl = a; sl < b; ++sl) {
      int w = 0;
      for (int64_t i = 64 * sl; i < std::min<int64_t>(n, 64 * sl + 64); ++i) w = std::max(w, rp[i + 1] - rp[i]);
      so[sl + 1] = 64 * w;
    }
  });
  for (int64_t sl = 0; sl < ns; ++sl) so[sl + 1] += so[sl];
  return so;
}

Sliced make_sliced(const std::vector<int>& rp, const std::vector<int>& ci, const std::vector<double>& v,
                   int ncols, int stride = 1, int off = 0, bool ordered = false) {
  const int64_t n = (int64_t)rp.size() - 1, ns = (n + 63) / 64;
  Sliced S;
  if (ordered) {
    std::vector<int> len(n);
    for (int64_t i = 0; i < n; ++i) len[i] = rp[i + 1] - rp[i];
    S.order = window_order(len);
    std::vector<int> rpo(n + 1, 0);   // row starts of the rows in position order (lengths only matter)
    for (int64_t q = 0; q < n; ++q) rpo[q + 1] = rpo[q] + len[S.order[q]];
    S.so = slice_offsets(rpo);
  } else {
    S.so = slice_offsets(rp);
  }
  S.sc.assign(S.so[ns], 0);
  S.sv.assign(S.so[ns], 0.0);
  parallel_for(ns, [&](int64_t a, int64_t b) {
    for (int64_t sl = a; sl < b; ++sl) {
      const int w = (S.so[sl + 1] - S.so[sl]) / 64;
      for (int r = 0; r < 64; ++r) {
        const int64_t pos = 64 * sl + r;
        const int64_t i = pos < n && ordered ? S.order[pos] : pos;
        const int len = pos < n ? rp[i + 1] - rp[i] : 0;
        for (int k = 0; k < w; ++k) {
          const int64_t q = S.so[sl] + 64LL * k + r;
          if (k < len) {
            S.sc[q] = ci[rp[i] + k];
            S.sv[q] = v[(size_t)stride * (rp[i] + k) + off];
          } else {
            S.sc[q] = (int)std::min<int64_t>(i, ncols - 1);
          }
        }
      }
    }
  });
  return S;
}

// The matrix the fused prolongation and post-smoothing sweeps: the union of
// the patterns of A P and P (P's lies inside A P's when A's diagonal is
// stored) with the value pairs {(A P)_ik, P_ik}, two values per entry in v.
// Each row lists P's columns first (front[i] of them, P's whole row), then
// the others, each part by ascending column.  Rows are built in parallel.
Csr fused_q(const Csr& AP, const Csr& P, std::vector<int>& front) {
  Csr Q;
  const int n = AP.nrows;
  Q.nrows = n;
  Q.ncols = AP.ncols;
  Q.rp.assign(n + 1, 0);
  front.assign(n, 0);
  // row lengths: |AP row| + P columns missing from it (rows sorted by column)
  parallel_for(n, [&](int64_t a0, int64_t b0) {
    for (int64_t i = a0; i < b0; ++i) {
      int a = AP.rp[i], extra = 0;
      for (int b = P.rp[i]; b < P.rp[i + 1]; ++b) {
        while (a < AP.rp[i + 1] && AP.ci[a] < P.ci[b]) ++a;
        if (a == AP.rp[i + 1] || AP.ci[a] != P.ci[b]) ++extra;
      }
      Q.rp[i + 1] = AP.rp[i + 1] - AP.rp[i] + extra;
      front[i] = P.rp[i + 1] - P.rp[i];
    }
  });
  for (int i = 0; i < n; ++i) Q.rp[i + 1] += Q.rp[i];
  Q.ci.resize(Q.rp[n]);
  Q.v.resize(2 * (size_t)Q.rp[n]);
  parallel_for(n, [&](int64_t a0, int64_t b0) {
    for (int64_t i = a0; i < b0; ++i) {
      int o = Q.rp[i];
      // P's columns, with the (A P) value where A P has the column
      int a = AP.rp[i];
      for (int b = P.rp[i]; b < P.rp[i + 1]; ++b, ++o) {
        while (a < AP.rp[i + 1] && AP.ci[a] < P.ci[b]) ++a;
        Q.ci[o] = P.ci[b];
        Q.v[2 * (size_t)o] = (a < AP.rp[i + 1] && AP.ci[a] == P.ci[b]) ? AP.v[a] : 0.0;
        Q.v[2 * (size_t)o + 1] = P.v[b];
      }
      // then A P's other columns
      int b = P.rp[i];
      for (a = AP.rp[i]; a < AP.rp[i + 1]; ++a) {
        while (b < P.rp[i + 1] && P.ci[b] < AP.ci[a]) ++b;
        if (b < P.rp[i + 1] && P.ci[b] == AP.ci[a]) continue;
        Q.ci[o] = AP.ci[a];
        Q.v[2 * (size_t)o] = AP.v[a];
        Q.v[2 * (size_t)o + 1] = 0.0;
        ++o;
      }
    }
  });
  return Q;
}

// The sliced form of Q, built from A P and P directly: the (A P) values over
// Q's pattern (rows ordered as in fused_q: P's columns first), and the P
// values of the row fronts as a sliced matrix of their own (same 64-row
// slices, entry k of row i at po[s] + 64 k + i mod 64, zero-padded).
// nnz receives Q's entry count.  Slices are built in parallel.
struct SlicedQ {
  Sliced ap;
  std::vector<int> po;
  std::vector<double> pv;
};
SlicedQ make_sliced_q(const Csr& AP, const Csr& P, int64_t& nnz, bool ordered = false) {
  const int64_t n = AP.nrows, ns = (n + 63) / 64;
  std::vector<int> len(n), front(n);
  parallel_for(n, [&](int64_t a0, int64_t b0) {
    for (int64_t i = a0; i < b0; ++i) {
      int a = AP.rp[i], extra = 0;
      for (int b = P.rp[i]; b < P.rp[i + 1]; ++b) {
        while (a < AP.rp[i + 1] && AP.ci[a] < P.ci[b]) ++a;
        if (a == AP.rp[i + 1] || AP.ci[a] != P.ci[b]) ++extra;
      }
      len[i] = AP.rp[i + 1] - AP.rp[i] + extra;
      front[i] = P.rp[i + 1] - P.rp[i];
    }
  });
  nnz = 0;
  for (int64_t i = 0; i < n; ++i) nnz += len[i];
  SlicedQ S;
  if (ordered) S.ap.order = window_order(len);
  auto row_of = [&](int64_t pos) { return ordered ? (int64_t)S.ap.order[pos] : pos; };
  S.ap.so.assign(ns + 1, 0);
  S.po.assign(ns + 1, 0);
  parallel_for(ns, [&](int64_t a, int64_t b) {
    for (int64_t sl = a; sl < b; ++sl) {
      int w = 0, wp = 0;
      for (int64_t q = 64 * sl; q < std::min<int64_t>(n, 64 * sl + 64); ++q) {
        w = std::max(w, len[row_of(q)]);
        wp = std::max(wp, front[row_of(q)]);
      }
      S.ap.so[sl + 1] = 64 * w;
      S.po[sl + 1] = 64 * wp;
    }
  });
  for (int64_t sl = 0; sl < ns; ++sl) {
    S.ap.so[sl + 1] += S.ap.so[sl];
    S.po[sl + 1] += S.po[sl];
  }
  S.ap.sc.assign(S.ap.so[ns], 0);
  S.ap.sv.assign(S.ap.so[ns], 0.0);
  S.pv.assign(S.po[ns], 0.0);
  parallel_for(ns, [&](int64_t a0, int64_t b0) {
    for (int64_t sl = a0; sl < b0; ++sl) {
      const int w = (S.ap.so[sl + 1] - S.ap.so[sl]) / 64;
      for (int r = 0; r < 64; ++r) {
        const int64_t pos = 64 * sl + r;
        const int64_t i = pos < n ? row_of(pos) : pos;
        auto at = [&](int k) { return S.ap.so[sl] + 64LL * k + r; };
        int k = 0;
        if (pos < n) {
          int a = AP.rp[i];
          for (int b = P.rp[i]; b < P.rp[i + 1]; ++b, ++k) {   // P's columns
            while (a < AP.rp[i + 1] && AP.ci[a] < P.ci[b]) ++a;
            S.ap.sc[at(k)] = P.ci[b];
            S.ap.sv[at(k)] = (a < AP.rp[i + 1] && AP.ci[a] == P.ci[b]) ? AP.v[a] : 0.0;
            S.pv[S.po[sl] + 64LL * k + r] = P.v[b];
          }
          int b = P.rp[i];
          for (a = AP.rp[i]; a < AP.rp[i + 1]; ++a) {   // A P's other columns
            while (b < P.rp[i + 1] && P.ci[b] < AP.ci[a]) ++b;
            if (b < P.rp[i + 1] && P.ci[b] == AP.ci[a]) continue;
            S.ap.sc[at(k)] = AP.ci[a];
            S.ap.sv[at(k)] = AP.v[a];
            ++k;
          }
        }
        for (; k < w; ++k) S.ap.sc[at(k)] = (int)std::min<int64_t>(i, AP.ncols - 1);   // padding
      }
    }
  });
  return S;
}

// Algorithmic bytes per executed phase: every matrix entry, index and
// row-local vector value moved once; gathered neighbour values counted as
// cache hits.
template <typename real>
void bytes_model(mmsd_problem p) {
  const Assembly& A = p->A;
  const double s = sizeof(real), N = A.N, Nt = A.Nt, zM = (double)A.mci.size(), zL = (double)A.lci.size();
  const double spmvL = 4 * (Nt + 1) + 4 * zL + s * zL;
  double* b = p->btab;
  for (int k = 0; k < kByteSlots; ++k) b[k] = 0;
  b[PH_PREP] = 4 * (N + 1) + 4 * zM + 3 * s * zM + 9 * s * N + spmvL + 3 * s * Nt;   // trial m, b = D1 m, r = b - L u
                                                                                       // (and the working u written)
  if (p->precision == MMSD_MIXED) b[PH_PREP] += s * Nt;   // row sums of L
  b[PH_CG0] = spmvL + 5 * s * Nt;                                                       // w = L D^-1 r
  b[PH_CG] = spmvL + 12 * s * Nt;                                                       // one CG iteration
  b[PH_FIELD] = 4 * (N + 1) + 4 * zM + 4 * s * zM + s * N * (3 + 1 + 6 + 1 + 6 + 3);
  if (p->precision == MMSD_MIXED) b[PH_FIELD] += 2 * s * N;   // m.h of the accepted state in, the trial's out
  b[PH_PCG_A] = spmvL + 7 * s * Nt;        // {z, p}, r, wd in; q, {wd r, wd q} out
  b[PH_PCG_B] = spmvL + 13 * s * Nt;       // {wd r, wd q}, r, q, {z, p}, u in; {z, p}, r, u, res out
  if (p->has_amg) {
    const auto& H = p->amg;
    for (size_t l = 0; l < H.lv.size(); ++l) {
      const AmgLevel& L = H.lv[l];
      const double n = L.A.nrows, nn = L.P.ncols;
      const double zA = (double)L.A.ci.size(), zP = (double)L.P.ci.size(), zQ = (double)p->amg_q_nnz[l];
      const double spA = 4 * (n + 1) + (4 + s) * zA, spR = 4 * (nn + 1) + (4 + s) * zP;
      // Q: CSR with value pairs, or sliced with the (A P) values and P's
      // values of the row fronts
      const double spQ = p->amg_q_sliced[l] ? 4 * (n + 1) + (4 + s) * zQ + s * (double)L.P.ci.size()
                                            : 4 * (n + 1) + (4 + 2 * s) * zQ;
      b[byte_slot(PH_MG, MG_DOWN, (int)l)] = spA + 3 * s * n;     // b, wd in; res out
      b[byte_slot(PH_MG, MG_REST, (int)l)] = spR + s * n + s * nn;   // res in; b out
      if (l + 1 < H.lv.size()) b[byte_slot(PH_MG, MG_REST, (int)l)] += 2 * s * nn;   // wd in; wd b out
      if (p->amg_folded && l + 1 == H.lv.size())   // DOWN also solves: dense Ainv M rows, x_c out
        b[byte_slot(PH_MG, MG_DOWN, (int)l)] += s * nn * n + s * nn;
      else if (p->amg_m_nnz[l] > 0)   // DOWN also restricts: M rows, b_{l+1} out (and wd in, wd b out)
        b[byte_slot(PH_MG, MG_DOWN, (int)l)] += 4 * (nn + 1) + (4 + s) * (double)p->amg_m_nnz[l] + s * nn +
                                               (l + 1 < H.lv.size() ? 2 * s * nn : 0.0);
      b[byte_slot(PH_MG, MG_POST, (int)l)] = spQ + s * nn + 4 * s * n;   // x_{l+1}, b, wd, res in; xb out
      if (l == 0) b[byte_slot(PH_MG, MG_POST, 0)] += 2 * s * n;     // p carried over into the {z, p} records
    }
    b[byte_slot(PH_MG, MG_SOLVE, 0)] = s * (double)H.nc * (H.nc + 2);
  }
  p->phase_bytes_h = 3 * s * N;
  p->prep_bytes_nodemag = 9 * s * N;
}

// Upload the multigrid hierarchy into its own arena and fill the level
// descriptors and the level-0 CG vectors of the descriptor.
template <typename real>
int build_amg(mmsd_problem p) {
  mmsd_ctx c = p->ctx;
  const AmgHierarchy& H = p->amg;
  const int nl = (int)H.lv.size();
  const size_t s = sizeof(real);
  const int64_t Nt = p->A.Nt;
  // layout
  std::vector<size_t> off;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    off.push_back(at);
    return at;
  };
  struct LvOff { size_t arp, aci, av, wd, qrp, qci, qv, qpo, qpv, rrp, rci, rv, mrp, mci, mv, b, wb, res, xb, sl[3][4]; };
  std::vector<LvOff> lo(nl);
  // the fused prolongation / post-smoothing matrices (two values per entry),
  // and on levels >= 1 the restriction M = R (I - A wd) that DOWN sweeps too
  std::vector<Csr> Q(nl), M(nl);
  std::vector<std::vector<int>> qfront(nl);
  std::vector<SlicedQ> sq(nl);
  // every matrix sliced, as on the largest meshes (a context option for tests)
  const bool slice_all = (c->vcycle & MMSD_VC_SLICE_ALL) != 0;
  p->amg_q_nnz.assign(nl, 0);
  p->amg_m_nnz.assign(nl, 0);
  p->amg_q_sliced.assign(nl, 0);
  for (int l = 0; l < nl; ++l) {
    const AmgLevel& L = H.lv[l];
    // Q's rows average about A P's entries: sliced by the same rule as A, R
    const bool q_sliced = slice_all || (L.AP.nrows >= kSlicedRows && L.AP.ci.size() <= kWideRow * (size_t)L.AP.nrows);
    if (q_sliced) {
      sq[l] = make_sliced_q(L.AP, L.P, p->amg_q_nnz[l], /*ordered=*/true);
      p->amg_q_sliced[l] = 1;
    } else {
      Q[l] = fused_q(L.AP, L.P, qfront[l]);
      p->amg_q_nnz[l] = (int64_t)Q[l].ci.size();
    }
    if (l >= 1) M[l] = residual_restriction(L);
  }
  // sliced copies (A of levels >= 1, Q, R) of the matrices with many rows
  std::vector<std::array<Sliced, 3>> sl(nl);
  for (int l = 0; l < nl; ++l) {
    const AmgLevel& L = H.lv[l];
    const Csr* M[3] = {&L.A, nullptr, &L.R};
    for (int k = 0; k < 3; ++k) {
      if (k == 1) {   // Q: sliced above when its level qualifies
        if (!p->amg_q_sliced[l]) continue;
        sl[l][1] = std::move(sq[l].ap);
      } else {
        if ((k == 0 && l == 0) ||
            (!slice_all && (M[k]->nrows < kSlicedRows || M[k]->ci.size() > kWideRow * (size_t)M[k]->nrows)))
          continue;
        sl[l][k] = make_sliced(M[k]->rp, M[k]->ci, M[k]->v, M[k]->ncols, 1, 0, /*ordered=*/true);
      }
      if ((int64_t)sl[l][k].so.back() >= (int64_t)1 << 30) return invalid("multigrid matrix too large to slice");
    }
  }
  // which levels' DOWN also restricts, and how
  std::vector<int> wm(nl, 4), mblk(nl, 0);
  for (int l = 1; l < nl && (c->vcycle & MMSD_VC_FUSE_REST); ++l) {
    const AmgLevel& L = H.lv[l];
    fused_shape(L.A.nrows, (double)L.A.ci.size() / L.A.nrows, sl[l][0].so.empty() ? model_lanes(L.A) : 1, L.R.nrows,
                (double)L.R.ci.size() / std::max(1, L.R.nrows), sl[l][2].so.empty() ? model_lanes(L.R) : 1, M[l], wm[l],
                mblk[l]);
  }
  // the last level's DOWN also solves the coarsest level when it restricts
  // and the dense product Ainv M is small: x_c = (Ainv M) b
  std::vector<double> ainv_m;
  p->amg_folded = false;
  int wa_last = 0;   // A's lanes on the last level when the solve is folded (0: the default)
  if ((c->vcycle & MMSD_VC_FOLD_SOLVE) && nl >= 2 && mblk[nl - 1] > 0 &&
      (double)H.nc * H.lv[nl - 1].A.nrows * s <= kMaxFoldedBytes) {
    const Csr& Ml = M[nl - 1];
    const int64_t nlast = H.lv[nl - 1].A.nrows;
    ainv_m.assign((size_t)H.nc * nlast, 0.0);
    parallel_for(H.nc, [&](int64_t I0, int64_t I1) {
      for (int64_t I = I0; I < I1; ++I) {
        double* out = &ainv_m[(size_t)I * nlast];
        for (int64_t K = 0; K < H.nc; ++K) {
          const double a = H.Ainv[(size_t)I * H.nc + K];
          for (int k = Ml.rp[K]; k < Ml.rp[K + 1]; ++k) out[Ml.ci[k]] += a * Ml.v[k];
        }
      }
    });
    p->amg_folded = true;
    const AmgLevel& Ll = H.lv[nl - 1];
    if (sl[nl - 1][0].so.empty())
      folded_shape(Ll.A.nrows, (double)Ll.A.ci.size() / Ll.A.nrows, H.nc, wa_last, mblk[nl - 1]);
  }
  for (int l = 1; l < nl; ++l) {
    if (mblk[l] > 0 && !(p->amg_folded && l == nl - 1)) p->amg_m_nnz[l] = (int64_t)M[l].ci.size();
    else if (mblk[l] == 0) M[l] = Csr{};
  }
  for (int l = 0; l < nl; ++l) {
    const AmgLevel& L = H.lv[l];
    const size_t n = L.A.nrows, nn = L.P.ncols;
    for (int k = 0; k < 3; ++k) {
      const Sliced& S = sl[l][k];
      if (S.so.empty()) continue;
      lo[l].sl[k][0] = take(4 * S.so.size());
      lo[l].sl[k][1] = take(4 * S.sc.size());
      lo[l].sl[k][2] = take(s * S.sv.size());
      lo[l].sl[k][3] = take(4 * S.order.size());
    }
    // CSR copies only of the matrices without a sliced one
    if (l > 0 && sl[l][0].so.empty()) {
      lo[l].arp = take(4 * (n + 1));
      lo[l].aci = take(4 * L.A.ci.size());
      lo[l].av = take(s * L.A.ci.size());
    }
    if (sl[l][1].so.empty()) {
      lo[l].qrp = take(4 * (n + 1));
      lo[l].qci = take(4 * Q[l].ci.size());
      lo[l].qv = take(2 * s * Q[l].ci.size());
    } else {
      lo[l].qpo = take(4 * sq[l].po.size());
      lo[l].qpv = take(s * sq[l].pv.size());
    }
    if (sl[l][2].so.empty()) {
      lo[l].rrp = take(4 * (nn + 1));
      lo[l].rci = take(4 * L.R.ci.size());
      lo[l].rv = take(s * L.R.ci.size());
    }
    if (mblk[l] > 0) {
      lo[l].mrp = take(4 * (nn + 1));
      lo[l].mci = take(4 * M[l].ci.size());
      lo[l].mv = take(s * M[l].ci.size());
    }
    lo[l].wd = take(s * n);
    lo[l].b = take(s * n);
    lo[l].wb = take(s * n);
    lo[l].res = take(s * n);
    lo[l].xb = take(s * n);
  }
  const size_t o_ainv = take(s * (size_t)H.nc * H.nc), o_bc = take(s * H.nc), o_xc = take(s * H.nc);
  const size_t o_ainvm = take(s * ainv_m.size());
  size_t o_r2[2];
  for (int k = 0; k < 2; ++k) o_r2[k] = take(s * Nt);
  const size_t o_zp = take(2 * s * Nt);
  const size_t o_q = take(s * Nt), o_rq = take(2 * s * Nt), o_lev = take(sizeof(MgLevel<real>) * nl);
  p->amg_arena = (char*)c->dalloc(o);
  if (!p->amg_arena) {
    set_error("device allocation of the multigrid hierarchy failed");
    return MMSD_E_NOMEM;
  }
  p->amg_bytes = o;
  char* base = p->amg_arena;
  hipStream_t st = c->stream;
  MMSD_HIP(hipMemsetAsync(base, 0, o, st));
  Prob<real>& P = desc_of<real>(p);
  std::vector<MgLevel<real>> lv(nl);
  int rc;
  for (int l = 0; l < nl; ++l) {
    const AmgLevel& L = H.lv[l];
    std::vector<double> wd(L.dinv.size());
    for (size_t i = 0; i < wd.size(); ++i) wd[i] = L.wsmooth * L.dinv[i];
    const bool csr[3] = {l > 0 && sl[l][0].so.empty(), sl[l][1].so.empty(), sl[l][2].so.empty()};
    if (csr[0] && ((rc = upload_int(st, base + lo[l].arp, L.A.rp)) || (rc = upload_int(st, base + lo[l].aci, L.A.ci)) ||
                   (rc = upload_vec<real>(st, base + lo[l].av, L.A.v))))
      return rc;
    if (csr[1] && ((rc = upload_int(st, base + lo[l].qrp, Q[l].rp)) || (rc = upload_int(st, base + lo[l].qci, Q[l].ci)) ||
                   (rc = upload_vec<real>(st, base + lo[l].qv, Q[l].v))))
      return rc;
    if (!csr[1] &&
        ((rc = upload_int(st, base + lo[l].qpo, sq[l].po)) || (rc = upload_vec<real>(st, base + lo[l].qpv, sq[l].pv))))
      return rc;
    if (csr[2] && ((rc = upload_int(st, base + lo[l].rrp, L.R.rp)) || (rc = upload_int(st, base + lo[l].rci, L.R.ci)) ||
                   (rc = upload_vec<real>(st, base + lo[l].rv, L.R.v))))
      return rc;
    if (mblk[l] > 0 && ((rc = upload_int(st, base + lo[l].mrp, M[l].rp)) || (rc = upload_int(st, base + lo[l].mci, M[l].ci)) ||
                   (rc = upload_vec<real>(st, base + lo[l].mv, M[l].v))))
      return rc;
    if ((rc = upload_vec<real>(st, base + lo[l].wd, wd))) return rc;
    const int* so[3] = {nullptr, nullptr, nullptr};
    const int* sc[3] = {nullptr, nullptr, nullptr};
    const real* sv[3] = {nullptr, nullptr, nullptr};
    const int* sp[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < 3; ++k) {
      const Sliced& S = sl[l][k];
      if (S.so.empty()) continue;
      if ((rc = upload_int(st, base + lo[l].sl[k][0], S.so)) || (rc = upload_int(st, base + lo[l].sl[k][1], S.sc)) ||
          (rc = upload_vec<real>(st, base + lo[l].sl[k][2], S.sv)) ||
          (rc = upload_int(st, base + lo[l].sl[k][3], S.order)))
        return rc;
      so[k] = (const int*)(base + lo[l].sl[k][0]);
      sc[k] = (const int*)(base + lo[l].sl[k][1]);
      sv[k] = (const real*)(base + lo[l].sl[k][2]);
      if (!S.order.empty()) sp[k] = (const int*)(base + lo[l].sl[k][3]);
    }
    if (l == 0) {   // level 0's operator is the potential matrix
      so[0] = P.lso;
      sc[0] = P.lsc;
      sv[0] = P.lsv;
    }
    MgLevel<real>& d = lv[l];
    d.aso = so[0];
    d.asc = sc[0];
    d.asv = sv[0];
    d.qso = so[1];
    d.qsc = sc[1];
    d.qsv = sv[1];
    d.qpo = csr[1] ? nullptr : (const int*)(base + lo[l].qpo);
    d.qpv = csr[1] ? nullptr : (const real*)(base + lo[l].qpv);
    d.rso = so[2];
    d.rsc = sc[2];
    d.rsv = sv[2];
    d.aord = sp[0];
    d.qord = sp[1];
    d.rord = sp[2];
    d.n = L.A.nrows;
    d.n_next = L.P.ncols;
    d.lanes_a = (l == nl - 1 && wa_last) ? wa_last : model_lanes(L.A);
    d.lanes_q = model_lanes(Q[l]);
    d.lanes_r = model_lanes(L.R);
    d.lanes_m = wm[l];
    d.m_blocks = mblk[l];
    d.mrp = mblk[l] > 0 ? (const int*)(base + lo[l].mrp) : nullptr;
    d.mci = mblk[l] > 0 ? (const int*)(base + lo[l].mci) : nullptr;
    d.mv = mblk[l] > 0 ? (const real*)(base + lo[l].mv) : nullptr;
    d.arp = csr[0] ? (const int*)(base + lo[l].arp) : nullptr;
    d.aci = csr[0] ? (const int*)(base + lo[l].aci) : nullptr;
    d.av = csr[0] ? (const real*)(base + lo[l].av) : nullptr;
    d.qrp = csr[1] ? (const int*)(base + lo[l].qrp) : nullptr;
    d.qci = csr[1] ? (const int*)(base + lo[l].qci) : nullptr;
    d.qv = csr[1] ? (const Pair<real>*)(base + lo[l].qv) : nullptr;
    d.rrp = csr[2] ? (const int*)(base + lo[l].rrp) : nullptr;
    d.rci = csr[2] ? (const int*)(base + lo[l].rci) : nullptr;
    d.rv = csr[2] ? (const real*)(base + lo[l].rv) : nullptr;
    d.wd = (const real*)(base + lo[l].wd);
    d.b = (real*)(base + lo[l].b);
    d.wb = (real*)(base + lo[l].wb);
    d.res = (real*)(base + lo[l].res);
    d.xb = (real*)(base + lo[l].xb);
  }
  if ((rc = upload_vec<real>(st, base + o_ainv, H.Ainv))) return rc;
  if ((rc = upload_vec<real>(st, base + o_ainvm, ainv_m))) return rc;
  MMSD_HIP(hipMemcpyAsync(base + o_lev, lv.data(), sizeof(MgLevel<real>) * nl, hipMemcpyHostToDevice, st));
  MMSD_HIP(hipStreamSynchronize(st));
  P.n_lev = nl;
  P.mg_fused = 0;
  for (int l = 0; l < nl; ++l) P.mg_fused |= (lv[l].m_blocks > 0) << l;
  P.nc = H.nc;
  P.lev = (const MgLevel<real>*)(base + o_lev);
  P.Ainv = (const real*)(base + o_ainv);
  P.AinvM = p->amg_folded ? (const real*)(base + o_ainvm) : nullptr;
  P.bc = (real*)(base + o_bc);
  P.xc = (real*)(base + o_xc);
  for (int k = 0; k < 2; ++k) {
    P.r2[k] = (real*)(base + o_r2[k]);
  }
  P.zp = (Pair<real>*)(base + o_zp);
  P.q = (real*)(base + o_q);
  P.rq = (Pair<real>*)(base + o_rq);
  return MMSD_OK;
}

constexpr double kStreamBytes = 128.0 * (1 << 20);

// The problem's device arena: operators, node state, control.  With D the
// operators come from the device assembly's buffers (converted on the
// device); otherwise they are uploaded from the host assembly.
template <typename real>
int build_device(mmsd_problem p, const DeviceAssembly* D = nullptr) {
  mmsd_ctx c = p->ctx;
  const Assembly& A = p->A;
  const int64_t N = A.N, Nt = A.Nt, nnzM = (int64_t)A.mci.size();
  const int64_t nnzLs = Nt ? sliced_entries(A.lrp) : 0;
  if (nnzLs >= (int64_t)1 << 31) return invalid("potential matrix too large for 32-bit slice offsets");
  p->lpr = c->lpr;
  p->G = blocks_for(std::max<int64_t>(N, Nt), p->lpr, c->max_blocks);
  const int G = p->G;
  Layout L = make_layout(N, nnzM, Nt, nnzLs, sizeof(real));
  p->arena = (char*)c->dalloc(L.total);
  if (!p->arena) {
    set_error("device allocation of " + std::to_string(L.total) + " bytes failed");
    return MMSD_E_NOMEM;
  }
  p->arena_bytes = L.total;
  hipStream_t st = c->stream;
  char* base = p->arena;
  MMSD_HIP(hipMemsetAsync(base, 0, L.total, st));
  int rc;
  if (D) {
    MMSD_HIP(hipMemcpyAsync(base + L.mrp, D->mrp, 4 * (N + 1), hipMemcpyDeviceToDevice, st));
    MMSD_HIP(hipMemcpyAsync(base + L.mci, D->mci, 4 * nnzM, hipMemcpyDeviceToDevice, st));
    MMSD_HIP(launch_to_real<real>(D->K, (real*)(base + L.K), nnzM, st));
    MMSD_HIP(launch_to_real<real>(D->V, (real*)(base + L.V), N, st));
    for (int k = 0; k < 3; ++k) {
      MMSD_HIP(launch_to_real<real>(D->D1 + k * nnzM, (real*)(base + L.D1[k]), nnzM, st));
      MMSD_HIP(launch_to_real<real>(D->D2 + k * nnzM, (real*)(base + L.D2[k]), nnzM, st));
    }
    for (int k = 0; k < 6; ++k) MMSD_HIP(launch_to_real<real>(D->Q + k * N, (real*)(base + L.Q[k]), N, st));
  } else {
    if ((rc = upload_int(st, base + L.mrp, A.mrp)) || (rc = upload_int(st, base + L.mci, A.mci)) ||
        (rc = upload_vec<real>(st, base + L.K, A.K)) || (rc = upload_vec<real>(st, base + L.V, A.V)))
      return rc;
    for (int k = 0; k < 3; ++k)
      if ((rc = upload_vec<real>(st, base + L.D1[k], A.D1[k])) ||
          (rc = upload_vec<real>(st, base + L.D2[k], A.D2[k])))
        return rc;
    for (int k = 0; k < 6; ++k)
      if ((rc = upload_vec<real>(st, base + L.Q[k], A.Q[k]))) return rc;
  }
  if (Nt > 0 && D) {
    // sliced on the device from the assembled CSR; only the slice offsets
    // come from the host (the copy of the row starts it keeps)
    if ((rc = upload_int(st, base + L.lso, slice_offsets(A.lrp)))) return rc;
    MMSD_HIP(launch_slice_rows<real>(D->lrp, D->lci, D->L, (const int32_t*)(base + L.lso), Nt,
                                     (int32_t*)(base + L.lsc), (real*)(base + L.lsv), (real*)(base + L.lsum),
                                     (real*)(base + L.rec[0]), (real*)(base + L.rec[1]), st));
  } else if (Nt > 0) {
    // the potential matrix lives on the device only in its sliced layout
    const Sliced S = make_sliced(A.lrp, A.lci, A.L, (int)Nt);
    if ((rc = upload_int(st, base + L.lso, S.so)) || (rc = upload_int(st, base + L.lsc, S.sc)) ||
        (rc = upload_vec<real>(st, base + L.lsv, S.sv)))
      return rc;
    // row sums, summed in FP64 from the assembled values
    std::vector<double> rs(Nt, 0.0);
    for (int64_t i = 0; i < Nt; ++i)
      for (int k = A.lrp[i]; k < A.lrp[i + 1]; ++k) rs[i] += A.L[k];
    if ((rc = upload_vec<real>(st, base + L.lsum, rs))) return rc;
    // Jacobi factors live in the d field of both CG record buffers
    std::vector<double> rec(4 * (size_t)Nt, 0.0);
    for (int64_t i = 0; i < Nt; ++i) rec[4 * i + 3] = A.invd[i];
    if ((rc = upload_vec<real>(st, base + L.rec[0], rec)) || (rc = upload_vec<real>(st, base + L.rec[1], rec)))
      return rc;
  }
  // initial state: m = +z in slot 0
  {
    std::vector<double> one(N, 1.0);
    if ((rc = upload_vec<real>(st, base + L.m[0][2], one))) return rc;
  }
  Prob<real>& P = desc_of<real>(p);
  std::memset(&P, 0, sizeof(P));
  P.N = (int)N;
  P.Nt = (int)Nt;
  P.G = G;
  // stream the sliced matrices past the caches when the potential matrix
  // alone exceeds half of the 256 MB Infinity Cache
  P.stream = (double)nnzLs * (4 + sizeof(real)) > kStreamBytes ? 1 : 0;
  P.blk0 = 0;
  P.mrp = (const int*)(base + L.mrp);
  P.mci = (const int*)(base + L.mci);
  P.K = (const real*)(base + L.K);
  for (int k = 0; k < 3; ++k) {
    P.D1[k] = (const real*)(base + L.D1[k]);
    P.D2[k] = (const real*)(base + L.D2[k]);
    P.h[k] = (real*)(base + L.h[k]);
    for (int s = 0; s < 2; ++s) {
      P.m[s][k] = (real*)(base + L.m[s][k]);
      P.H[s][k] = (real*)(base + L.H[s][k]);
    }
  }
  for (int k = 0; k < 6; ++k) P.Q[k] = (const real*)(base + L.Q[k]);
  for (int k = 0; k < 2; ++k) P.mh[k] = (real*)(base + L.mh[k]);
  P.V = (const real*)(base + L.V);
  P.lso = (const int*)(base + L.lso);
  P.lsc = (const int*)(base + L.lsc);
  P.lsv = (const real*)(base + L.lsv);
  P.lsum = (const real*)(base + L.lsum);
  for (int k = 0; k < 3; ++k) P.u3[k] = (real*)(base + L.u[k]);
  P.p = (real*)(base + L.p);
  for (int k = 0; k < 2; ++k) P.rec[k] = (Rec<real>*)(base + L.rec[k]);
  P.ndone = nullptr;
  P.part = (double*)(base + L.part);
  P.ctrl = (Ctrl*)(base + L.ctrl);
  p->dctrl = P.ctrl;
  p->dprob = base + L.prob;
  p->dblk = (int*)(base + L.blk);
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2; ++j) p->snap[k][j] = base + L.snap[k][j];
  if (p->has_amg && (rc = build_amg<real>(p))) return rc;
  bytes_model<real>(p);
  P.btab = (const double*)(base + L.btab);
  MMSD_HIP(hipMemcpyAsync(base + L.btab, p->btab, 8 * kByteSlots, hipMemcpyHostToDevice, st));
  int blk[2] = {0, G};
  MMSD_HIP(hipMemcpyAsync(p->dprob, &P, sizeof(P), hipMemcpyHostToDevice, st));
  MMSD_HIP(hipMemcpyAsync(p->dblk, blk, sizeof(blk), hipMemcpyHostToDevice, st));
  MMSD_HIP(hipStreamSynchronize(st));
  return MMSD_OK;
}

// Change a problem's launch shape (lanes per row, block cap) between runs.
int set_launch(mmsd_problem p, int lpr, int max_blocks) {
  const int G = blocks_for(std::max<int64_t>(p->A.N, p->A.Nt), lpr, max_blocks);
  if (G == p->G && lpr == p->lpr) return MMSD_OK;
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
  p->lpr = lpr;
  p->G = G;
  if (p->precision == MMSD_MIXED) desc_of<float>(p).G = G;
  else desc_of<double>(p).G = G;
  const int blk[2] = {0, G};
  hipStream_t st = p->ctx->stream;
  MMSD_HIP(hipMemcpyAsync(p->dprob, p->desc, sizeof(Prob<double>), hipMemcpyHostToDevice, st));
  MMSD_HIP(hipMemcpyAsync(p->dblk, blk, sizeof(blk), hipMemcpyHostToDevice, st));
  MMSD_HIP(hipStreamSynchronize(st));
  return MMSD_OK;
}

}  // namespace

int resolve(mmsd_problem p, const mmsd_options* o, Resolved* r) {
  mmsd_options d;
  mmsd_options_default(&d);
  if (o) {
    if (o->tol_torque > 0) d.tol_torque = o->tol_torque;
    if (o->max_evals > 0) d.max_evals = o->max_evals;
    if (o->terms > 0) d.terms = o->terms;
    if (o->nonmono_M > 0) d.nonmono_M = o->nonmono_M;
    if (o->pcg_rtol > 0) d.pcg_rtol = o->pcg_rtol;
    if (o->pcg_maxit > 0) d.pcg_maxit = o->pcg_maxit;
    if (o->step_rule > 0) d.step_rule = o->step_rule;
    if (o->refine_tol_T > 0) d.refine_tol_T = o->refine_tol_T;
    if (o->precond > 0) d.precond = o->precond;
    if (o->precond < 0 || o->precond > MMSD_PRECOND_AMG) return invalid("unknown preconditioner");
    if (o->stop_rule < 0 || o->stop_rule > MMSD_STOP_SUM_SQ) return invalid("unknown stopping test");
    d.stop_rule = o->stop_rule;
    if (o->terms < 0 || o->terms > MMSD_ALL || o->nonmono_M > kMaxHist || o->step_rule < 0 ||
        o->step_rule > MMSD_STEP_BB2)
      return invalid("options out of range");
  }
  if (!o || !(o->pcg_rtol > 0)) d.pcg_rtol = p->precision == MMSD_MIXED ? 1e-6 : 1e-10;
  if ((d.terms & MMSD_DEMAG) && p->A.Nt == 0)
    return invalid("stray field requested on a mesh without Dirichlet (outer boundary) nodes");
  r->tol = d.tol_torque;
  r->rtol = d.pcg_rtol;
  r->max_evals = d.max_evals;
  r->terms = d.terms;
  r->M = d.nonmono_M;
  r->rule = d.step_rule;
  r->maxit = d.pcg_maxit;
  r->refine = d.refine_tol_T;
  r->stop = d.stop_rule;
  if (d.precond == MMSD_PRECOND_AMG && !p->has_amg)
    return invalid("multigrid preconditioner requested but not available for this mesh");
  r->precond = (d.precond == MMSD_PRECOND_JACOBI || !p->has_amg) ? PC_JACOBI : PC_AMG;
  return MMSD_OK;
}

constexpr int kMixedHalvings = 20;   // a factor of 1e6 on the trial step

int arm(mmsd_problem p, const Resolved& r, int stage, int store_h) {
  const Assembly& A = p->A;
  // FP64 runs decide on the energies themselves and halve down to the tau
  // floor, as the oracle.  The mixed form decides on the accepted energy plus
  // each trial's change (summed from products of the step, accurate relative
  // to the change; the difference of two FP32-field energies is not), and a
  // line search gives up after kMixedHalvings failed trials: once the torque
  // reaches the error of the FP32 fields, halving no longer resolves a decrease.
  // The mixed form also stops after a run of accepted steps without
  // progress; it counts an energy decrease as progress from 2^-20 of the sum
  // of the term magnitudes (the resolution of an energy built from FP32
  // fields).  Its anisotropy energy is summed per node as m.(tr(Q) I - Q) m,
  // which already holds the constant sum_e V_e K1_e.
  const bool mixed = p->precision == MMSD_MIXED;
  const double dp[15] = {r.tol, r.rtol * r.rtol, 1e-4, 0.5, 0.5, 0.1, 1e-10, 1e10, 1e-14,
                         p->b_ext[0] / A.Js, p->b_ext[1] / A.Js, p->b_ext[2] / A.Js, mixed ? 0.0 : A.c_an, A.vol,
                         mixed ? std::ldexp(1.0, -20) : 0.0};
  MMSD_HIP(launch_ctrl_init(p->dctrl, kArmSlot, stage, r.terms, r.M, r.rule, r.maxit, store_h,
                            (r.terms & MMSD_DEMAG) ? 1 : 0, p->acc, r.precond, mixed ? 1 : 0,
                            mixed ? kMixedHalvings : 0, r.stop, p->ucur, (long long)r.max_evals, dp,
                            p->ctx->stream));
  return MMSD_OK;
}

int launch_table(const Table& t, int parity, hipStream_t st) {
  hipError_t e =
      t.precision == MMSD_MIXED
          ? launch_step<float>(t.lpr, (const Prob<float>*)t.dprobs, t.nprob, t.dblk, t.grid, parity, st)
          : launch_step<double>(t.lpr, (const Prob<double>*)t.dprobs, t.nprob, t.dblk, t.grid, parity, st);
  if (e != hipSuccess) return hip_fail(e, "step launch");
  return MMSD_OK;
}

// Issue B ticks (one launch per table per tick), through a cached graph
// when allowed and timing is off.
int issue(mmsd_ctx c, const std::vector<Table>& tabs, int B, std::map<int, hipGraphExec_t>* graphs) {
  hipStream_t st = c->stream;
  if (B <= 0 || (B & 1)) return invalid("launch batches must have an even length");
  TimingState& T = c->timing;
  // With timing on, one event pair brackets the whole batch: it measures the
  // kernels back to back plus the gaps between them, the same launches a
  // kernel trace records.
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (T.stride > 0) {
    for (hipEvent_t* e : {&e0, &e1}) {
      if (T.pool.empty()) {
        MMSD_HIP(hipEventCreate(e));
      } else {
        *e = T.pool.back();
        T.pool.pop_back();
      }
    }
    MMSD_HIP(hipEventRecord(e0, st));
  }
  int rc = MMSD_OK;
  if (c->use_graph && graphs) {
    auto it = graphs->find(B);
    if (it == graphs->end()) {
      hipGraph_t g;
      MMSD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      for (int b = 0; b < B && !rc; ++b)
        for (const Table& t : tabs)
          if (!rc) rc = launch_table(t, b & 1, st);
      hipError_t ec = hipStreamEndCapture(st, &g);
      if (rc) return rc;
      if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
      hipGraphExec_t ex;
      hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
      it = graphs->emplace(B, ex).first;
    }
    MMSD_HIP(hipGraphLaunch(it->second, st));
  } else {
    for (int b = 0; b < B && !rc; ++b)
      for (const Table& t : tabs)
        if (!rc) rc = launch_table(t, b & 1, st);
    if (rc) return rc;
  }
  if (T.stride > 0) {
    MMSD_HIP(hipEventRecord(e1, st));
    T.pending.push_back(e0);
    T.pending.push_back(e1);
    T.pending_launches.push_back((double)B * (double)tabs.size());
  }
  return MMSD_OK;
}

// Collect the event timings of finished launches.
int drain_timing(mmsd_ctx c) {
  TimingState& T = c->timing;
  for (size_t k = 0; k + 1 < T.pending.size(); k += 2) {
    float ms = 0;
    MMSD_HIP(hipEventElapsedTime(&ms, T.pending[k], T.pending[k + 1]));
    T.ms += ms;
    T.count += T.pending_launches[k / 2];
    T.pool.push_back(T.pending[k]);
    T.pool.push_back(T.pending[k + 1]);
  }
  T.pending.clear();
  T.pending_launches.clear();
  return MMSD_OK;
}

double run_bytes(mmsd_problem p, const Ctrl& C) {
  double b = C.alg_bytes;
  if (!C.demag) b += (double)C.nphase[0] * (p->prep_bytes_nodemag - p->btab[PH_PREP]);
  if (C.store_h) b += (double)C.nphase[3] * p->phase_bytes_h;
  return b;
}

void fill_result(mmsd_problem p, const Ctrl& C, mmsd_result* out, double secs, int64_t launches) {
  const Assembly& A = p->A;
  const double E0 = A.mu0Ms2 * kNmCube;
  out->status = C.status;
  out->e_exch_J = C.eterm_acc[0] * E0;
  out->e_anis_J = C.eterm_acc[1] * E0;
  out->e_zeem_J = C.eterm_acc[2] * E0;
  out->e_demag_J = C.eterm_acc[3] * E0;
  out->energy_J = out->e_exch_J + out->e_anis_J + out->e_zeem_J + out->e_demag_J;
  out->max_torque = C.T_acc;
  out->sum_V_torque2 = C.d_acc * kNmCube;
  out->sum_torque2 = C.h2_acc;
  for (int k = 0; k < 3; ++k) out->m_avg[k] = C.mavg_acc[k];
  out->iterations = C.iters;
  out->evals = C.evals;
  out->pcg_iters = C.pcg_total;
  out->launches = launches;
  out->seconds = secs;
}

// Host-side bound on one run's wall time (env MMSD_RUN_TIMEOUT_S, default 1800 s).
bool run_timed_out(std::chrono::steady_clock::time_point t0) {
  static const double limit = [] {
    const char* e = std::getenv("MMSD_RUN_TIMEOUT_S");
    double v = e ? std::atof(e) : 0.0;
    return v > 0 ? v : 1800.0;
  }();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > limit;
}

int ensure_pinned(mmsd_problem p) {
  if (!p->hctrl) MMSD_HIP(hipHostMalloc((void**)&p->hctrl, 4 * sizeof(Ctrl), hipHostMallocDefault));
  return MMSD_OK;
}

namespace {

// Arm, then launch batches until the control block reports DONE.
int run_single(mmsd_problem p, const Resolved& r, int stage, int store_h, mmsd_result* out) {
  mmsd_ctx c = p->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  auto t0 = std::chrono::steady_clock::now();
  MMSD_HIP(hipSetDevice(c->device));
  int rc;
  if ((rc = ensure_pinned(p)) || (rc = arm(p, r, stage, store_h))) return rc;
  hipStream_t st = c->stream;
  std::vector<Table> tabs{{p->precision, p->dprob, p->dblk, 1, p->G, p->lpr}};
  int B = 8, cur = 0, stalls = 0;
  long long last_done = -1;
  bool have_prev = false;
  int64_t launched = 0;
  hipEvent_t ev[2];
  MMSD_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  MMSD_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  for (;;) {
    if ((rc = issue(c, tabs, B, &p->graphs))) break;
    launched += B;
    if (hipMemcpyAsync(&p->hctrl[2 * cur], p->dctrl, 2 * sizeof(Ctrl), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(ev[cur], st) != hipSuccess) {
      rc = hip_fail(hipGetLastError(), "poll copy");
      break;
    }
    if (have_prev) {
      hipError_t e = hipEventSynchronize(ev[1 - cur]);
      if (e != hipSuccess) {
        rc = hip_fail(e, "poll wait");
        break;
      }
      const Ctrl& H = latest(&p->hctrl[2 * (1 - cur)]);
      if (H.phase == PH_DONE) break;
      // every launch of an unfinished problem executes one phase; a counter
      // that stops moving means the phase machine is stuck
      if (H.launches_done == last_done) {
        if (++stalls >= 3) {
          set_error("device phase machine stalled");
          rc = MMSD_E_HIP;
          break;
        }
      } else {
        stalls = 0;
        last_done = H.launches_done;
      }
      if (run_timed_out(t0)) {
        set_error("run exceeded MMSD_RUN_TIMEOUT_S");
        rc = MMSD_E_HIP;
        break;
      }
    }
    have_prev = true;
    cur ^= 1;
    B = std::min(B * 2, 64);
  }
  hipError_t e = hipStreamSynchronize(st);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  const Ctrl& C = latest(&p->hctrl[2 * cur]);
  if (c->timing.stride > 0) {
    if ((rc = drain_timing(c))) return rc;
    c->timing.bytes += run_bytes(p, C);
  }
  p->acc = C.acc;
  p->ucur = C.ucur;
  p->h_valid = store_h != 0 && C.status == MMSD_OK;
  p->last_launches = launched;
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_result(p, C, out, secs, C.launches_done);
  return C.status;
}

template <typename real>
int copy_m_to_host(mmsd_problem p, double* m_out) {
  const Prob<real>& P = desc_of<real>(p);
  const int N = p->A.N;
  std::vector<real> tmp(3 * (size_t)N);
  hipStream_t st = p->ctx->stream;
  for (int k = 0; k < 3; ++k)
    MMSD_HIP(hipMemcpyAsync(tmp.data() + (size_t)k * N, P.m[p->acc][k], sizeof(real) * N, hipMemcpyDeviceToHost, st));
  MMSD_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) m_out[3 * (size_t)i + k] = (double)tmp[(size_t)k * N + i];
  return MMSD_OK;
}

// normalize = false restores a checkpointed m bit for bit.
template <typename real>
int copy_m_to_device(mmsd_problem p, const double* m, bool normalize) {
  const Prob<real>& P = desc_of<real>(p);
  const int N = p->A.N;
  std::vector<real> tmp(3 * (size_t)N);
  for (int i = 0; i < N; ++i) {
    const double x = m[3 * (size_t)i], y = m[3 * (size_t)i + 1], z = m[3 * (size_t)i + 2];
    const double n = std::sqrt(x * x + y * y + z * z);
    if (!(n > 0) || !std::isfinite(n)) return invalid("zero or non-finite magnetization at node " + std::to_string(i));
    const double s = normalize ? 1.0 / n : 1.0;
    tmp[i] = (real)(normalize ? x / n : x * s);
    tmp[(size_t)N + i] = (real)(normalize ? y / n : y * s);
    tmp[2 * (size_t)N + i] = (real)(normalize ? z / n : z * s);
  }
  hipStream_t st = p->ctx->stream;
  for (int k = 0; k < 3; ++k)
    MMSD_HIP(hipMemcpyAsync(P.m[p->acc][k], tmp.data() + (size_t)k * N, sizeof(real) * N, hipMemcpyHostToDevice, st));
  MMSD_HIP(hipStreamSynchronize(st));
  p->h_valid = false;
  return MMSD_OK;
}

// Device-side copies of (m, u) between the live state and snapshot `k`.
template <typename real>
int snapshot(mmsd_problem p, int k, bool save) {
  const Prob<real>& P = desc_of<real>(p);
  const size_t N = p->A.N, Nt = p->A.Nt;
  hipStream_t st = p->ctx->stream;
  real* sm = (real*)p->snap[k][0];
  for (int c = 0; c < 3; ++c) {
    real* live = P.m[p->acc][c];
    if (save) MMSD_HIP(hipMemcpyAsync(sm + c * N, live, sizeof(real) * N, hipMemcpyDeviceToDevice, st));
    else MMSD_HIP(hipMemcpyAsync(live, sm + c * N, sizeof(real) * N, hipMemcpyDeviceToDevice, st));
  }
  if (Nt) {
    if (save) MMSD_HIP(hipMemcpyAsync(p->snap[k][1], P.u3[p->ucur], sizeof(real) * Nt, hipMemcpyDeviceToDevice, st));
    else MMSD_HIP(hipMemcpyAsync(P.u3[p->ucur], p->snap[k][1], sizeof(real) * Nt, hipMemcpyDeviceToDevice, st));
  }
  return MMSD_OK;
}

int snap_locked(mmsd_problem p, int k, bool save) {
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  (void)hipSetDevice(p->ctx->device);
  int rc = p->precision == MMSD_MIXED ? snapshot<float>(p, k, save) : snapshot<double>(p, k, save);
  if (rc) return rc;
  MMSD_HIP(hipStreamSynchronize(p->ctx->stream));
  return MMSD_OK;
}

double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

}  // namespace

// Blocks of one problem inside a shared launch: about four passes of a block
// over its chunk of rows, a multiple of 8, capped by the problem's own shape.
int batch_blocks(mmsd_problem_s* p, bool demag) {
  const int64_t rows = std::max<int64_t>(p->A.N, demag ? p->A.Nt : 0);
  const int64_t per_block = 4LL * (kBlock / p->lpr);
  int64_t g = (rows + per_block - 1) / per_block;
  g = (g + 7) / 8 * 8;
  return (int)std::max<int64_t>(8, std::min<int64_t>(g, p->G));
}
}  // namespace mmsd

void* mmsd_ctx_s::dalloc(size_t bytes) {
  if (alloc) return alloc(bytes, user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void mmsd_ctx_s::dfree(void* p) {
  if (!p) return;
  if (free_fn) free_fn(p, user);
  else (void)hipFree(p);
}

// Key of the autotuner's cache: a problem class (precision, floor(log2(N + 1)),
// floor(log2(N_t + 1))).
static int64_t tune_key(int precision, int log2_n, int log2_nt) {
  return ((int64_t)precision << 40) | ((int64_t)log2_n << 20) | (int64_t)log2_nt;
}

// ============================ C ABI =======================================
// Operators assembled on the device (into D) and the host side the problem
// keeps: the magnet pattern and lumped volumes (sizes, material changes) and
// the potential matrix (multigrid setup) come back; the coupling, exchange
// and anisotropy values stay on the device.
int assemble_on_device(mmsd_problem p, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                       DeviceAssembly* D) {
  mmsd_ctx c = p->ctx;
  AssemblyStructure S;
  int rc = assemble_device_owned(c, mesh, mats, n_mats, D, &S);
  if (rc) return rc;
  Assembly& A = p->A;
  std::vector<double> V(D->N);
  A.mrp.resize(D->N + 1);
  A.mci.resize(D->nnzM);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    MMSD_HIP(hipSetDevice(c->device));
    hipStream_t st = c->stream;
    MMSD_HIP(hipMemcpyAsync(V.data(), D->V, 8 * D->N, hipMemcpyDeviceToHost, st));
    MMSD_HIP(hipMemcpyAsync(A.mrp.data(), D->mrp, 4 * (D->N + 1), hipMemcpyDeviceToHost, st));
    MMSD_HIP(hipMemcpyAsync(A.mci.data(), D->mci, 4 * D->nnzM, hipMemcpyDeviceToHost, st));
    if (D->Nt > 0) {
      A.lrp.resize(D->Nt + 1);
      A.lci.resize(D->nnzL);
      A.L.resize(D->nnzL);
      MMSD_HIP(hipMemcpyAsync(A.lrp.data(), D->lrp, 4 * (D->Nt + 1), hipMemcpyDeviceToHost, st));
      MMSD_HIP(hipMemcpyAsync(A.lci.data(), D->lci, 4 * D->nnzL, hipMemcpyDeviceToHost, st));
      MMSD_HIP(hipMemcpyAsync(A.L.data(), D->L, 8 * D->nnzL, hipMemcpyDeviceToHost, st));
    }
    MMSD_HIP(hipStreamSynchronize(st));
  }
  std::string err;
  if ((rc = assemble_host_side(mesh, mats, n_mats, &S, std::move(V), &A, &err))) set_error(err);
  return rc;
}

extern "C" {

const char* mmsd_last_error(void) { return mmsd::g_err.c_str(); }

void mmsd_options_default(mmsd_options* o) {
  if (!o) return;
  o->tol_torque = 1e-6;
  o->max_evals = 100000;
  o->terms = MMSD_ALL;
  o->nonmono_M = 20;
  o->pcg_rtol = 1e-10;
  o->pcg_maxit = 5000;
  o->step_rule = MMSD_STEP_ADAPTIVE;
  o->refine_tol_T = 0;
  o->precond = MMSD_PRECOND_AUTO;
  o->stop_rule = MMSD_STOP_MAX_TORQUE;
}

int mmsd_ctx_create(int device, void* hip_stream, mmsd_alloc_fn alloc, mmsd_free_fn free_fn, void* user,
                    mmsd_ctx* out) {
  if (!out) return invalid("null output handle");
  if ((alloc == nullptr) != (free_fn == nullptr)) return invalid("alloc and free must both be set or both NULL");
  int n = 0;
  MMSD_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return invalid("no such HIP device");
  MMSD_HIP(hipSetDevice(device));
  auto* c = new mmsd_ctx_s;
  c->device = device;
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = user;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "hipStreamCreate");
    }
    c->own_stream = true;
  }
  *out = c;
  return MMSD_OK;
}

int mmsd_ctx_destroy(mmsd_ctx c) {
  if (!c) return invalid("null context");
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->timing.pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->timing.pending) (void)hipEventDestroy(e);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return MMSD_OK;
}

int mmsd_set_launch_config(mmsd_ctx c, int lanes_per_row, int max_blocks) {
  if (!c) return invalid("null context");
  if (lanes_per_row && lanes_per_row != 4 && lanes_per_row != 8 && lanes_per_row != 16)
    return invalid("lanes_per_row must be 4, 8 or 16");
  if (max_blocks && (max_blocks < 8 || max_blocks > kMaxBlocks || max_blocks % 8))
    return invalid("max_blocks must be a multiple of 8 in [8, 2048]");
  if (lanes_per_row) c->lpr = lanes_per_row;
  if (max_blocks) c->max_blocks = max_blocks;
  return MMSD_OK;
}

int mmsd_set_vcycle(mmsd_ctx c, int flags) {
  if (!c) return invalid("null context");
  if (flags & ~(MMSD_VC_FUSE_REST | MMSD_VC_FOLD_SOLVE | MMSD_VC_SLICE_ALL)) return invalid("unknown V-cycle flags");
  c->vcycle = flags;
  return MMSD_OK;
}

int mmsd_set_assembly(mmsd_ctx c, int where) {
  if (!c) return invalid("null context");
  if (where != MMSD_ASSEMBLE_HOST && where != MMSD_ASSEMBLE_DEVICE)
    return invalid("assembly must be MMSD_ASSEMBLE_HOST or MMSD_ASSEMBLE_DEVICE");
  c->assembly = where;
  return MMSD_OK;
}

int mmsd_problem_setup_times(mmsd_problem p, double t[4]) {
  if (!p || !t) return invalid("null argument");
  for (int k = 0; k < 4; ++k) t[k] = p->setup_t[k];
  return MMSD_OK;
}

int mmsd_timing_enable(mmsd_ctx c, int stride) {
  if (!c || stride < 0) return invalid("bad timing request");
  c->timing.stride = stride;
  return MMSD_OK;
}

int mmsd_timing_read(mmsd_ctx c, double stats[3], int reset) {
  if (!c || !stats) return invalid("bad timing request");
  stats[0] = c->timing.ms;
  stats[1] = c->timing.count;
  stats[2] = c->timing.bytes;
  if (reset) c->timing.ms = c->timing.count = c->timing.bytes = 0;
  return MMSD_OK;
}

int mmsd_footprint(const mmsd_mesh* mesh, int precision, size_t* bytes_out) {
  if (!bytes_out || (precision != MMSD_FP64 && precision != MMSD_MIXED)) return invalid("bad footprint request");
  std::string err;
  PatternSizes ps;
  int rc = pattern_sizes(mesh, &ps, &err);
  if (rc) {
    set_error(err);
    return rc;
  }
  const size_t sv = precision == MMSD_MIXED ? 4 : 8;
  // the multigrid hierarchy's arena, known only after its setup: an
  // allowance of (24 + 2 s) bytes per potential-matrix entry and 8 s per
  // potential node (the 80 nm cube's FP64 hierarchy, counted from its
  // layout: ~155 MB against 166 MB allowed)
  const size_t amg = ps.Nt > 0 ? (24 + 2 * sv) * (size_t)ps.nnzLs + 8 * sv * (size_t)ps.Nt : 0;
  *bytes_out = make_layout(ps.N, ps.nnzM, ps.Nt, ps.nnzLs, sv).total + amg;
  return MMSD_OK;
}

int mmsd_problem_create(mmsd_ctx c, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, int precision,
                        mmsd_problem* out) {
  if (!c || !out) return invalid("null handle");
  if (precision != MMSD_FP64 && precision != MMSD_MIXED) return invalid("precision must be MMSD_FP64 or MMSD_MIXED");
  if (n_mats < 0 || (n_mats > 0 && !mats)) return invalid("bad material table");
  using Clock = std::chrono::steady_clock;
  const auto t0 = Clock::now();
  auto* p = new mmsd_problem_s;
  p->ctx = c;
  p->precision = precision;
  std::string err;
  DeviceAssembly D;
  int rc = MMSD_OK;
  if (c->assembly == MMSD_ASSEMBLE_DEVICE) {
    rc = assemble_on_device(p, mesh, mats, n_mats, &D);
  } else if ((rc = assemble(mesh, mats, n_mats, &p->A, &err))) {
    set_error(err);
  }
  if (rc) {
    D.release(c);
    delete p;
    return rc;
  }
  const auto t1 = Clock::now();
  if (p->A.Nt > 0) {
    Csr L0;
    L0.nrows = L0.ncols = p->A.Nt;
    L0.rp = p->A.lrp;
    L0.ci = p->A.lci;
    L0.v = p->A.L;
    p->has_amg = amg_setup(std::move(L0), AmgParams{}, &p->amg) && (int)p->amg.lv.size() <= kMaxLevels;
    // the level operators are kept only for sizes and byte counts
  }
  const auto t2 = Clock::now();
  {
    std::lock_guard<std::mutex> lk(c->mu);
    (void)hipSetDevice(c->device);
    const DeviceAssembly* dp = c->assembly == MMSD_ASSEMBLE_DEVICE ? &D : nullptr;
    rc = precision == MMSD_MIXED ? build_device<float>(p, dp) : build_device<double>(p, dp);
    // the build's copies and kernels read D and write the arena: both are
    // released below only once they are done, on failure too
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (!rc && e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
  }
  D.release(c);
  if (rc) {
    if (p->arena) c->dfree(p->arena);
    if (p->amg_arena) c->dfree(p->amg_arena);
    delete p;
    return rc;
  }
  const auto t3 = Clock::now();
  auto secs = [](Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); };
  p->setup_t[0] = secs(t0, t1);
  p->setup_t[1] = secs(t1, t2);
  p->setup_t[2] = secs(t2, t3);
  p->setup_t[3] = secs(t0, t3);
  *out = p;
  return MMSD_OK;
}

int mmsd_problem_destroy(mmsd_problem p) {
  if (!p) return invalid("null problem");
  mmsd_ctx c = p->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->hctrl) (void)hipHostFree(p->hctrl);
  c->dfree(p->arena);
  if (p->amg_arena) c->dfree(p->amg_arena);
  delete p;
  return MMSD_OK;
}

int mmsd_n_magnetic(mmsd_problem p, int64_t* n) {
  if (!p || !n) return invalid("null argument");
  *n = p->A.N;
  return MMSD_OK;
}

int mmsd_n_potential(mmsd_problem p, int64_t* n) {
  if (!p || !n) return invalid("null argument");
  *n = p->A.Nt;
  return MMSD_OK;
}

int mmsd_problem_sizes(mmsd_problem p, int64_t sizes[4]) {
  if (!p || !sizes) return invalid("null argument");
  sizes[0] = p->A.N;
  sizes[1] = (int64_t)p->A.mci.size();
  sizes[2] = p->A.Nt;
  sizes[3] = (int64_t)p->A.lci.size();
  return MMSD_OK;
}

int mmsd_set_material(mmsd_problem p, const mmsd_material* m) {
  if (!p || !m) return invalid("null argument");
  double un = std::sqrt(dot3(m->easy_axis, m->easy_axis));
  if (m->region < 1 || !(un > 0) || !(m->Js_T > 0) || !(m->A_Jm >= 0) || !std::isfinite(m->K1_Jm3))
    return invalid("invalid material");
  ensure_magnet_adjacency(&p->A);
  auto saved = p->A.mats;
  p->A.mats[m->region] = MatLine{m->Js_T, m->K1_Jm3, m->A_Jm, {m->easy_axis[0], m->easy_axis[1], m->easy_axis[2]}};
  std::string err;
  int rc = assemble_material_values(&p->A, &err);
  if (rc) {
    p->A.mats = saved;
    assemble_material_values(&p->A, &err);
    set_error(err);
    return rc;
  }
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  (void)hipSetDevice(p->ctx->device);
  hipStream_t st = p->ctx->stream;
  if (p->precision == MMSD_MIXED) {
    Prob<float>& P = desc_of<float>(p);
    if ((rc = upload_vec<float>(st, (char*)P.K, p->A.K))) return rc;
    for (int k = 0; k < 6; ++k)
      if ((rc = upload_vec<float>(st, (char*)P.Q[k], p->A.Q[k]))) return rc;
  } else {
    Prob<double>& P = desc_of<double>(p);
    if ((rc = upload_vec<double>(st, (char*)P.K, p->A.K))) return rc;
    for (int k = 0; k < 6; ++k)
      if ((rc = upload_vec<double>(st, (char*)P.Q[k], p->A.Q[k]))) return rc;
  }
  return MMSD_OK;
}

int mmsd_set_field(mmsd_problem p, const double b[3]) {
  if (!p || !b) return invalid("null argument");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(b[k])) return invalid("non-finite field");
  for (int k = 0; k < 3; ++k) p->b_ext[k] = b[k];
  return MMSD_OK;
}

int mmsd_set_m(mmsd_problem p, const double* m) {
  if (!p || !m) return invalid("null argument");
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  (void)hipSetDevice(p->ctx->device);
  return p->precision == MMSD_MIXED ? copy_m_to_device<float>(p, m, true) : copy_m_to_device<double>(p, m, true);
}

int mmsd_get_m(mmsd_problem p, double* m_out) {
  if (!p || !m_out) return invalid("null argument");
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  (void)hipSetDevice(p->ctx->device);
  return p->precision == MMSD_MIXED ? copy_m_to_host<float>(p, m_out) : copy_m_to_host<double>(p, m_out);
}

int mmsd_minimize(mmsd_problem p, const mmsd_options* o, mmsd_result* out) {
  if (!p || !out) return invalid("null argument");
  Resolved r;
  int rc = resolve(p, o, &r);
  if (rc) return rc;
  return run_single(p, r, ST_INIT, 0, out);
}

int mmsd_evaluate(mmsd_problem p, const mmsd_options* o, mmsd_result* out) {
  if (!p || !out) return invalid("null argument");
  Resolved r;
  int rc = resolve(p, o, &r);
  if (rc) return rc;
  return run_single(p, r, ST_EVAL, 1, out);
}

int mmsd_get_field(mmsd_problem p, double* h_out) {
  if (!p || !h_out) return invalid("null argument");
  if (!p->h_valid) return invalid("no field stored: call mmsd_evaluate first");
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  (void)hipSetDevice(p->ctx->device);
  const int N = p->A.N;
  hipStream_t st = p->ctx->stream;
  std::vector<double> tmp(3 * (size_t)N);
  for (int k = 0; k < 3; ++k) {
    if (p->precision == MMSD_MIXED) {
      std::vector<float> f(N);
      MMSD_HIP(hipMemcpyAsync(f.data(), desc_of<float>(p).h[k], 4 * (size_t)N, hipMemcpyDeviceToHost, st));
      MMSD_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < N; ++i) tmp[(size_t)k * N + i] = f[i];
    } else {
      MMSD_HIP(hipMemcpyAsync(tmp.data() + (size_t)k * N, desc_of<double>(p).h[k], 8 * (size_t)N,
                              hipMemcpyDeviceToHost, st));
    }
  }
  MMSD_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) h_out[3 * (size_t)i + k] = tmp[(size_t)k * N + i];
  return MMSD_OK;
}

int mmsd_get_potential(mmsd_problem p, double* u_out) {
  if (!p || !u_out) return invalid("null argument");
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  (void)hipSetDevice(p->ctx->device);
  const Assembly& A = p->A;
  std::fill(u_out, u_out + A.n_nodes, 0.0);
  if (!A.Nt) return MMSD_OK;
  hipStream_t st = p->ctx->stream;
  std::vector<double> u(A.Nt);
  if (p->precision == MMSD_MIXED) {
    std::vector<float> f(A.Nt);
    MMSD_HIP(hipMemcpyAsync(f.data(), desc_of<float>(p).u3[p->ucur], 4 * (size_t)A.Nt, hipMemcpyDeviceToHost, st));
    MMSD_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < A.Nt; ++i) u[i] = f[i];
  } else {
    MMSD_HIP(hipMemcpyAsync(u.data(), desc_of<double>(p).u3[p->ucur], 8 * (size_t)A.Nt, hipMemcpyDeviceToHost, st));
    MMSD_HIP(hipStreamSynchronize(st));
  }
  const double scale = A.Ms * 1e-9;   // internal unit of the potential: Ms nm
  for (int i = 0; i < A.Nt; ++i) u_out[A.pot_global[i]] = u[i] * scale;
  return MMSD_OK;
}

int mmsd_hysteresis(mmsd_problem p, const double* bT, int64_t n, const mmsd_options* o, mmsd_result* per_step,
                    double* b_switch_out, int64_t* n_switch_out) {
  if (!p || !bT || n <= 0 || !per_step) return invalid("bad hysteresis arguments");
  Resolved r;
  int rc = resolve(p, o, &r);
  if (rc) return rc;
  double uh[3] = {0, 0, 0};
  for (int64_t k = 0; k < n; ++k) {
    double nb = std::sqrt(dot3(bT + 3 * k, bT + 3 * k));
    if (nb > 0) {
      for (int c = 0; c < 3; ++c) uh[c] = bT[3 * k + c] / nb;
      break;
    }
  }
  if (dot3(uh, uh) == 0) return invalid("all fields are zero");
  int64_t nsw = 0;
  int prev_sign = 0;
  for (int64_t k = 0; k < n; ++k) {
    if ((rc = mmsd_set_field(p, bT + 3 * k))) return rc;
    rc = run_single(p, r, ST_INIT, 0, &per_step[k]);
    if (rc < 0) return rc;
    const double proj = dot3(per_step[k].m_avg, uh);
    const int sgn = proj > 0 ? 1 : (proj < 0 ? -1 : 0);
    if (k > 0 && sgn != prev_sign) {
      const double* B0 = bT + 3 * (k - 1);
      const double* B1 = bT + 3 * k;
      double bsw = 0.5 * (dot3(B0, uh) + dot3(B1, uh));
      if (r.refine > 0) {
        // bisect from the last unswitched minimum (snapshot 0); the switched
        // state of step k waits in snapshot 1
        if ((rc = snap_locked(p, 1, true))) return rc;
        double lo[3], hi[3];
        for (int c = 0; c < 3; ++c) {
          lo[c] = B0[c];
          hi[c] = B1[c];
        }
        for (;;) {
          const double d[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
          if (std::sqrt(dot3(d, d)) <= r.refine) break;
          double mid[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
          if ((rc = snap_locked(p, 0, false)) || (rc = mmsd_set_field(p, mid))) return rc;
          mmsd_result rm;
          rc = run_single(p, r, ST_INIT, 0, &rm);
          if (rc < 0) return rc;
          const double pm = dot3(rm.m_avg, uh);
          const int sm = pm > 0 ? 1 : (pm < 0 ? -1 : 0);
          if (sm != prev_sign) {
            for (int c = 0; c < 3; ++c) hi[c] = mid[c];
          } else {
            for (int c = 0; c < 3; ++c) lo[c] = mid[c];
            if ((rc = snap_locked(p, 0, true))) return rc;
          }
        }
        bsw = 0.5 * (dot3(lo, uh) + dot3(hi, uh));
        if ((rc = snap_locked(p, 1, false)) || (rc = mmsd_set_field(p, B1))) return rc;
      }
      if (b_switch_out) b_switch_out[nsw] = bsw;
      ++nsw;
    }
    if ((rc = snap_locked(p, 0, true))) return rc;
    prev_sign = sgn;
  }
  if (n_switch_out) *n_switch_out = nsw;
  return MMSD_OK;
}

int mmsd_minimize_batch(mmsd_problem* probs, int n, const mmsd_options* o, mmsd_result* out) {
  if (!probs || n <= 0 || !out) return invalid("bad batch arguments");
  mmsd_ctx c = probs[0]->ctx;
  for (int i = 0; i < n; ++i)
    if (!probs[i] || probs[i]->ctx != c) return invalid("batch problems must share one context");
  std::vector<Resolved> rs(n);
  for (int i = 0; i < n; ++i) {
    int rc = resolve(probs[i], o, &rs[i]);
    if (rc) return rc;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  auto t0 = std::chrono::steady_clock::now();
  MMSD_HIP(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  // Each problem gets blocks in proportion to its rows (about four passes of
  // a block over its chunk), capped by its own launch shape; the count stays
  // fixed for the run because a launch reduces the previous launch's G
  // partials.
  std::vector<int> gb(n);
  for (int i = 0; i < n; ++i) gb[i] = batch_blocks(probs[i], (rs[i].terms & MMSD_DEMAG) != 0);
  // scratch: the finished count and list, then the tables
  const size_t list_bytes = align_up(256 + 4 * (size_t)n);
  char* misc = (char*)c->dalloc(list_bytes);
  if (!misc) return invalid("batch allocation failed");
  unsigned* dndone = (unsigned*)misc;
  int* dlist = (int*)(misc + 256);
  char* tab = nullptr;
  std::vector<Table> tabs;
  // One table per precision over the unfinished problems; finished ones are
  // dropped when the table is rebuilt (problems keep their block counts).
  auto build_tables = [&](const std::vector<char>& done) -> int {
    if (tab) c->dfree(tab);
    tab = nullptr;
    tabs.clear();
    std::vector<int> idx[2];
    for (int i = 0; i < n; ++i)
      if (!done[i]) idx[probs[i]->precision == MMSD_MIXED ? 1 : 0].push_back(i);
    size_t bytes = 256;
    for (int q = 0; q < 2; ++q) bytes += align_up(sizeof(Prob<double>) * idx[q].size()) + align_up(4 * (idx[q].size() + 1));
    tab = (char*)c->dalloc(bytes);
    if (!tab) return invalid("batch table allocation failed");
    size_t off = 0;
    for (int q = 0; q < 2; ++q) {
      if (idx[q].empty()) continue;
      const size_t ps = q ? sizeof(Prob<float>) : sizeof(Prob<double>);
      std::vector<unsigned char> h(ps * idx[q].size());
      std::vector<int> blk(idx[q].size() + 1, 0);
      const int lpr = probs[idx[q][0]]->lpr;
      for (size_t k = 0; k < idx[q].size(); ++k) {
        const int i = idx[q][k];
        mmsd_problem p = probs[i];
        if (p->lpr != lpr) return invalid("batch problems of one precision must share lanes per row");
        blk[k + 1] = blk[k] + gb[i];
        std::memcpy(&h[k * ps], p->desc, ps);
        auto patch = [&](auto* d) {
          d->G = gb[i];
          d->blk0 = blk[k];
          d->ndone = dndone;
          d->done_list = dlist;
          d->slot = i;
        };
        if (q) patch(reinterpret_cast<Prob<float>*>(&h[k * ps]));
        else patch(reinterpret_cast<Prob<double>*>(&h[k * ps]));
      }
      char* dp = tab + off;
      off += align_up(h.size());
      char* db = tab + off;
      off += align_up(4 * blk.size());
      if (hipMemcpyAsync(dp, h.data(), h.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(db, blk.data(), 4 * blk.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return hip_fail(hipGetLastError(), "batch table upload");
      tabs.push_back(Table{q ? MMSD_MIXED : MMSD_FP64, dp, (const int*)db, (int)idx[q].size(), blk.back(), lpr});
    }
    return MMSD_OK;
  };
  std::vector<char> done(n, 0);
  int rc = build_tables(done);
  unsigned* hdone = nullptr;
  if (!rc && hipHostMalloc((void**)&hdone, 2 * sizeof(unsigned), hipHostMallocDefault) != hipSuccess)
    rc = hip_fail(hipGetLastError(), "pinned poll buffer");
  if (!rc && hipMemsetAsync(dndone, 0, 4, st) != hipSuccess) rc = hip_fail(hipGetLastError(), "memset");
  for (int i = 0; i < n && !rc; ++i) {
    if ((rc = ensure_pinned(probs[i]))) break;
    rc = arm(probs[i], rs[i], ST_INIT, 0);
  }
  std::map<int, hipGraphExec_t> graphs;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (!rc && (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess))
    rc = hip_fail(hipGetLastError(), "poll events");
  if (!rc) {
    int B = 8, cur = 0;
    bool have_prev = false;
    unsigned compacted_at = 0;
    for (;;) {
      if ((rc = issue(c, tabs, B, &graphs))) break;
      if (hipMemcpyAsync(&hdone[cur], dndone, sizeof(unsigned), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipEventRecord(ev[cur], st) != hipSuccess) {
        rc = hip_fail(hipGetLastError(), "batch poll");
        break;
      }
      if (have_prev) {
        hipError_t e = hipEventSynchronize(ev[1 - cur]);
        if (e != hipSuccess) {
          rc = hip_fail(e, "batch poll");
          break;
        }
        const unsigned nd = hdone[1 - cur];
        if (nd >= (unsigned)n) break;
        if (run_timed_out(t0)) {
          set_error("run exceeded MMSD_RUN_TIMEOUT_S");
          rc = MMSD_E_HIP;
          break;
        }
        // drop finished problems once an eighth of the rest has finished
        if (nd > compacted_at && (nd - compacted_at) * 8 >= (unsigned)n - compacted_at) {
          if (hipStreamSynchronize(st) != hipSuccess) {
            rc = hip_fail(hipGetLastError(), "batch compaction");
            break;
          }
          unsigned nd_now = 0;
          std::vector<int> list(n);
          if (hipMemcpy(&nd_now, dndone, 4, hipMemcpyDeviceToHost) != hipSuccess ||
              (nd_now && hipMemcpy(list.data(), dlist, 4 * (size_t)nd_now, hipMemcpyDeviceToHost) != hipSuccess)) {
            rc = hip_fail(hipGetLastError(), "batch compaction");
            break;
          }
          if (nd_now >= (unsigned)n) break;
          for (unsigned k = 0; k < nd_now; ++k) done[list[k]] = 1;
          for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
          graphs.clear();
          if ((rc = build_tables(done))) break;
          compacted_at = nd_now;
          have_prev = false;
          cur = 0;
          B = 8;
          continue;
        }
      }
      have_prev = true;
      cur ^= 1;
      B = std::min(B * 2, 64);
    }
    (void)hipStreamSynchronize(st);
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  if (!rc && c->timing.stride > 0) rc = drain_timing(c);
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = MMSD_OK;
  for (int i = 0; i < n && !rc; ++i) {
    mmsd_problem p = probs[i];
    if (hipMemcpy(&p->hctrl[0], p->dctrl, 2 * sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess) {
      rc = hip_fail(hipGetLastError(), "batch result copy");
      break;
    }
    const Ctrl& C = latest(&p->hctrl[0]);
    p->acc = C.acc;
    p->ucur = C.ucur;
    p->h_valid = false;
    if (c->timing.stride > 0) c->timing.bytes += run_bytes(p, C);
    fill_result(p, C, &out[i], secs, C.launches_done);
    if (C.status < 0) worst = C.status;
    else if (worst == MMSD_OK && C.status > 0) worst = C.status;
  }
  if (hdone) (void)hipHostFree(hdone);
  if (tab) c->dfree(tab);
  c->dfree(misc);
  return rc ? rc : worst;
}

int mmsd_copy_probe(mmsd_ctx c, size_t bytes, int reps, double* ms_out) {
  if (!c || bytes < 16 || reps < 1) return invalid("bad copy probe request");
  std::lock_guard<std::mutex> lk(c->mu);
  MMSD_HIP(hipSetDevice(c->device));
  bytes &= ~size_t(15);
  void* a = c->dalloc(bytes);
  void* b = c->dalloc(bytes);
  if (!a || !b) {
    c->dfree(a);
    c->dfree(b);
    return invalid("copy probe allocation failed");
  }
  hipStream_t st = c->stream;
  hipEvent_t e0, e1;
  int rc = MMSD_OK;
  if (hipMemsetAsync(a, 0, bytes, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    rc = hip_fail(hipGetLastError(), "copy probe setup");
  } else {
    if (hipEventRecord(e0, st) != hipSuccess) rc = hip_fail(hipGetLastError(), "copy probe event");
    for (int k = 0; k < reps && !rc; ++k)
      if (launch_copy_probe(a, b, bytes, st) != hipSuccess) rc = hip_fail(hipGetLastError(), "copy probe");
    float ms = 0;
    if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = hip_fail(hipGetLastError(), "copy probe timing");
    if (!rc && ms_out) *ms_out = ms / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  (void)hipStreamSynchronize(st);
  c->dfree(a);
  c->dfree(b);
  return rc;
}

int mmsd_set_problem_launch(mmsd_problem p, int lanes_per_row, int max_blocks) {
  if (!p) return invalid("null problem");
  if (lanes_per_row != 4 && lanes_per_row != 8 && lanes_per_row != 16)
    return invalid("lanes_per_row must be 4, 8 or 16");
  if (max_blocks < 8 || max_blocks > kMaxBlocks || max_blocks % 8)
    return invalid("max_blocks must be a multiple of 8 in [8, 2048]");
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  MMSD_HIP(hipSetDevice(p->ctx->device));
  return set_launch(p, lanes_per_row, max_blocks);
}

int mmsd_autotune(mmsd_problem p, int* lanes_out, int* blocks_out, double* us_out) {
  if (!p) return invalid("null problem");
  mmsd_ctx c = p->ctx;
  // cache: (precision, log2 N, log2 Nt) -> best shape, per context
  const int64_t key =
      tune_key(p->precision, std::ilogb((double)p->A.N + 1), std::ilogb((double)p->A.Nt + 1));
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
      MMSD_HIP(hipSetDevice(c->device));
      int rc = set_launch(p, it->second.first, it->second.second);
      if (rc) return rc;
      if (lanes_out) *lanes_out = p->lpr;
      if (blocks_out) *blocks_out = it->second.second;
      if (us_out) *us_out = -1.0;
      return MMSD_OK;
    }
  }
  // Time a fixed slice of the potential solve (PREP, CG0 and CG iterations,
  // no convergence test) for each shape; the potential is restored after.
  Resolved r;
  mmsd_options o;
  mmsd_options_default(&o);
  o.pcg_rtol = 1e-300;
  o.pcg_maxit = 1 << 30;
  o.terms = p->A.Nt ? MMSD_ALL : (MMSD_EXCH | MMSD_ANIS | MMSD_ZEEM);
  int rc = resolve(p, &o, &r);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(c->mu);
  MMSD_HIP(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const int B = 32;
  const int saved_stride = c->timing.stride;
  c->timing.stride = 0;
  hipEvent_t e0, e1;
  MMSD_HIP(hipEventCreate(&e0));
  MMSD_HIP(hipEventCreate(&e1));
  double best = 1e300;
  int best_l = p->lpr, best_b = c->max_blocks;
  for (int lpr : {4, 8, 16}) {
    int lastG = -1;
    for (int mb : {128, 256, 512, 1024, 2048}) {
      if ((rc = set_launch(p, lpr, mb))) break;
      if (p->G == lastG) continue;
      lastG = p->G;
      double t_best = 1e300;
      for (int rep = 0; rep < 2 && !rc; ++rep) {
        if ((rc = (p->precision == MMSD_MIXED ? snapshot<float>(p, 1, true) : snapshot<double>(p, 1, true)))) break;
        if ((rc = arm(p, r, ST_EVAL, 0))) break;
        std::vector<Table> tabs{{p->precision, p->dprob, p->dblk, 1, p->G, p->lpr}};
        MMSD_HIP(hipEventRecord(e0, st));
        if ((rc = issue(c, tabs, B, nullptr))) break;
        MMSD_HIP(hipEventRecord(e1, st));
        MMSD_HIP(hipEventSynchronize(e1));
        float ms = 0;
        MMSD_HIP(hipEventElapsedTime(&ms, e0, e1));
        t_best = std::min(t_best, (double)ms * 1e3 / B);
        if ((rc = (p->precision == MMSD_MIXED ? snapshot<float>(p, 1, false) : snapshot<double>(p, 1, false)))) break;
        MMSD_HIP(hipStreamSynchronize(st));
      }
      if (rc) break;
      if (t_best < best) {
        best = t_best;
        best_l = lpr;
        best_b = mb;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->timing.stride = saved_stride;
  if (rc) return rc;
  // leave the problem idle at the chosen shape
  if ((rc = set_launch(p, best_l, best_b))) return rc;
  c->tuned[key] = {best_l, best_b};
  if (lanes_out) *lanes_out = best_l;
  if (blocks_out) *blocks_out = best_b;
  if (us_out) *us_out = best;
  return MMSD_OK;
}

int mmsd_autotune_cache_get(mmsd_ctx c, int32_t* rec, int cap, int* n) {
  if (!c || !n || cap < 0 || (cap > 0 && !rec)) return invalid("bad autotune cache request");
  std::lock_guard<std::mutex> lk(c->mu);
  int k = 0;
  for (const auto& kv : c->tuned) {   // std::map: ascending keys
    if (k < cap) {
      int32_t* r = rec + 5 * (size_t)k;
      r[0] = (int32_t)(kv.first >> 40);
      r[1] = (int32_t)((kv.first >> 20) & 0xFFFFF);
      r[2] = (int32_t)(kv.first & 0xFFFFF);
      r[3] = kv.second.first;
      r[4] = kv.second.second;
    }
    ++k;
  }
  *n = k;
  return MMSD_OK;
}

int mmsd_autotune_cache_put(mmsd_ctx c, const int32_t* rec, int n) {
  if (!c || n < 0 || (n > 0 && !rec)) return invalid("bad autotune cache request");
  for (int k = 0; k < n; ++k) {
    const int32_t* r = rec + 5 * (size_t)k;
    if ((r[0] != MMSD_FP64 && r[0] != MMSD_MIXED) || r[1] < 0 || r[1] > 62 || r[2] < 0 || r[2] > 62 ||
        (r[3] != 4 && r[3] != 8 && r[3] != 16) || r[4] < 8 || r[4] > kMaxBlocks || r[4] % 8)
      return invalid("autotune cache record " + std::to_string(k) + " is not valid");
  }
  std::lock_guard<std::mutex> lk(c->mu);
  for (int k = 0; k < n; ++k) {
    const int32_t* r = rec + 5 * (size_t)k;
    c->tuned[tune_key(r[0], r[1], r[2])] = {r[3], r[4]};
  }
  return MMSD_OK;
}

int mmsd_assembly_export(const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, int64_t sizes[4],
                         int32_t* mrp, int32_t* mci, double* K, double* D1, double* D2, double* Q, double* V,
                         int32_t* pot_global, int32_t* lrp, int32_t* lci, double* L, double* scalars) {
  if (!sizes) return invalid("null sizes");
  Assembly A;
  std::string err;
  int rc = assemble(mesh, mats, n_mats, &A, &err);
  if (rc) {
    set_error(err);
    return rc;
  }
  const int64_t nnzM = (int64_t)A.mci.size(), nnzL = (int64_t)A.lci.size();
  sizes[0] = A.N;
  sizes[1] = nnzM;
  sizes[2] = A.Nt;
  sizes[3] = nnzL;
  auto put_i = [](int32_t* dst, const std::vector<int>& v) {
    if (dst) std::copy(v.begin(), v.end(), dst);
  };
  auto put_d = [](double* dst, const std::vector<double>& v) {
    if (dst) std::copy(v.begin(), v.end(), dst);
  };
  put_i(mrp, A.mrp);
  put_i(mci, A.mci);
  put_d(K, A.K);
  for (int c3 = 0; c3 < 3; ++c3) {
    if (D1) std::copy(A.D1[c3].begin(), A.D1[c3].end(), D1 + c3 * nnzM);
    if (D2) std::copy(A.D2[c3].begin(), A.D2[c3].end(), D2 + c3 * nnzM);
  }
  for (int c6 = 0; c6 < 6; ++c6)
    if (Q) std::copy(A.Q[c6].begin(), A.Q[c6].end(), Q + c6 * (int64_t)A.N);
  put_d(V, A.V);
  put_i(pot_global, A.pot_global);
  put_i(lrp, A.lrp);
  put_i(lci, A.lci);
  put_d(L, A.L);
  if (scalars) {
    scalars[0] = A.c_an;
    scalars[1] = A.vol;
    scalars[2] = A.Ms;
    scalars[3] = A.mu0Ms2;
  }
  return MMSD_OK;
}

int mmsd_get_state(mmsd_problem p, void* buf, size_t* bytes) {
  if (!p || !bytes) return invalid("null argument");
  const size_t N = p->A.N, Nt = p->A.Nt;
  const size_t need = 64 + 8 * (3 * N + Nt);
  if (!buf) {
    *bytes = need;
    return MMSD_OK;
  }
  if (*bytes < need) return invalid("state buffer too small");
  char* b = (char*)buf;
  std::memset(b, 0, 64);
  std::memcpy(b, "MMSDST01", 8);
  int64_t hdr[4] = {(int64_t)p->precision, (int64_t)N, (int64_t)Nt, 0};
  std::memcpy(b + 8, hdr, sizeof(hdr));
  std::memcpy(b + 40, p->b_ext, 24);
  int rc = mmsd_get_m(p, (double*)(b + 64));
  if (rc) return rc;
  double* u = (double*)(b + 64 + 24 * N);
  if (Nt) {
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    hipStream_t st = p->ctx->stream;
    if (p->precision == MMSD_MIXED) {
      std::vector<float> f(Nt);
      MMSD_HIP(hipMemcpyAsync(f.data(), desc_of<float>(p).u3[p->ucur], 4 * Nt, hipMemcpyDeviceToHost, st));
      MMSD_HIP(hipStreamSynchronize(st));
      for (size_t i = 0; i < Nt; ++i) u[i] = f[i];
    } else {
      MMSD_HIP(hipMemcpyAsync(u, desc_of<double>(p).u3[p->ucur], 8 * Nt, hipMemcpyDeviceToHost, st));
      MMSD_HIP(hipStreamSynchronize(st));
    }
  }
  *bytes = need;
  return MMSD_OK;
}

int mmsd_set_state(mmsd_problem p, const void* buf, size_t bytes) {
  if (!p || !buf) return invalid("null argument");
  const size_t N = p->A.N, Nt = p->A.Nt;
  const char* b = (const char*)buf;
  if (bytes < 64 || std::memcmp(b, "MMSDST01", 8)) return invalid("not a state buffer");
  int64_t hdr[4];
  std::memcpy(hdr, b + 8, sizeof(hdr));
  if (hdr[0] != p->precision || hdr[1] != (int64_t)N || hdr[2] != (int64_t)Nt || bytes < 64 + 8 * (3 * N + Nt))
    return invalid("state does not match this problem");
  double bf[3];
  std::memcpy(bf, b + 40, 24);
  int rc;
  {
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    (void)hipSetDevice(p->ctx->device);
    rc = p->precision == MMSD_MIXED ? copy_m_to_device<float>(p, (const double*)(b + 64), false)
                                    : copy_m_to_device<double>(p, (const double*)(b + 64), false);
  }
  if (rc || (rc = mmsd_set_field(p, bf))) return rc;
  if (Nt) {
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    hipStream_t st = p->ctx->stream;
    const double* u = (const double*)(b + 64 + 24 * N);
    if (p->precision == MMSD_MIXED) {
      std::vector<float> f(u, u + Nt);
      MMSD_HIP(hipMemcpyAsync(desc_of<float>(p).u3[p->ucur], f.data(), 4 * Nt, hipMemcpyHostToDevice, st));
      MMSD_HIP(hipStreamSynchronize(st));
    } else {
      MMSD_HIP(hipMemcpyAsync(desc_of<double>(p).u3[p->ucur], u, 8 * Nt, hipMemcpyHostToDevice, st));
      MMSD_HIP(hipStreamSynchronize(st));
    }
  }
  return MMSD_OK;
}

}  // extern "C"
