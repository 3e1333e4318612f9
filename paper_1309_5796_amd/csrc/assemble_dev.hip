// Device-side assembly of the operator values: the P1 tetrahedral
// exchange stiffness, the potential-coupling matrices, the lumped
// anisotropy tensors and volumes (Abstract: linear tetrahedral finite
// elements), and the transformed Laplacian of the scalar potential with its
// diagonal shell metric (Results, comparison section: the open boundary is
// handled by a space transformation).
//
// The host validates the mesh, numbers the nodes and builds the per-region
// material table (assemble_structure without patterns).  Kernels build the
// node-to-tet adjacency (count, fill, sort) and both sparsity patterns
// (k_pattern: sorted distinct columns of each row), then compute every
// value:
//   k_asm_geo        one thread per tet: volume, P1 gradients, shell metric
//   k_asm_magnet     one wavefront per magnetic row: V, D1, D2, K, Q
//   k_asm_potential  one wavefront per potential row: L and its diagonal check
// In a row kernel the lanes first load one tet each and stage its terms in
// LDS; then each row entry is summed by one lane, in the host assembly's
// order (the adjacency lists' order), so the sums need no atomics and are
// deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "assemble.h"
#include "mmsd.h"
#include "runtime.h"

namespace mmsd {
namespace {

constexpr int kAsmBlock = 256;
constexpr int kGeo = 16;   // doubles per tet: V, grad[4][3], shell metric T[3]
constexpr double kNmDev = 1e-9;

enum : unsigned char { TET_DEGENERATE = 1, TET_OUTSIDE_SHELL = 2 };

struct ShellDev {
  int on;
  double c[3], a[3], b[3];   // nm
};

// Volume and gradients of the barycentric functions: with D the matrix of
// edge vectors x_k - x_0 (k = 1..3), grad(lambda_k) is column k of D^-1 and
// grad(lambda_0) is minus the sum of the others.  The shell metric is the
// diagonal |det J| J^-1 J^-T of the per-axis map x = a (b - a) / (b - |t - c|)
// beyond |t - c| = a, taken at the centroid.
__global__ __launch_bounds__(kAsmBlock) void k_asm_geo(const double* __restrict__ xyz,
                                                       const int32_t* __restrict__ tets, int64_t E, ShellDev sh,
                                                       double* __restrict__ geo, unsigned char* __restrict__ flag) {
  const int64_t e = (int64_t)blockIdx.x * kAsmBlock + threadIdx.x;
  if (e >= E) return;
  int t[4];
  for (int k = 0; k < 4; ++k) t[k] = tets[4 * e + k];
  double D[3][3];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) D[k][c] = (xyz[3 * (int64_t)t[k + 1] + c] - xyz[3 * (int64_t)t[0] + c]) / kNmDev;
  const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  double sc = 0;
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) sc = fmax(sc, fabs(D[k][c]));
  unsigned char f = 0;
  double* G = geo + kGeo * e;
  if (!(fabs(det) > 1e-10 * sc * sc * sc)) {
    f |= TET_DEGENERATE;
    for (int k = 0; k < 13; ++k) G[k] = 0.0;
  } else {
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
    double g[4][3];
    for (int k = 1; k < 4; ++k)
      for (int c = 0; c < 3; ++c) g[k][c] = inv[c][k - 1];
    for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    G[0] = fabs(det) / 6.0;
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c) G[1 + 3 * k + c] = g[k][c];
  }
  double fp[3] = {1, 1, 1};
  if (sh.on) {
    for (int k = 0; k < 3; ++k) {
      double cen = 0;
      for (int v = 0; v < 4; ++v) cen += 0.25 * xyz[3 * (int64_t)t[v] + k] / kNmDev;
      const double d = fabs(cen - sh.c[k]);
      if (d > sh.a[k]) {
        if (!(d < sh.b[k])) f |= TET_OUTSIDE_SHELL;
        else fp[k] = sh.a[k] * (sh.b[k] - sh.a[k]) / ((sh.b[k] - d) * (sh.b[k] - d));
      }
    }
  }
  G[13] = fp[1] * fp[2] / fp[0];
  G[14] = fp[0] * fp[2] / fp[1];
  G[15] = fp[0] * fp[1] / fp[2];
  flag[e] = f;
}

constexpr int kWave = 64;

struct MagnetArgs {
  int N;
  int64_t nnz;
  const int32_t* mrp;
  const int32_t* mci;
  const int32_t* adj_ptr;     // magnetic node -> (magnetic tet << 2 | vertex)
  const int32_t* adj;
  const int32_t* mtet;        // [Em*4] magnetic-node ids
  const int32_t* mtet_mesh;   // [Em] mesh tet
  const int32_t* mregion;     // [Em]
  const double* reg;          // [8 per region]
  const double* geo;
  double mu0Ms2;
  double *K, *D1, *D2, *Q, *V;   // D1, D2: [3][nnz]; Q: [6][N]
};

// One magnetic row per block of one wavefront, in two phases per chunk of
// up to 64 of the row's tets: lane j loads tet j (adjacency, geometry,
// material) and writes its four (column, terms) records to LDS, so the
// row's gathers are all in flight at once; then each lane, owning one row
// entry (rows longer than 64 entries take several passes), adds the records
// of its column in adjacency order (the host assembly's order).  Lumped
// volume, D1/D2 (coupling to the potential's gradient), the exchange
// stiffness and the anisotropy tensor, each scaled by the row's volume as
// the host does.
__global__ __launch_bounds__(kWave) void k_asm_magnet(MagnetArgs a) {
  __shared__ int s_col[4 * kWave];
  __shared__ double s_t[4][4 * kWave];   // D2 x3 and K terms per (tet, vertex)
  __shared__ double s_d1[3][kWave];      // D1 terms per tet (the same for its four vertices)
  __shared__ double s_ve[kWave], s_kan[kWave];
  __shared__ int s_reg[kWave];
  const int lane = threadIdx.x;
  const int i = blockIdx.x;
  const int r0 = a.mrp[i], r1 = a.mrp[i + 1];
  const int k0 = a.adj_ptr[i], k1 = a.adj_ptr[i + 1];
  double V = 0, q[6] = {0, 0, 0, 0, 0, 0};
  for (int base = r0; base < r1; base += kWave) {
    const int p = base + lane;
    const int col = p < r1 ? a.mci[p] : -1;
    double kk = 0, d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
    for (int kb = k0; kb < k1; kb += kWave) {
      const int n = min(kWave, k1 - kb);
      if (lane < n) {
        const int e = a.adj[kb + lane] >> 2, va = a.adj[kb + lane] & 3;
        const double* G = a.geo + kGeo * (int64_t)a.mtet_mesh[e];
        const double Ve = G[0];
        const double* g = G + 1;
        const int reg = a.mregion[e];
        const double* R = a.reg + 8 * (int64_t)reg;
        const double qv = 0.25 * Ve;
        const double kex = R[0] * Ve;
        s_ve[lane] = Ve;
        s_kan[lane] = 0.25 * Ve * R[1] / a.mu0Ms2;
        s_reg[lane] = reg;
        for (int c = 0; c < 3; ++c) s_d1[c][lane] = qv * g[3 * va + c];
        for (int vb = 0; vb < 4; ++vb) {
          const int slot = 4 * lane + vb;
          s_col[slot] = a.mtet[4 * (int64_t)e + vb];
          for (int c = 0; c < 3; ++c) s_t[c][slot] = qv * g[3 * vb + c];
          const double dot = g[3 * va] * g[3 * vb] + g[3 * va + 1] * g[3 * vb + 1] + g[3 * va + 2] * g[3 * vb + 2];
          s_t[3][slot] = kex * dot;
        }
      }
      __syncthreads();
      for (int j = 0; j < n; ++j) {
        if (base == r0) {
          V += 0.25 * s_ve[j];
          const double* R = a.reg + 8 * (int64_t)s_reg[j];
          for (int c = 0; c < 6; ++c) q[c] += s_kan[j] * R[2 + c];
        }
        for (int vb = 0; vb < 4; ++vb) {
          const int slot = 4 * j + vb;
          if (s_col[slot] != col) continue;
          for (int c = 0; c < 3; ++c) {
            d1[c] += s_d1[c][j];
            d2[c] += s_t[c][slot];
          }
          kk += s_t[3][slot];
        }
      }
      __syncthreads();
    }
    const double s1 = 1.0 / V, s2 = 2.0 / V;
    if (p < r1) {
      for (int c = 0; c < 3; ++c) {
        a.D1[c * a.nnz + p] = d1[c];
        a.D2[c * a.nnz + p] = d2[c] * s1;
      }
      a.K[p] = kk * s2;
    }
    if (base == r0 && lane == 0) {
      for (int c = 0; c < 6; ++c) a.Q[c * (int64_t)a.N + i] = q[c] * s2;
      a.V[i] = V;
    }
  }
}

struct PotentialArgs {
  int Nt;
  const int32_t* lrp;
  const int32_t* lci;
  const int32_t* pot_global;
  const int32_t* pot_of;   // [n_nodes]
  const int32_t* tptr;     // mesh node -> (mesh tet << 2 | vertex)
  const int32_t* tlst;
  const int32_t* tets;
  const double* geo;
  double* L;
  unsigned char* bad;      // [Nt] 1 = diagonal missing or not positive
};

// One row of the transformed Laplacian per block of one wavefront, in the
// same two phases as the magnetic rows: lane j loads tet j of the node's
// adjacency and writes V_e grad(phi_a) . T_e grad(phi_b) for its four
// vertices (T_e the diagonal shell metric) with their columns to LDS; each
// lane then adds the records of its own entry's column in adjacency order.
__global__ __launch_bounds__(kWave) void k_asm_potential(PotentialArgs a) {
  __shared__ int s_col[4 * kWave];
  __shared__ double s_val[4 * kWave];
  const int lane = threadIdx.x;
  const int r = blockIdx.x;
  const int g = a.pot_global[r];
  const int r0 = a.lrp[r], r1 = a.lrp[r + 1];
  const int t0 = a.tptr[g], t1 = a.tptr[g + 1];
  bool diag_ok = false;
  for (int base = r0; base < r1; base += kWave) {
    const int p = base + lane;
    const int mine = p < r1 ? a.lci[p] : -1;
    double l = 0;
    for (int tb = t0; tb < t1; tb += kWave) {
      const int n = min(kWave, t1 - tb);
      if (lane < n) {
        const int64_t e = a.tlst[tb + lane] >> 2;
        const int va = a.tlst[tb + lane] & 3;
        const double* G = a.geo + kGeo * e;
        const double Ve = G[0];
        const double* gr = G + 1;
        const double* T = G + 13;
        for (int vb = 0; vb < 4; ++vb) {
          const int col = a.pot_of[a.tets[4 * e + vb]];
          s_col[4 * lane + vb] = col < 0 ? -2 : col;   // -2 matches no lane
          s_val[4 * lane + vb] = Ve * (gr[3 * va] * T[0] * gr[3 * vb] + gr[3 * va + 1] * T[1] * gr[3 * vb + 1] +
                                       gr[3 * va + 2] * T[2] * gr[3 * vb + 2]);
        }
      }
      __syncthreads();
      for (int j = 0; j < 4 * n; ++j)
        if (s_col[j] == mine) l += s_val[j];
      __syncthreads();
    }
    if (p < r1) a.L[p] = l;
    diag_ok = diag_ok || __ballot(p < r1 && mine == r && l > 0) != 0;
  }
  if (lane == 0) a.bad[r] = diag_ok ? 0 : 1;
}

// ---- structure: node-to-tet adjacency and sparsity patterns ----------

// Candidate columns of one row (4 per incident tet) held in LDS by the
// pattern kernel, 5 bytes each: at most 64 KB.
constexpr int kMaxCand = 13104;

__global__ __launch_bounds__(kAsmBlock) void k_asm_zero(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kAsmBlock + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Adjacency, first pass: the number of (tet, vertex) pairs at each node.
__global__ __launch_bounds__(kAsmBlock) void k_adj_count(const int32_t* __restrict__ tets, int64_t E,
                                                         int32_t* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * kAsmBlock + threadIdx.x;
  if (e >= E) return;
  for (int v = 0; v < 4; ++v) atomicAdd(&cnt[tets[4 * e + v]], 1);
}

// Second pass, after the prefix sum of the counts: each pair into its
// node's list (in arrival order; the third pass sorts).
__global__ __launch_bounds__(kAsmBlock) void k_adj_fill(const int32_t* __restrict__ tets, int64_t E,
                                                        const int32_t* __restrict__ ptr, int32_t* __restrict__ cur,
                                                        int32_t* __restrict__ lst) {
  const int64_t e = (int64_t)blockIdx.x * kAsmBlock + threadIdx.x;
  if (e >= E) return;
  for (int v = 0; v < 4; ++v) {
    const int node = tets[4 * e + v];
    lst[ptr[node] + atomicAdd(&cur[node], 1)] = (int)(4 * e + v);
  }
}

// Third pass: each node's list ascending in 4 tet + vertex, the order a
// serial pass over the tets gives (insertion sort: the lists are short).
__global__ __launch_bounds__(kAsmBlock) void k_adj_sort(const int32_t* __restrict__ ptr, int64_t n,
                                                        int32_t* __restrict__ lst) {
  const int64_t i = (int64_t)blockIdx.x * kAsmBlock + threadIdx.x;
  if (i >= n) return;
  const int a = ptr[i], b = ptr[i + 1];
  for (int j = a + 1; j < b; ++j) {
    const int x = lst[j];
    int k = j - 1;
    while (k >= a && lst[k] > x) {
      lst[k + 1] = lst[k];
      --k;
    }
    lst[k + 1] = x;
  }
}

struct PatternArgs {
  int R;
  const int32_t* row_node;   // node of row r; null: row r is node r
  const int32_t* adj_ptr;    // node -> (tet << 2 | vertex)
  const int32_t* adj;
  const int32_t* tets4;      // 4 node ids per tet
  const int32_t* col_of;     // column of a node, -1 = none; null: the node id is the column
  int32_t* cnt;              // [R] distinct columns (count pass)
  const int32_t* rp;         // row starts (write pass)
  int32_t* ci;               // columns, ascending per row (write pass)
  int cand;                  // 4 x the longest adjacency list: the LDS candidate slots
};

// The columns of row r are the distinct columns of the vertices of the
// tets around its node.  One 64-lane block per row: the lanes stage the
// 4 x (incident tets) candidates in LDS and mark first occurrences; the
// count pass sums the marks, the write pass puts each distinct column at
// its rank among them, so every row comes out sorted and unique.  The
// candidate list takes a.cand ints and a.cand bytes of dynamic LDS.
template <bool WRITE>
__global__ __launch_bounds__(kWave) void k_pattern(PatternArgs a) {
  extern __shared__ int s_dyn[];
  int* s_c = s_dyn;
  unsigned char* s_first = reinterpret_cast<unsigned char*>(s_dyn + a.cand);
  const int lane = threadIdx.x;
  const int r = blockIdx.x;
  const int g = a.row_node ? a.row_node[r] : r;
  const int k0 = a.adj_ptr[g];
  const int m = 4 * (a.adj_ptr[g + 1] - k0);   // at most a.cand <= kMaxCand (set and checked on the host)
  for (int j = lane; j < m; j += kWave) {
    const int e = a.adj[k0 + j / 4] >> 2;
    const int x = a.tets4[4 * (int64_t)e + (j & 3)];
    s_c[j] = a.col_of ? a.col_of[x] : x;
  }
  __syncthreads();
  for (int j = lane; j < m; j += kWave) {
    const int c = s_c[j];
    bool first = c >= 0;
    for (int i = 0; i < j && first; ++i) first = s_c[i] != c;
    s_first[j] = first ? 1 : 0;
  }
  __syncthreads();
  if (!WRITE) {
    int u = 0;
    for (int j = lane; j < m; j += kWave) u += s_first[j];
    for (int off = kWave / 2; off > 0; off >>= 1) u += __shfl_down(u, off);
    if (lane == 0) a.cnt[r] = u;
  } else {
    const int base = a.rp[r];
    for (int j = lane; j < m; j += kWave) {
      if (!s_first[j]) continue;
      const int c = s_c[j];
      int rank = 0;
      for (int i = 0; i < m; ++i) rank += (s_first[i] && s_c[i] < c) ? 1 : 0;
      a.ci[base + rank] = c;
    }
  }
}

// Device temporaries of one call.  Heap mode: from the context's allocator,
// freed (after the stream has drained) on every return.  Arena mode: carved
// in call order, 256-byte aligned, from a device region of `cap` bytes that
// the library owns for the life of the process (the allocation-free entry
// point); nothing is allocated or freed.
struct Scratch {
  mmsd_ctx_s* c;
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  std::vector<void*> ptrs;
  explicit Scratch(mmsd_ctx_s* ctx) : c(ctx) {}
  Scratch(mmsd_ctx_s* ctx, void* base, size_t bytes) : c(ctx), arena((char*)base), cap(bytes) {}
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  template <typename T>
  T* get(size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (arena) {
      const size_t at = (used + 255) & ~size_t(255);
      if (at + bytes > cap) return nullptr;
      used = at + bytes;
      return (T*)(arena + at);
    }
    void* p = c->dalloc(bytes);
    if (p) ptrs.push_back(p);
    return (T*)p;
  }
  ~Scratch() {
    (void)hipStreamSynchronize(c->stream);
    for (void* p : ptrs) c->dfree(p);
  }
};

// Bytes of the temporaries one call takes from an arena, in the order the
// call takes them (each piece 256-byte aligned).
size_t arena_bytes(int64_t N, int64_t Nt, int64_t E, int64_t Em, int64_t n_nodes, size_t n_reg, bool query) {
  size_t used = 0;
  auto take = [&](size_t n, size_t elem) {
    used = ((used + 255) & ~size_t(255)) + std::max<size_t>(n, 1) * elem;
  };
  take(4 * (size_t)Em, 4);                                   // magnetic tets
  take(N + 1, 4);                                            // their adjacency: row starts
  take(4 * (size_t)Em, 4);                                   // and lists
  take(std::max(n_nodes, std::max(N, Nt)), 4);               // counts / cursor
  if (query) take(std::max(N, Nt) + 1, 4);                   // row starts of the queried patterns
  take(4 * (size_t)E, 4);                                    // all tets
  if (Nt > 0) {
    take(n_nodes + 1, 4);                                    // node-to-tet adjacency
    take(4 * (size_t)E, 4);
    take(n_nodes, 4);                                        // potential row of each node
    if (query) take(Nt, 4);                                  // node of each potential row
  }
  if (query) return used;
  take(3 * (size_t)n_nodes, 8);                              // coordinates
  take(kGeo * (size_t)E, 8);                                 // geometry records
  take(E, 1);                                                // tet flags
  take(Em, 4);                                               // magnetic tets' mesh ids
  take(Em, 4);                                               // and regions
  take(n_reg, 8);                                            // material table
  if (Nt > 0) take(Nt, 1);                                   // diagonal checks
  return used;
}

template <typename T>
hipError_t put(T* dst, const std::vector<T>& v, hipStream_t s) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kAsmBlock - 1) / kAsmBlock); }

}  // namespace
}  // namespace mmsd

using namespace mmsd;

namespace mmsd {
namespace {

// Exclusive prefix sum of n device counts into ptr[n + 1] (on the host: the
// counts make one round trip); returns the total and the largest count.
int scan_counts(const int32_t* d_cnt, int64_t n, int32_t* d_ptr, hipStream_t st, int64_t* total, int* largest) {
  std::vector<int32_t> h(n + 1, 0);
  MMSD_HIP(hipMemcpyAsync(h.data() + 1, d_cnt, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MMSD_HIP(hipStreamSynchronize(st));
  int64_t acc = 0;
  int mx = 0;
  for (int64_t i = 1; i <= n; ++i) {
    mx = std::max(mx, h[i]);
    acc += h[i];
    if (acc > INT32_MAX) {
      set_error("device assembly: more than 2^31 entries");
      return MMSD_E_INVALID;
    }
    h[i] = (int32_t)acc;
  }
  if (d_ptr) MMSD_HIP(hipMemcpyAsync(d_ptr, h.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
  MMSD_HIP(hipStreamSynchronize(st));   // h is released on return
  *total = acc;
  if (largest) *largest = mx;
  return MMSD_OK;
}

// Node-to-(tet, vertex) adjacency of n nodes over E tets, into ptr[n + 1]
// and lst[4 E] (device); cur is an n-int temporary; *longest gets the
// longest list's length.
int build_adjacency(const int32_t* d_tets, int64_t E, int64_t n, int32_t* ptr, int32_t* lst, int32_t* cur,
                    hipStream_t st, int* longest) {
  k_asm_zero<<<grid_of(n), kAsmBlock, 0, st>>>(cur, n);
  k_adj_count<<<grid_of(E), kAsmBlock, 0, st>>>(d_tets, E, cur);
  MMSD_HIP(hipGetLastError());
  int64_t total = 0;
  int largest = 0;
  int rc = scan_counts(cur, n, ptr, st, &total, &largest);
  if (rc) return rc;
  if (4 * (int64_t)largest > kMaxCand) {
    set_error("device assembly: a node lies in more than " + std::to_string(kMaxCand / 4) + " tets");
    return MMSD_E_INVALID;
  }
  *longest = largest;
  k_asm_zero<<<grid_of(n), kAsmBlock, 0, st>>>(cur, n);
  k_adj_fill<<<grid_of(E), kAsmBlock, 0, st>>>(d_tets, E, ptr, cur, lst);
  k_adj_sort<<<grid_of(n), kAsmBlock, 0, st>>>(ptr, n, lst);
  MMSD_HIP(hipGetLastError());
  return MMSD_OK;
}

// Dynamic LDS bytes of a pattern launch: the candidate columns and their
// first-occurrence marks.
size_t pattern_lds(const PatternArgs& pa) { return (size_t)std::max(pa.cand, 4) * (sizeof(int) + 1); }

// Pattern of R rows, first pass: counts and row starts into rp[R + 1];
// returns the entry count.
int pattern_count(PatternArgs pa, int32_t* cnt, int32_t* rp, hipStream_t st, int64_t* nnz) {
  pa.cnt = cnt;
  k_pattern<false><<<(unsigned)pa.R, kWave, pattern_lds(pa), st>>>(pa);
  MMSD_HIP(hipGetLastError());
  return scan_counts(cnt, pa.R, rp, st, nnz, nullptr);
}

// Second pass: the columns, ascending per row, into ci[rp[R]].
int pattern_write(PatternArgs pa, const int32_t* rp, int32_t* ci, hipStream_t st) {
  pa.rp = rp;
  pa.ci = ci;
  k_pattern<true><<<(unsigned)pa.R, kWave, pattern_lds(pa), st>>>(pa);
  MMSD_HIP(hipGetLastError());
  return MMSD_OK;
}

}  // namespace
}  // namespace mmsd

// ---- the allocation-free variant's device region ---------------------------
// Temporaries of mmsd_assemble_device_noalloc live in this file-scope array
// (one copy per GPU, held until the process ends).  Host code must not pass
// its name to a kernel: it is resolved once per device with
// hipGetSymbolAddress and the resolved address is used everywhere.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace mmsd {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, which must be current.
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device id out of range for the allocation-free scratch table");
    return MMSD_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) {
      set_error("hipGetSymbolAddress(scratch) returned no address");
      return MMSD_E_HIP;
    }
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return MMSD_OK;
}

enum class Outputs { QUERY, CALLER, OWNED };

// The device assembly.  QUERY: sizes only.  CALLER: into the eleven device
// arrays of `o`, sized by sizes[].  OWNED: `o`'s arrays are allocated here,
// from the context's allocator, as their sizes become known (the caller
// releases them).  S_keep, when set, receives the host structure.
int assemble_device_run(mmsd_ctx c, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                        int64_t sizes[4], DeviceAssembly* o, Outputs mode, bool no_alloc,
                        AssemblyStructure* S_keep) {
  if (!c || !sizes) {
    set_error("null context or sizes");
    return MMSD_E_INVALID;
  }
  if (n_mats < 0 || (n_mats > 0 && !mats)) {
    set_error("bad material table");
    return MMSD_E_INVALID;
  }
  const bool query = mode == Outputs::QUERY;
  // host: validation, numbering, magnetic tets, material table
  AssemblyStructure S;
  std::string err;
  int rc = assemble_structure(mesh, mats, n_mats, &S, &err, /*with_patterns=*/false);
  if (rc) {
    set_error(err);
    return rc;
  }
  const int64_t N = S.N, Nt = S.Nt, E = S.E, Em = (int64_t)S.mregion.size(), n_nodes = mesh->n_nodes;
  // the assemble call gets the query's sizes back: the output buffers' sizes
  const int64_t cap[4] = {sizes[0], sizes[1], sizes[2], sizes[3]};
  if (mode == Outputs::CALLER && (cap[0] != N || cap[2] != Nt)) {
    set_error("device assembly: sizes[] does not hold this mesh's sizes (query them first)");
    return MMSD_E_INVALID;
  }
  // the row kernels launch one 64-lane block per row: grid threads must fit 32 bits
  if (N > (int64_t(1) << 26) || Nt > (int64_t(1) << 26)) {
    set_error("device assembly: more than 2^26 rows");
    return MMSD_E_INVALID;
  }

  std::lock_guard<std::mutex> lk(c->mu);
  MMSD_HIP(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  std::unique_ptr<Scratch> heap_or_arena;
  if (no_alloc) {
    const size_t need = arena_bytes(N, Nt, E, Em, n_nodes, S.reg.size(), query);
    if (need > kNoAllocScratchBytes) {
      set_error("mmsd_assemble_device_noalloc: this mesh needs " + std::to_string(need) +
                " bytes of device temporaries, above the fixed " + std::to_string(kNoAllocScratchBytes) +
                " (use mmsd_assemble_device)");
      return MMSD_E_INVALID;
    }
    void* base = nullptr;
    if ((rc = scratch_address(c->device, &base))) return rc;
    heap_or_arena.reset(new Scratch(c, base, kNoAllocScratchBytes));
  } else {
    heap_or_arena.reset(new Scratch(c));
  }
  Scratch& tmp = *heap_or_arena;
  // an output array of n elements (OWNED mode)
  auto own = [&](auto*& slot, size_t n) {
    using T = std::remove_reference_t<decltype(*slot)>;
    void* q = c->dalloc(std::max<size_t>(n, 1) * sizeof(T));
    if (q) o->owned.push_back(q);
    slot = (T*)q;
    return q != nullptr;
  };
  auto nomem = [] {
    set_error("device allocation failed (assembly)");
    return MMSD_E_NOMEM;
  };
  auto mismatch = [] {
    set_error("device assembly: sizes[] does not hold this mesh's sizes (query them first)");
    return MMSD_E_INVALID;
  };
  // device structure: adjacency and patterns
  int32_t* d_mtet = tmp.get<int32_t>(4 * (size_t)Em);
  int32_t* d_madj_ptr = tmp.get<int32_t>(N + 1);
  int32_t* d_madj = tmp.get<int32_t>(4 * (size_t)Em);
  int32_t* d_cur = tmp.get<int32_t>(std::max(n_nodes, std::max(N, Nt)));
  int32_t* d_rp = query ? tmp.get<int32_t>(std::max(N, Nt) + 1) : nullptr;
  if (!d_mtet || !d_madj_ptr || !d_madj || !d_cur || (query && !d_rp)) return nomem();
  if (mode == Outputs::OWNED && (!own(o->mrp, N + 1) || !own(o->lrp, Nt + 1))) return nomem();
  MMSD_HIP(put(d_mtet, S.mtet, st));
  int longest = 0;
  if ((rc = build_adjacency(d_mtet, Em, N, d_madj_ptr, d_madj, d_cur, st, &longest))) return rc;
  int64_t nnzM = 0, nnzL = 0;
  PatternArgs pm{(int)N, nullptr, d_madj_ptr, d_madj, d_mtet, nullptr, nullptr, nullptr, nullptr, 4 * longest};
  if ((rc = pattern_count(pm, d_cur, query ? d_rp : o->mrp, st, &nnzM))) return rc;
  if (mode == Outputs::CALLER && nnzM != cap[1]) return mismatch();
  if (mode == Outputs::OWNED && !own(o->mci, nnzM)) return nomem();
  if (!query && (rc = pattern_write(pm, o->mrp, o->mci, st))) return rc;
  int32_t *d_tets = nullptr, *d_tptr = nullptr, *d_tlst = nullptr, *d_pot_of = nullptr, *d_pot_global = nullptr;
  d_tets = tmp.get<int32_t>(4 * (size_t)E);
  if (!d_tets) return nomem();
  MMSD_HIP(hipMemcpyAsync(d_tets, mesh->tets, 4 * E * sizeof(int32_t), hipMemcpyHostToDevice, st));
  if (Nt > 0) {
    d_tptr = tmp.get<int32_t>(n_nodes + 1);
    d_tlst = tmp.get<int32_t>(4 * (size_t)E);
    d_pot_of = tmp.get<int32_t>(n_nodes);
    if (mode == Outputs::OWNED && !own(o->pot_global, Nt)) return nomem();
    d_pot_global = query ? tmp.get<int32_t>(Nt) : o->pot_global;
    if (!d_tptr || !d_tlst || !d_pot_of || !d_pot_global) return nomem();
    MMSD_HIP(put(d_pot_of, S.pot_of, st));
    MMSD_HIP(put(d_pot_global, S.pot_global, st));
    if ((rc = build_adjacency(d_tets, E, n_nodes, d_tptr, d_tlst, d_cur, st, &longest))) return rc;
    PatternArgs pp{(int)Nt, d_pot_global, d_tptr, d_tlst, d_tets, d_pot_of, nullptr, nullptr, nullptr, 4 * longest};
    if ((rc = pattern_count(pp, d_cur, query ? d_rp : o->lrp, st, &nnzL))) return rc;
    if (mode == Outputs::CALLER && nnzL != cap[3]) return mismatch();
    if (mode == Outputs::OWNED && !own(o->lci, nnzL)) return nomem();
    if (!query && (rc = pattern_write(pp, o->lrp, o->lci, st))) return rc;
  }
  sizes[0] = N;
  sizes[1] = nnzM;
  sizes[2] = Nt;
  sizes[3] = nnzL;
  if (query) return MMSD_OK;
  if (mode == Outputs::OWNED) {
    o->N = N;
    o->nnzM = nnzM;
    o->Nt = Nt;
    o->nnzL = nnzL;
    if (!own(o->K, nnzM) || !own(o->D1, 3 * (size_t)nnzM) || !own(o->D2, 3 * (size_t)nnzM) ||
        !own(o->Q, 6 * (size_t)N) || !own(o->V, N) || !own(o->L, nnzL))
      return nomem();
  }

  // geometry, shell metric and validity of every tet
  double* d_xyz = tmp.get<double>(3 * (size_t)n_nodes);
  double* d_geo = tmp.get<double>(kGeo * (size_t)E);
  unsigned char* d_flag = tmp.get<unsigned char>(E);
  int32_t* d_mtet_mesh = tmp.get<int32_t>(Em);
  int32_t* d_mregion = tmp.get<int32_t>(Em);
  double* d_reg = tmp.get<double>(S.reg.size());
  if (!d_xyz || !d_geo || !d_flag || !d_mtet_mesh || !d_mregion || !d_reg) return nomem();
  MMSD_HIP(hipMemcpyAsync(d_xyz, mesh->xyz, 3 * n_nodes * sizeof(double), hipMemcpyHostToDevice, st));
  ShellDev sh{};
  sh.on = mesh->shell != nullptr;
  if (sh.on)
    for (int k = 0; k < 3; ++k) {
      sh.c[k] = mesh->shell[k] / kNmDev;
      sh.a[k] = mesh->shell[3 + k] / kNmDev;
      sh.b[k] = mesh->shell[6 + k] / kNmDev;
    }
  k_asm_geo<<<grid_of(E), kAsmBlock, 0, st>>>(d_xyz, d_tets, E, sh, d_geo, d_flag);
  MMSD_HIP(hipGetLastError());
  std::vector<unsigned char> flag(E);
  MMSD_HIP(hipMemcpyAsync(flag.data(), d_flag, E, hipMemcpyDeviceToHost, st));
  MMSD_HIP(hipStreamSynchronize(st));
  for (int64_t e = 0; e < E; ++e)
    if (flag[e] & TET_DEGENERATE) {
      set_error("mesh: degenerate tetrahedron " + std::to_string(e));
      return MMSD_E_MESH;
    }
  if (Nt > 0)
    for (int64_t e = 0; e < E; ++e)
      if (flag[e] & TET_OUTSIDE_SHELL) {
        set_error("mesh: tetrahedron outside the transformation shell");
        return MMSD_E_MESH;
      }

  // values
  MMSD_HIP(put(d_mtet_mesh, S.mtet_mesh, st));
  MMSD_HIP(put(d_mregion, S.mregion, st));
  MMSD_HIP(put(d_reg, S.reg, st));
  MagnetArgs ma{(int)N, nnzM, o->mrp, o->mci, d_madj_ptr, d_madj, d_mtet, d_mtet_mesh, d_mregion, d_reg, d_geo,
                S.mu0Ms2, o->K, o->D1, o->D2, o->Q, o->V};
  k_asm_magnet<<<(unsigned)N, kWave, 0, st>>>(ma);
  MMSD_HIP(hipGetLastError());
  if (Nt > 0) {
    unsigned char* d_bad = tmp.get<unsigned char>(Nt);
    if (!d_bad) return nomem();
    PotentialArgs pa{(int)Nt, o->lrp, o->lci, o->pot_global, d_pot_of, d_tptr, d_tlst, d_tets, d_geo, o->L, d_bad};
    k_asm_potential<<<(unsigned)Nt, kWave, 0, st>>>(pa);
    MMSD_HIP(hipGetLastError());
    std::vector<unsigned char> bad(Nt);
    MMSD_HIP(hipMemcpyAsync(bad.data(), d_bad, Nt, hipMemcpyDeviceToHost, st));
    MMSD_HIP(hipStreamSynchronize(st));
    for (int64_t r = 0; r < Nt; ++r)
      if (bad[r]) {
        set_error("mesh: potential matrix has a non-positive diagonal");
        return MMSD_E_MESH;
      }
  } else {
    // no potential problem: lrp still holds its single zero
    static const int32_t zero = 0;
    MMSD_HIP(hipMemcpyAsync(o->lrp, &zero, sizeof(int32_t), hipMemcpyHostToDevice, st));
  }
  MMSD_HIP(hipStreamSynchronize(st));
  if (S_keep) *S_keep = std::move(S);
  return MMSD_OK;
}

int assemble_device_impl(mmsd_ctx c, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                         int64_t sizes[4], int32_t* mrp, int32_t* mci, double* K, double* D1, double* D2,
                         double* Q, double* V, int32_t* pot_global, int32_t* lrp, int32_t* lci, double* L,
                         bool no_alloc) {
  const void* outs[11] = {mrp, mci, K, D1, D2, Q, V, pot_global, lrp, lci, L};
  const int given = (int)std::count_if(outs, outs + 11, [](const void* p) { return p != nullptr; });
  if (given != 0 && given != 11) {
    set_error("output pointers must be all null (size query) or all set");
    return MMSD_E_INVALID;
  }
  DeviceAssembly o;
  o.mrp = mrp;
  o.mci = mci;
  o.K = K;
  o.D1 = D1;
  o.D2 = D2;
  o.Q = Q;
  o.V = V;
  o.pot_global = pot_global;
  o.lrp = lrp;
  o.lci = lci;
  o.L = L;
  return assemble_device_run(c, mesh, mats, n_mats, sizes, &o, given == 0 ? Outputs::QUERY : Outputs::CALLER,
                             no_alloc, nullptr);
}

}  // namespace
}  // namespace mmsd

// ---- device-assembled operators into a problem's arena ----------------------

namespace mmsd {
namespace {

template <typename real>
__global__ __launch_bounds__(kAsmBlock) void k_to_real(const double* __restrict__ src, real* __restrict__ dst,
                                                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kAsmBlock + threadIdx.x;
  if (i < n) dst[i] = (real)src[i];
}

// The potential matrix into the 64-row sliced layout: one thread per row of
// the padded slices.  Slice s holds w_s = (so[s+1] - so[s]) / 64 columns
// per row, column k of its row r at so[s] + 64 k + r; a row's entries past
// its length (and the rows past the last) get column min(row, n - 1) and
// value 0.  Each real row also gets its FP64 row sum and the reciprocal of
// its diagonal, written into the d field of both CG record buffers.
template <typename real>
__global__ __launch_bounds__(kAsmBlock) void k_slice_rows(const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const double* __restrict__ v,
                                                           const int32_t* __restrict__ so, int64_t n,
                                                           int32_t* __restrict__ sc, real* __restrict__ sv,
                                                           real* __restrict__ lsum, real* __restrict__ rec0,
                                                           real* __restrict__ rec1) {
  const int64_t i = (int64_t)blockIdx.x * kAsmBlock + threadIdx.x;
  const int64_t sl = i >> 6;
  if (sl >= (n + 63) / 64) return;
  const int r = (int)(i & 63);
  const int w = (so[sl + 1] - so[sl]) / 64;
  const int a = i < n ? rp[i] : 0, len = i < n ? rp[i + 1] - a : 0;
  const int pad = (int)(i < n - 1 ? i : n - 1);
  double sum = 0, dinv = 0;
  for (int k = 0; k < w; ++k) {
    const int64_t q = so[sl] + 64LL * k + r;
    if (k < len) {
      const int c = ci[a + k];
      const double x = v[a + k];
      sc[q] = c;
      sv[q] = (real)x;
      sum += x;
      if (c == i) dinv = 1.0 / x;
    } else {
      sc[q] = pad;
      sv[q] = (real)0;
    }
  }
  if (i < n) {
    lsum[i] = (real)sum;
    rec0[4 * i + 3] = (real)dinv;
    rec1[4 * i + 3] = (real)dinv;
  }
}

}  // namespace

template <typename real>
hipError_t launch_to_real(const double* src, real* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_to_real<real><<<grid_of(n), kAsmBlock, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_slice_rows(const int32_t* rp, const int32_t* ci, const double* v, const int32_t* so, int64_t n,
                             int32_t* sc, real* sv, real* lsum, real* rec0, real* rec1, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_slice_rows<real><<<grid_of(64 * ((n + 63) / 64)), kAsmBlock, 0, s>>>(rp, ci, v, so, n, sc, sv, lsum, rec0, rec1);
  return hipGetLastError();
}

template hipError_t launch_to_real<float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_to_real<double>(const double*, double*, int64_t, hipStream_t);
template hipError_t launch_slice_rows<float>(const int32_t*, const int32_t*, const double*, const int32_t*, int64_t,
                                             int32_t*, float*, float*, float*, float*, hipStream_t);
template hipError_t launch_slice_rows<double>(const int32_t*, const int32_t*, const double*, const int32_t*,
                                              int64_t, int32_t*, double*, double*, double*, double*, hipStream_t);

}  // namespace mmsd

namespace mmsd {

void DeviceAssembly::release(mmsd_ctx_s* c) {
  if (!owned.empty()) (void)hipStreamSynchronize(c->stream);
  for (void* q : owned) c->dfree(q);
  owned.clear();
  *this = DeviceAssembly();
}

int assemble_device_owned(mmsd_ctx_s* c, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                          DeviceAssembly* out, AssemblyStructure* S) {
  int64_t sizes[4] = {0, 0, 0, 0};
  const int rc = assemble_device_run(c, mesh, mats, n_mats, sizes, out, Outputs::OWNED, false, S);
  if (rc) out->release(c);
  return rc;
}

}  // namespace mmsd

extern "C" int mmsd_assemble_device(mmsd_ctx c, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                                    int64_t sizes[4], int32_t* mrp, int32_t* mci, double* K, double* D1,
                                    double* D2, double* Q, double* V, int32_t* pot_global, int32_t* lrp,
                                    int32_t* lci, double* L) {
  return assemble_device_impl(c, mesh, mats, n_mats, sizes, mrp, mci, K, D1, D2, Q, V, pot_global, lrp, lci, L,
                              false);
}

extern "C" int mmsd_assemble_device_noalloc(mmsd_ctx c, const mmsd_mesh* mesh, const mmsd_material* mats,
                                            int n_mats, int64_t sizes[4], int32_t* mrp, int32_t* mci, double* K,
                                            double* D1, double* D2, double* Q, double* V, int32_t* pot_global,
                                            int32_t* lrp, int32_t* lci, double* L) {
  return assemble_device_impl(c, mesh, mats, n_mats, sizes, mrp, mci, K, D1, D2, Q, V, pot_global, lrp, lci, L,
                              true);
}

