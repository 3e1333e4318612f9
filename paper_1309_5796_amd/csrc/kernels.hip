// Step kernel of the curvilinear steepest-descent minimizer for gfx950.
//
// One launch advances every unfinished problem of a table by one phase (see
// device.h for the phases and the parity protocol).  Work layout:
//  * Rows of the potential matrix (and of multigrid matrices with many short
//    rows) are swept one per thread from a 64-row sliced layout: a wavefront
//    owns a slice, so index and value loads are contiguous 64-wide accesses.
//  * Other CSR rows (magnet matrices, coarse multigrid levels) are split over
//    `LPR` lanes (4, 8 or 16) of a 64-wide wavefront.  A block of 512 threads
//    walks a contiguous chunk of rows in passes.  Node vectors are gathered
//    (they stay in L2: every entry is reused by ~15 rows); values gathered
//    together are packed into records.
//  * Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8);
//    the row chunks are cut into 8 contiguous runs, one per XCD, so that
//    neighbour gathers stay inside an XCD's own L2 and every XCD gets an
//    equal share also of a coarse level's few chunks.
//  * Reductions are deterministic and need no atomics: wavefront butterfly,
//    then the 8 waves in order, one partial per block; the next launch's
//    blocks each combine those G partials in the same fixed order.
// All node arrays are structure-of-arrays.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "mmsd.h"

namespace mmsd {
namespace {

// Sums (and the max) over groups of W consecutive lanes of a wavefront,
// the result in every lane of the group: a butterfly whose steps are VALU
// cross-lane moves (CDNA4) instead of LDS permutes: quad permutations for
// lane distances 1 and 2, the half-row and row mirrors for 4 and 8 (after
// the earlier steps every lane of a quad, then of a half-row, holds the same
// partial, so a mirror partner holds what the xor partner would), and the
// 16- and 32-lane permlane swaps.  Each step adds two partials, so every
// lane of the group ends with the same value.
namespace xl {
constexpr int kXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kHalfMirror = 0x141; // row_half_mirror
constexpr int kMirror = 0x140;     // row_mirror

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// {lower, upper}: the values of lane l and of lane l ^ 16 (S = 16) or
// l ^ 32 (S = 32), the one of the lower row (half) first
template <int S>
__device__ __forceinline__ void swap_pair(float x, float& a, float& b) {
  const int v = __float_as_int(x);
  const auto r = S == 16 ? __builtin_amdgcn_permlane16_swap(v, v, false, false)
                         : __builtin_amdgcn_permlane32_swap(v, v, false, false);
  a = __int_as_float(r[0]);
  b = __int_as_float(r[1]);
}
template <int S>
__device__ __forceinline__ void swap_pair(double x, double& a, double& b) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const auto rl = S == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                          : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto rh = S == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                          : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  a = __hiloint2double(rh[0], rl[0]);
  b = __hiloint2double(rh[1], rl[1]);
}
template <typename T, int W, bool MAX>
__device__ __forceinline__ T reduce(T v) {
  auto op = [](T p, T q) { return MAX ? fmax(p, q) : p + q; };
  if constexpr (W >= 2) v = op(v, dpp<kXor1>(v));
  if constexpr (W >= 4) v = op(v, dpp<kXor2>(v));
  if constexpr (W >= 8) v = op(v, dpp<kHalfMirror>(v));
  if constexpr (W >= 16) v = op(v, dpp<kMirror>(v));
  if constexpr (W >= 32) {
    T a, b;
    swap_pair<16>(v, a, b);
    v = op(a, b);
  }
  if constexpr (W >= 64) {
    T a, b;
    swap_pair<32>(v, a, b);
    v = op(a, b);
  }
  return v;
}
}  // namespace xl

template <typename T, int W>
__device__ __forceinline__ T group_sum(T v) {
  return xl::reduce<T, W, false>(v);
}

__device__ __forceinline__ double wave_sum(double v) { return xl::reduce<double, 64, false>(v); }

__device__ __forceinline__ double wave_max(double v) { return xl::reduce<double, 64, true>(v); }

// Explicit solution of the curvilinear step m+ = m - tau (m + m+)/2 x H
// (eq. (8)): with a = (tau/2) H and c = a x m, m+ = m + 2 (c + a x c) / (1 + a.a).
// ht = tau / 2.  In FP32 the result is renormalized to keep |m| = 1 at
// single-precision rounding.
template <typename real>
__device__ __forceinline__ void cayley(real mx, real my, real mz, real Hx, real Hy, real Hz, real ht,
                                       real& ox, real& oy, real& oz) {
  if (ht == real(0)) {
    ox = mx;
    oy = my;
    oz = mz;
    return;
  }
  const real ax = ht * Hx, ay = ht * Hy, az = ht * Hz;
  const real cx = ay * mz - az * my, cy = az * mx - ax * mz, cz = ax * my - ay * mx;
  const real dx = ay * cz - az * cy, dy = az * cx - ax * cz, dz = ax * cy - ay * cx;
  const real f = real(2) / (real(1) + ax * ax + ay * ay + az * az);
  ox = mx + f * (cx + dx);
  oy = my + f * (cy + dy);
  oz = mz + f * (cz + dz);
  if constexpr (std::is_same<real, float>::value) {
    const float s = rsqrtf(ox * ox + oy * oy + oz * oz);
    ox *= s;
    oy *= s;
    oz *= s;
  }
}

// Row loops load kUnroll column indices per lane first, then issue all the
// gathers, then accumulate: two dependent memory round trips per row batch
// instead of two per nonzero.
constexpr int kUnroll = 4;
// The FIELD phase gathers four values per neighbour (m and u) and takes half
// the batch in FP64 to bound its register use (the kernel's VGPR count is
// the largest phase's).
template <typename real>
constexpr int kUnrollWide = sizeof(real) == 8 ? 2 : 4;

// Record loads and stores through global pointers, as one vector access each.
template <typename real>
using vec2 = real __attribute__((ext_vector_type(2)));
template <typename real>
using vec4 = real __attribute__((ext_vector_type(4)));
template <typename real>
__device__ __forceinline__ Pair<real> ld(DevPtr<const Pair<real>> p, int i) {
  const vec2<real> v = reinterpret_cast<DevPtr<const vec2<real>>>(p)[i];
  return Pair<real>{v.x, v.y};
}
template <typename real>
__device__ __forceinline__ void st(DevPtr<Pair<real>> p, int i, Pair<real> x) {
  reinterpret_cast<DevPtr<vec2<real>>>(p)[i] = vec2<real>{x.a, x.b};
}
template <typename real>
__device__ __forceinline__ Rec<real> ld(DevPtr<const Rec<real>> p, int i) {
  const vec4<real> v = reinterpret_cast<DevPtr<const vec4<real>>>(p)[i];
  Rec<real> r;
  r.r = v.x;
  r.s = v.y;
  r.w = v.z;
  r.d = v.w;
  return r;
}
template <typename real>
__device__ __forceinline__ void st(DevPtr<Rec<real>> p, int i, const Rec<real>& x) {
  reinterpret_cast<DevPtr<vec4<real>>>(p)[i] = vec4<real>{x.r, x.s, x.w, x.d};
}

// Rows of block `blk` (of G, a multiple of 8) for R rows, as passes of
// `rpp` rows starting at r0, r0 + rs, ... below r1 (row i of a pass is valid
// when i < r1).  The rows are cut into chunks of ceil(R / G) rounded up to
// `align` (64 for the sliced layout, whose wavefronts each own one slice),
// and to whole passes when a chunk takes more than one, so a small level
// spreads over up to G blocks.  The chunks are dealt to the 8 XCDs (block b
// runs on XCD b % 8) as 8 contiguous runs of almost equal length: each XCD
// sweeps neighbouring rows, which keeps their gathers in its own L2, and all
// 8 XCDs share the work also when there are fewer chunks than blocks.  When
// a chunk takes several passes, the blocks of an XCD take the passes of the
// XCD's run in turn (block k the passes k, k + n, k + 2n, ... of its n
// blocks) instead of one contiguous chunk each: the XCD then sweeps its run
// as one front of n passes, so a row's neighbours a grid plane away (tens
// of thousands of rows on the largest meshes) were just loaded by the front
// and are still in the L2 when they are gathered.
__device__ __forceinline__ void chunk_rows(int R, int G, int blk, int rpp, int align, int& r0, int& r1, int& rs) {
  r0 = r1 = R;
  rs = rpp;
  if (R <= 0) return;
  long long c = ((long long)R + G - 1) / G;
  c = (c + align - 1) / align * align;
  if (c > rpp) c = (c + rpp - 1) / rpp * rpp;
  const int nch = (int)((R + c - 1) / c);          // <= G
  const int x = blk & 7, k = blk >> 3;
  const int s = x * nch / 8, e = (x + 1) * nch / 8;
  if (k >= e - s) return;
  if (c <= rpp) {   // one pass: the block's own chunk
    const long long a = (long long)(s + k) * c;
    r0 = (int)a;
    r1 = (int)(a + c < R ? a + c : R);
    return;
  }
  const long long a = (long long)s * c, b = (long long)e * c;
  r0 = (int)(a + (long long)k * rpp);
  r1 = (int)(b < R ? b : R);
  rs = (e - s) * rpp;
}

// Matrix entries of the sliced sweeps are read once per sweep.  On problems
// whose potential matrix exceeds the Infinity Cache they are streamed with the
// non-temporal hint (nt), so that they do not push the gathered vectors and
// the coarse levels' data out of the L2 (polycrystal: -6% per launch); on
// smaller ones, which the Infinity Cache holds, the plain loads are faster.
template <bool NT, typename T>
__device__ __forceinline__ T stream_ld(DevPtr<const T> p, int i) {
  if constexpr (NT) return __builtin_nontemporal_load(p + i);
  else return p[i];
}

// Rows of the potential matrix are swept one per thread from its 64-row
// sliced layout: a wavefront owns one slice, so every index and value load
// is one contiguous 64-wide access, and a whole block-pass covers 512 rows.
constexpr int kSellU = 4;   // entries per thread loaded before their gathers

// sum_k v[k] * g(column k) over row i of a matrix in the sliced layout
// (slice offsets so, columns sc, values sv).  The calling wavefront's active
// lanes all lie in one slice.
template <typename real, bool NT, typename G>
__device__ __forceinline__ real sell_row_t(DevPtr<const int> so, DevPtr<const int> sc, DevPtr<const real> sv, int i,
                                           G&& g) {
  const int sl = __builtin_amdgcn_readfirstlane(i >> 6);
  const int o0 = so[sl];
  const int w = (so[sl + 1] - o0) >> 6;
  const int o = o0 + (i & 63);
  real acc = 0;
  for (int k0 = 0; k0 < w; k0 += kSellU) {
    int j[kSellU];
    real v[kSellU];
#pragma unroll
    for (int u = 0; u < kSellU; ++u) {
      const bool ok = k0 + u < w;
      const int q = o + 64 * (ok ? k0 + u : 0);
      j[u] = stream_ld<NT>(sc, q);
      v[u] = ok ? stream_ld<NT>(sv, q) : real(0);
    }
    real x[kSellU];
#pragma unroll
    for (int u = 0; u < kSellU; ++u) x[u] = g(j[u]);
#pragma unroll
    for (int u = 0; u < kSellU; ++u) acc += v[u] * x[u];
  }
  return acc;
}

// Row i of the sliced fused matrix Q: {sum (A P)_ik g(k), sum P_ik g(k)}
// from one gather per entry; P's values cover the first wp entries of the
// row (sliced with offsets po), the (A P) values all of them.
template <typename real, bool NT, typename G>
__device__ __forceinline__ Pair<real> sell_row_q_t(DevPtr<const int> so, DevPtr<const int> sc, DevPtr<const real> sv,
                                                   DevPtr<const int> po, DevPtr<const real> pv, int i, G&& g) {
  const int sl = __builtin_amdgcn_readfirstlane(i >> 6);
  const int o0 = so[sl], p0 = po[sl];
  const int w = (so[sl + 1] - o0) >> 6, wp = (po[sl + 1] - p0) >> 6;
  const int o = o0 + (i & 63), op = p0 + (i & 63);
  real sa = 0, sb = 0;
  for (int k0 = 0; k0 < w; k0 += kSellU) {
    int j[kSellU];
    real va[kSellU], vb[kSellU];
#pragma unroll
    for (int u = 0; u < kSellU; ++u) {
      const int k = k0 + u;
      const bool ok = k < w;
      const int q = o + 64 * (ok ? k : 0);
      j[u] = stream_ld<NT>(sc, q);
      va[u] = ok ? stream_ld<NT>(sv, q) : real(0);
      vb[u] = k < wp ? stream_ld<NT>(pv, op + 64 * k) : real(0);
    }
    real x[kSellU];
#pragma unroll
    for (int u = 0; u < kSellU; ++u) x[u] = g(j[u]);
#pragma unroll
    for (int u = 0; u < kSellU; ++u) {
      sa += va[u] * x[u];
      sb += vb[u] * x[u];
    }
  }
  return Pair<real>{sa, sb};
}

// The sliced sweeps with the problem's load form (a uniform branch: both
// loops are compiled, one runs).
template <typename real, typename G>
__device__ __forceinline__ real sell_row(DevPtr<const int> so, DevPtr<const int> sc, DevPtr<const real> sv, int i,
                                         bool nt, G&& g) {
  return nt ? sell_row_t<real, true>(so, sc, sv, i, g) : sell_row_t<real, false>(so, sc, sv, i, g);
}
template <typename real, typename G>
__device__ __forceinline__ Pair<real> sell_row_q(DevPtr<const int> so, DevPtr<const int> sc, DevPtr<const real> sv,
                                                 DevPtr<const int> po, DevPtr<const real> pv, int i, bool nt,
                                                 G&& g) {
  return nt ? sell_row_q_t<real, true>(so, sc, sv, po, pv, i, g) : sell_row_q_t<real, false>(so, sc, sv, po, pv, i, g);
}

// ... over row i of the potential matrix
template <typename real, typename G>
__device__ __forceinline__ real sell_sum(const ProbDev<real>& P, int i, G&& g) {
  return sell_row<real>(P.lso, P.lsc, P.lsv, i, P.stream != 0, g);
}

// ---- PREP: trial magnetization, Poisson right-hand side, initial residual ----
// Over the block's chunk of rows, first the magnet rows with LPR lanes per
// row: the trial m_t (Cayley step, also recomputed at magnet neighbours) and
// b = D1 m_t, stored in the residual slot; then every potential row, one
// thread per row over the sliced matrix: r = b - L u.  The block barrier
// between the two orders each row's b before its reuse (same block).
template <typename real, int LPR>
__device__ void phase_prep(const ProbDev<real>& P, const Ctrl* C, int blk, double* acc) {
  constexpr int RPP = kBlock / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  const int slot = threadIdx.x / LPR;
  const bool demag = C->demag != 0;
  const bool amg = C->precond == PC_AMG;
  const int R = demag ? P.Nt : P.N;
  int r0, r1, rs;
  chunk_rows(R, P.G, blk, kBlock, 64, r0, r1, rs);
  const int a = C->acc, tr = 1 - a;
  const real ht = real(0.5 * C->tau);
  DevPtr<const real> __restrict__ max_ = P.m[a][0];
  DevPtr<const real> __restrict__ may = P.m[a][1];
  DevPtr<const real> __restrict__ maz = P.m[a][2];
  DevPtr<const real> __restrict__ Hax = P.H[a][0];
  DevPtr<const real> __restrict__ Hay = P.H[a][1];
  DevPtr<const real> __restrict__ Haz = P.H[a][2];
  DevPtr<real> __restrict__ r2 = P.r2[C->rcur];
  DevPtr<Rec<real>> __restrict__ rec = P.rec[C->pcur];
  const int m1 = r1 < P.N ? r1 : P.N;
  for (int pass = r0; pass < m1; pass += rs)
  for (int base = pass; base < pass + kBlock && base < m1; base += RPP) {
    const int i = base + slot;
    const bool valid = i < m1;
    real bi = 0;
    if (valid) {
      if (lane == 0) {
        real ox, oy, oz;
        cayley<real>(max_[i], may[i], maz[i], Hax[i], Hay[i], Haz[i], ht, ox, oy, oz);
        P.m[tr][0][i] = ox;
        P.m[tr][1][i] = oy;
        P.m[tr][2][i] = oz;
      }
      if (demag) {
        const int k1 = P.mrp[i + 1];
        for (int k = P.mrp[i] + lane; k < k1; k += LPR) {
          const int j = P.mci[k];
          real ox, oy, oz;
          cayley<real>(max_[j], may[j], maz[j], Hax[j], Hay[j], Haz[j], ht, ox, oy, oz);
          bi += P.D1[0][k] * ox + P.D1[1][k] * oy + P.D1[2][k] * oz;
        }
      }
    }
    if (demag) {
      bi = group_sum<real, LPR>(bi);
      if (valid && lane == 0) {
        if (amg) r2[i] = bi;
        else rec[i].r = bi;
      }
    }
  }
  if (!demag) return;
  __syncthreads();
  // warm start of the solve: the accepted state's potential, or after a
  // rejected trial (tau halved) the interpolation between the accepted and
  // the rejected trial's potentials at the halved step, which leaves only the
  // curvature of the Cayley curve in the starting residual.  It is written to
  // the solve's working buffer while L u is formed from it.
  DevPtr<const real> __restrict__ ua = P.u3[C->u_src];
  DevPtr<const real> __restrict__ ub = C->u_src2 >= 0 ? P.u3[C->u_src2] : ua;
  DevPtr<real> __restrict__ uw = P.u3[C->ucur];
  const bool interp = C->u_src2 >= 0;
  const real wr = real(C->u_w);
  auto u_at = [&](int j) -> real { return interp ? ua[j] + wr * (ub[j] - ua[j]) : ua[j]; };
  for (int base = r0; base < r1; base += rs) {
    const int i = base + threadIdx.x;
    if (i >= r1) continue;
    const real bi = i < P.N ? (amg ? r2[i] : rec[i].r) : real(0);
    const real ui = u_at(i);
    uw[i] = ui;
    // FP32: the potential is large and smooth next to its residual, and the
    // rounding of the matrix values times u would swamp b - L u; L's rows sum
    // to zero away from the Dirichlet boundary, so the sum is taken over
    // differences u_j - u_i plus the (exactly assembled) row sum times u_i
    real lu;
    if constexpr (std::is_same<real, float>::value)
      lu = sell_sum(P, i, [&](int j) { return u_at(j) - ui; }) + P.lsum[i] * ui;
    else
      lu = sell_sum(P, i, [&](int j) { return u_at(j); });
    const real ri = bi - lu;
    if (amg) r2[i] = ri;
    else rec[i].r = ri;
    acc[0] += (double)bi * (double)bi;
    acc[1] += (double)ri * (double)ri;
    acc[2] += (double)ri * (double)ui;
  }
}

// ---- CG0: w = L D^-1 r for the starting residual (one thread per row) ----
template <typename real, int LPR>
__device__ void phase_cg0(const ProbDev<real>& P, const Ctrl* C, int blk, double* acc) {
  constexpr int RPP = kBlock;
  int r0, r1, rs;
  chunk_rows(P.Nt, P.G, blk, RPP, 64, r0, r1, rs);
  DevPtr<Rec<real>> __restrict__ rec = P.rec[C->pcur];
  for (int base = r0; base < r1; base += rs) {
    const int i = base + threadIdx.x;
    if (i >= r1) continue;
    const Rec<real> own = ld<real>(rec, i);
    const real sw = sell_sum(P, i, [&](int j) {
      const Rec<real> nb = ld<real>(rec, j);
      return nb.d * nb.r;
    });
    const real ui = own.d * own.r;
    rec[i].w = sw;
    acc[0] += (double)own.r * (double)ui;
    acc[1] += (double)sw * (double)ui;
  }
}

// ---- CG: one single-reduction PCG iteration (one thread per row) ----
// Reads records of buffer c = pcur (r_i, s_{i-1}, w_i) and writes buffer
// 1 - c.  A gathered neighbour's new residual is recomputed as
// r_j - alpha (w_j + beta s_j), so the sweep needs no grid-wide barrier
// between the vector updates and w = L D^-1 r.
template <typename real, int LPR>
__device__ void phase_cg(const ProbDev<real>& P, const Ctrl* C, int blk, double* acc) {
  constexpr int RPP = kBlock;
  int r0, r1, rs;
  chunk_rows(P.Nt, P.G, blk, RPP, 64, r0, r1, rs);
  const int c = C->pcur;
  const real alpha = real(C->alpha), beta = real(C->beta);
  DevPtr<const Rec<real>> __restrict__ ro = P.rec[c];
  DevPtr<Rec<real>> __restrict__ rn = P.rec[1 - c];
  for (int base = r0; base < r1; base += rs) {
    const int i = base + threadIdx.x;
    if (i >= r1) continue;
    const Rec<real> own = ld<real>(ro, i);
    real pi = P.p[i];
    real ui = P.u3[C->ucur][i];
    const real sw = sell_sum(P, i, [&](int j) {
      const Rec<real> nb = ld<real>(ro, j);
      return nb.d * (nb.r - alpha * (nb.w + beta * nb.s));
    });
    pi = own.d * own.r + beta * pi;
    const real si = own.w + beta * own.s;
    ui = ui + alpha * pi;
    const real ri = own.r - alpha * si;
    const real zi = own.d * ri;
    P.p[i] = pi;
    P.u3[C->ucur][i] = ui;
    Rec<real> out;
    out.r = ri;
    out.s = si;
    out.w = sw;
    out.d = own.d;
    st<real>(rn, i, out);
    acc[0] += (double)ri * (double)zi;
    acc[1] += (double)sw * (double)zi;
    acc[2] += (double)ri * (double)ri;
    acc[3] += (double)ri * (double)ui;
  }
}

// The level descriptors, copied to LDS by every block in the prologue
// (their loads then travel with the control block's instead of after it).
__shared__ __align__(16) unsigned char s_lev_raw[kMaxLevels * sizeof(MgLevelDev<double>)];
static_assert(sizeof(MgLevelDev<double>) == sizeof(MgLevelDev<float>) && sizeof(MgLevelDev<double>) % 8 == 0,
              "level descriptors are copied as 8-byte words");
template <typename real>
__device__ __forceinline__ const MgLevelDev<real>& lev_of(int l) {
  return reinterpret_cast<const MgLevelDev<real>*>(s_lev_raw)[l];
}

// ---- multigrid-preconditioned CG ----
// Lane-partial sum over row i of a CSR matrix of v[k] * g(column): column
// indices and values first, then all the gathers, then the products.
template <typename real, int LPR, int U = kUnroll, typename G>
__device__ __forceinline__ real row_sum(DevPtr<const int> __restrict__ rp, DevPtr<const int> __restrict__ ci,
                                        DevPtr<const real> __restrict__ v, int i, int lane, G&& g) {
  real acc = 0;
  const int ke = rp[i + 1];
  for (int k0 = rp[i] + lane; k0 < ke; k0 += U * LPR) {
    int j[U];
    real lv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * LPR;
      const int ks = k < ke ? k : k0;
      j[u] = ci[ks];
      lv[u] = k < ke ? v[ks] : real(0);
    }
    real x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = g(j[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += lv[u] * x[u];
  }
  return acc;
}

// The same over a matrix with two values per entry {a, b}: returns
// {sum a * g, sum b * g} from one gather per entry.
template <typename real, int LPR, int U, typename G>
__device__ __forceinline__ Pair<real> row_sum2(DevPtr<const int> __restrict__ rp, DevPtr<const int> __restrict__ ci,
                                               DevPtr<const Pair<real>> __restrict__ v, int i, int lane, G&& g) {
  real sa = 0, sb = 0;
  const int ke = rp[i + 1];
  for (int k0 = rp[i] + lane; k0 < ke; k0 += U * LPR) {
    int j[U];
    Pair<real> lv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * LPR;
      const int ks = k < ke ? k : k0;
      j[u] = ci[ks];
      lv[u] = k < ke ? ld<real>(v, ks) : Pair<real>{0, 0};
    }
    real x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = g(j[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      sa += lv[u].a * x[u];
      sb += lv[u].b * x[u];
    }
  }
  return Pair<real>{sa, sb};
}

// One operation of the symmetric V(1,1) cycle with damped-Jacobi smoothing
// (x = wd b before the coarse correction, one sweep after it):
//   DOWN(l)  res = b - A (wd b); on the levels l >= 1 where the host finds
//            it pays, the same launch also restricts, b_{l+1} = M b with
//            M = R (I - A wd) (a share of the blocks sweeps M's rows), and
//            REST(l) is skipped; on the last level, with the host's dense
//            Ainv M, those blocks form x_c = (Ainv M) b and SOLVE is skipped
//   REST(l)  b_{l+1} = R res (and wb_{l+1} = wd_{l+1} b_{l+1}, what DOWN and
//            POST of level l + 1 gather)
//   SOLVE    x_c = A_c^-1 b_c (dense)
//   POST(l)  coarse correction and post-smoothing in one sweep:
//            xa = wd b + P x_{l+1}, xb = xa + wd (b - A xa).  Since
//            A xa = A (wd b) + (A P) x_{l+1} and DOWN left res = b - A (wd b),
//            xb = xa + wd (res - (A P) x_{l+1}): one sweep of the matrix with
//            the pattern of A P and the value pairs {(A P)_ik, P_ik} (P's
//            pattern lies inside A P's) over x_{l+1}.  At level 0 the result
//            is z, stored in the {z, p} records (whole records are written:
//            p is carried over), and b.z is reduced.
// W lanes share a row (4, 8, 16 or 32, chosen per matrix by the host); W = 1
// (one thread per row) reads the operation's matrix in the sliced layout,
// in which matrices with many short rows are held (the level-0 operator is
// the potential matrix).  A lane loads 8 entries per batch with 8 or more lanes (matrices
// with long rows), kUnroll with 4 (8 for Q's value pairs: the 39k-row level-1
// post-smoothing of the 80 nm cube then takes one batch per row, 0.5 us
// faster; R and A at 4 lanes measured no faster with 8).
template <int W>
constexpr int kRowU = W >= 8 ? 8 : kUnroll;

template <typename real, int W, typename G>
__device__ __forceinline__ real a_row(const MgLevelDev<real>& L, int i, int lane, bool nt, G&& g) {
  if constexpr (W == 1) return sell_row<real>(L.aso, L.asc, L.asv, i, nt, g);
  else return row_sum<real, W, kRowU<W>>(L.arp, L.aci, L.av, i, lane, g);
}
template <typename real, int W, typename G>
__device__ __forceinline__ Pair<real> q_row(const MgLevelDev<real>& L, int i, int lane, bool nt, G&& g) {
  if constexpr (W == 1) return sell_row_q<real>(L.qso, L.qsc, L.qsv, L.qpo, L.qpv, i, nt, g);
  else return row_sum2<real, W, W == 4 ? 8 : kUnroll>(L.qrp, L.qci, L.qv, i, lane, g);   // two values per entry
}
template <typename real, int W, typename G>
__device__ __forceinline__ real r_row(const MgLevelDev<real>& L, int i, int lane, bool nt, G&& g) {
  if constexpr (W == 1) return sell_row<real>(L.rso, L.rsc, L.rsv, i, nt, g);
  else return row_sum<real, W, kRowU<W>>(L.rrp, L.rci, L.rv, i, lane, g);
}

template <typename real, int W, typename G>
__device__ __forceinline__ real m_row(const MgLevelDev<real>& L, int i, int lane, G&& g) {
  return row_sum<real, W, kRowU<W>>(L.mrp, L.mci, L.mv, i, lane, g);
}

// Rows of operation `op` on level l, block blk of the G blocks that share
// them.
template <typename real, int W>
__device__ void mg_rows(const ProbDev<real>& P, const Ctrl* C, const MgLevelDev<real>& L, int op, int l, int blk,
                        int G, double* acc) {
  constexpr int RPP = kBlock / W;
  const int lane = threadIdx.x & (W - 1);
  const int slot = threadIdx.x / W;
  DevPtr<const real> __restrict__ b = l == 0 ? P.r2[C->rcur] : L.b;
  DevPtr<const real> __restrict__ wd = L.wd;
  DevPtr<const real> __restrict__ wb = L.wb;
  const bool last = l + 1 == P.n_lev;
  const bool nt = P.stream != 0;
  int r0, r1, rs;
  if (op == MG_REST || op == MG_RESTM) {
    DevPtr<real> __restrict__ bn = last ? P.bc : lev_of<real>(l + 1).b;
    DevPtr<real> __restrict__ wbn = last ? nullptr : lev_of<real>(l + 1).wb;
    DevPtr<const real> __restrict__ wdn = last ? nullptr : lev_of<real>(l + 1).wd;
    DevPtr<const real> __restrict__ res = L.res;
    const bool m = op == MG_RESTM;   // b_{l+1} = M b, else R res
    // a sliced R holds its rows in a windowed order: position i is row ri
    DevPtr<const int> __restrict__ ord = W == 1 ? L.rord : nullptr;
    chunk_rows(L.n_next, G, blk, RPP, W == 1 ? 64 : 1, r0, r1, rs);
    for (int base = r0; base < r1; base += rs) {
      const int i = base + slot;
      const bool valid = i < r1;
      const int ri = (valid && ord) ? ord[i] : i;
      // the row's own values: before the sweep when rows are in place, after
      // it when their index comes from the row order (so that its load does
      // not hold up the sweep's)
      real wi = (valid && lane == 0 && !last && !ord) ? wdn[i] : real(0);
      real sum = 0;
      if (valid)
        sum = m ? m_row<real, W>(L, i, lane, [&](int j) { return b[j]; })
                : r_row<real, W>(L, i, lane, nt, [&](int j) { return res[j]; });
      sum = group_sum<real, W>(sum);
      if (valid && lane == 0) {
        if (ord && !last) wi = wdn[ri];
        bn[ri] = sum;
        if (!last) wbn[ri] = wi * sum;
      }
    }
    return;
  }
  chunk_rows(L.n, G, blk, RPP, W == 1 ? 64 : 1, r0, r1, rs);
  if (op == MG_DOWN) {
    DevPtr<const int> __restrict__ ord = W == 1 ? L.aord : nullptr;   // windowed row order of a sliced A
    for (int base = r0; base < r1; base += rs) {
      const int i = base + slot;
      const bool valid = i < r1;
      const int ri = (valid && ord) ? ord[i] : i;
      real bi = (valid && lane == 0 && !ord) ? b[i] : real(0);   // (as in REST)
      real sum = valid ? a_row<real, W>(L, i, lane, nt, [&](int j) { return l == 0 ? wd[j] * b[j] : wb[j]; })
                       : real(0);
      sum = group_sum<real, W>(sum);
      if (valid && lane == 0) {
        if (ord) bi = b[ri];
        L.res[ri] = bi - sum;
      }
    }
  } else {   // MG_POST
    DevPtr<const real> __restrict__ xn = last ? P.xc : lev_of<real>(l + 1).xb;
    DevPtr<const real> __restrict__ res = L.res;
    DevPtr<const int> __restrict__ ord = W == 1 ? L.qord : nullptr;   // windowed row order of a sliced Q
    for (int base = r0; base < r1; base += rs) {
      const int i = base + slot;
      const bool valid = i < r1;
      const int ri = (valid && ord) ? ord[i] : i;
      real bi = 0, wi = 0, rr = 0, pold = 0;
      auto own = [&](int r) {   // (as in REST)
        bi = b[r];
        wi = wd[r];
        rr = res[r];
        if (l == 0) pold = P.zp[r].b;
      };
      if (valid && lane == 0 && !ord) own(i);
      Pair<real> sum = valid ? q_row<real, W>(L, i, lane, nt, [&](int j) { return xn[j]; }) : Pair<real>{0, 0};
      sum.a = group_sum<real, W>(sum.a);
      sum.b = group_sum<real, W>(sum.b);
      if (valid && lane == 0) {
        if (ord) own(ri);
        const real xai = wi * bi + sum.b;
        const real zi = xai + wi * (rr - sum.a);
        if (l == 0) {
          st<real>(P.zp, ri, Pair<real>{zi, pold});
          acc[0] += (double)bi * (double)zi;
        } else {
          L.xb[ri] = zi;
        }
      }
    }
  }
}

// The row layout of an operation's matrix picks the kernel variant.
template <typename real>
__device__ __forceinline__ void mg_dispatch(const ProbDev<real>& P, const Ctrl* C, const MgLevelDev<real>& L, int op, int l,
                            int blk, int G, double* acc) {
  const int lanes = op == MG_REST    ? L.lanes_r
                    : op == MG_RESTM ? L.lanes_m
                    : op == MG_POST  ? L.lanes_q
                                     : L.lanes_a;
  const bool sliced = op == MG_REST    ? L.rso != nullptr
                      : op == MG_RESTM ? false
                      : op == MG_POST  ? L.qso != nullptr
                                       : L.aso != nullptr;
  if (sliced)
    mg_rows<real, 1>(P, C, L, op, l, blk, G, acc);
  else if (lanes == 32)
    mg_rows<real, 32>(P, C, L, op, l, blk, G, acc);
  else if (lanes == 16)
    mg_rows<real, 16>(P, C, L, op, l, blk, G, acc);
  else if (lanes == 8)
    mg_rows<real, 8>(P, C, L, op, l, blk, G, acc);
  else
    mg_rows<real, 4>(P, C, L, op, l, blk, G, acc);
}

// x_c = (Ainv M) b_l on the last level: one dense row per block at a time,
// streamed coalesced by the whole block, wavefront sums, then the waves in
// order.
template <typename real>
__device__ void coarse_rows(const ProbDev<real>& P, const MgLevelDev<real>& L, int blk, int G) {
  __shared__ double s_row[kBlock / 64];
  const int nc = P.nc, n = L.n;
  DevPtr<const real> __restrict__ b = L.b;
  const int wid = threadIdx.x >> 6, lid = threadIdx.x & 63;
  for (int i = blk; i < nc; i += G) {
    DevPtr<const real> __restrict__ row = P.AinvM + (size_t)i * n;
    double sum = 0;
    for (int j = threadIdx.x; j < n; j += kBlock) sum += (double)(row[j] * b[j]);
    sum = wave_sum(sum);
    if (lid == 0) s_row[wid] = sum;
    __syncthreads();
    double v = s_row[0];
    for (int w = 1; w < kBlock / 64; ++w) v += s_row[w];
    if (threadIdx.x == 0) P.xc[i] = real(v);
    __syncthreads();
  }
}

template <typename real, int LPR>
__device__ void phase_mg(const ProbDev<real>& P, const Ctrl* C, int op, int l, int blk, double* acc) {
  if (op == MG_SOLVE) {
    // dense coarsest solve: one row per block at a time, the whole block
    // streams the row coalesced, then wavefront sums and the waves in order
    __shared__ double s_row[kBlock / 64];
    const int nc = P.nc;
    const int wid = threadIdx.x >> 6, lid = threadIdx.x & 63;
    for (int i = blk; i < nc; i += P.G) {
      DevPtr<const real> __restrict__ row = P.Ainv + (size_t)i * nc;
      double sum = 0;
      for (int j = threadIdx.x; j < nc; j += kBlock) sum += (double)(row[j] * P.bc[j]);
      sum = wave_sum(sum);
      if (lid == 0) s_row[wid] = sum;
      __syncthreads();
      double v = s_row[0];
      for (int w = 1; w < kBlock / 64; ++w) v += s_row[w];
      if (threadIdx.x == 0) P.xc[i] = real(v);
      __syncthreads();
    }
    return;
  }
  const MgLevelDev<real>& L = lev_of<real>(l);
  int o = op, b = blk, g = P.G, passes = 1;
  if (op == MG_DOWN && L.m_blocks > 0) {
    // fused restriction: the last gm blocks sweep M, the others A; with
    // too few blocks to split, every block does both, one after the other
    if (g >= 16) {
      int gm = (g * L.m_blocks / 512 + 7) / 8 * 8;
      gm = gm < 8 ? 8 : gm > g - 8 ? g - 8 : gm;
      if (blk >= g - gm) {
        o = MG_RESTM;
        b = blk - (g - gm);
        g = gm;
      } else {
        g -= gm;
      }
    } else {
      passes = 2;
    }
  }
  for (int k = 0; k < passes; ++k) {
    const int ok = k == 0 ? o : MG_RESTM;
    if (ok == MG_RESTM && P.AinvM && l + 1 == P.n_lev)
      coarse_rows<real>(P, L, b, g);   // x_c = (Ainv M) b
    else
      mg_dispatch<real>(P, C, L, ok, l, b, g, acc);
  }
}

// PCG_A: p = z + beta p_old (recomputed at gathered neighbours from the
// {z, p} records), q = L p, p.q; also the {wd r, wd q} records PCG_B gathers.
// p itself is stored by PCG_B, which gathers no {z, p} record.  One thread
// per row.
template <typename real, int LPR>
__device__ void phase_pcg_a(const ProbDev<real>& P, const Ctrl* C, int blk, double* acc) {
  constexpr int RPP = kBlock;
  int r0, r1, rs;
  chunk_rows(P.Nt, P.G, blk, RPP, 64, r0, r1, rs);
  const real beta = real(C->beta);
  const bool first = C->beta == 0.0;
  DevPtr<const Pair<real>> __restrict__ zp = P.zp;
  DevPtr<const real> __restrict__ r = P.r2[C->rcur];
  DevPtr<const real> __restrict__ wd = lev_of<real>(0).wd;
  for (int base = r0; base < r1; base += rs) {
    const int i = base + threadIdx.x;
    if (i >= r1) continue;
    const Pair<real> own = ld<real>(zp, i);
    const real ri = r[i], wi = wd[i];
    // beta = 0 starts a solve: the p half then holds the previous solve's
    // direction and is not read
    const real sum = sell_sum(P, i, [&](int j) {
      const Pair<real> e = ld<real>(zp, j);
      return first ? e.a : e.a + beta * e.b;
    });
    const real pi = first ? own.a : own.a + beta * own.b;
    P.q[i] = sum;
    st<real>(P.rq, i, Pair<real>{wi * ri, wi * sum});
    acc[0] += (double)pi * (double)sum;
  }
}

// PCG_B: p = z + beta p_old (stored), r -= alpha q, u += alpha p, then the
// finest pre-smoothing residual of the next V-cycle, res = r - L (wd r),
// with neighbours' wd r_new recomputed from their {wd r, wd q} records.
// Partials: r.r, r.u.  One thread per row.
template <typename real, int LPR>
__device__ void phase_pcg_b(const ProbDev<real>& P, const Ctrl* C, int blk, double* acc) {
  constexpr int RPP = kBlock;
  int r0, r1, rs;
  chunk_rows(P.Nt, P.G, blk, RPP, 64, r0, r1, rs);
  const real alpha = real(C->alpha), beta = real(C->beta);
  const bool first = C->beta == 0.0;
  DevPtr<Pair<real>> __restrict__ zp = P.zp;
  DevPtr<const real> __restrict__ ro = P.r2[C->rcur];
  DevPtr<real> __restrict__ rn = P.r2[1 - C->rcur];
  DevPtr<const real> __restrict__ q = P.q;
  DevPtr<const Pair<real>> __restrict__ rq = P.rq;
  DevPtr<real> __restrict__ U = P.u3[C->ucur];
  for (int base = r0; base < r1; base += rs) {
    const int i = base + threadIdx.x;
    if (i >= r1) continue;
    const real roi = ro[i], qi = q[i], uo = U[i];
    const Pair<real> own = ld<real>(zp, i);
    const real sum = sell_sum(P, i, [&](int j) {
      const Pair<real> e = ld<real>(rq, j);
      return e.a - alpha * e.b;
    });
    const real pi = first ? own.a : own.a + beta * own.b;
    st<real>(zp, i, Pair<real>{own.a, pi});
    const real ri = roi - alpha * qi;
    const real ui = uo + alpha * pi;
    rn[i] = ri;
    U[i] = ui;
    lev_of<real>(0).res[i] = ri - sum;
    acc[0] += (double)ri * (double)ri;
    acc[1] += (double)ri * (double)ui;
  }
}

// ---- FIELD: effective field, torque, fused reductions ----
template <typename real, int LPR>
__device__ void phase_field(const ProbDev<real>& P, const Ctrl* C, int blk, double* acc) {
  constexpr int RPP = kBlock / LPR;
  constexpr int kU = kUnrollWide<real>;
  const int lane = threadIdx.x & (LPR - 1);
  const int slot = threadIdx.x / LPR;
  // FP32: the rows of K and D2 sum to zero (the P1 gradients of an element
  // sum to zero), so the sums are taken over differences from the row's own
  // node, sum_j K_ij (m_j - m_i) and sum_j D2_ij (u_j - u_i): the large
  // diagonal no longer cancels against its neighbours in single precision.
  constexpr bool kDiff = std::is_same<real, float>::value;
  int r0, r1, rs;
  chunk_rows(P.N, P.G, blk, RPP, RPP, r0, r1, rs);
  const int a = C->acc, tr = 1 - a;
  const int terms = C->terms;
  const bool exch = terms & MMSD_EXCH, anis = terms & MMSD_ANIS, zeem = terms & MMSD_ZEEM;
  const bool demag = C->demag != 0;
  const real bzx = zeem ? real(C->bz[0]) : real(0);
  const real bzy = zeem ? real(C->bz[1]) : real(0);
  const real bzz = zeem ? real(C->bz[2]) : real(0);
  DevPtr<const real> __restrict__ mx = P.m[tr][0];
  DevPtr<const real> __restrict__ my = P.m[tr][1];
  DevPtr<const real> __restrict__ mz = P.m[tr][2];
  // the row group's 13 running sums live in LDS, not in registers, during the
  // sweep (same additions in the same order)
  __shared__ double s_facc[RPP][kNPart];
  double* fa = s_facc[slot];
  if (lane == 0)
    for (int k = 0; k < kNPart; ++k) fa[k] = 0.0;
  for (int base = r0; base < r1; base += rs) {
    const int i = base + slot;
    const bool valid = i < r1;
    real kx = 0, ky = 0, kz = 0, dx = 0, dy = 0, dz = 0;
    real oi0 = 0, oi1 = 0, oi2 = 0, oiu = 0;   // own values subtracted in the difference form
    if (kDiff && valid) {
      oi0 = mx[i];
      oi1 = my[i];
      oi2 = mz[i];
      if (demag) oiu = P.u3[C->ucur][i];
    }
    if (valid) {
      const int ke = P.mrp[i + 1];
      for (int k0 = P.mrp[i] + lane; k0 < ke; k0 += kU * LPR) {
        int j[kU];
        bool ok[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int k = k0 + u * LPR;
          ok[u] = k < ke;
          j[u] = P.mci[ok[u] ? k : k0];
        }
        if (exch) {
          real kv[kU], gx[kU], gy[kU], gz[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int k = ok[u] ? k0 + u * LPR : k0;
            kv[u] = ok[u] ? P.K[k] : real(0);
            gx[u] = mx[j[u]] - oi0;
            gy[u] = my[j[u]] - oi1;
            gz[u] = mz[j[u]] - oi2;
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            kx += kv[u] * gx[u];
            ky += kv[u] * gy[u];
            kz += kv[u] * gz[u];
          }
        }
        if (demag) {
          real ex[kU], ey[kU], ez[kU], uj[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int k = ok[u] ? k0 + u * LPR : k0;
            const real f = ok[u] ? real(1) : real(0);
            ex[u] = f * P.D2[0][k];
            ey[u] = f * P.D2[1][k];
            ez[u] = f * P.D2[2][k];
            uj[u] = P.u3[C->ucur][j[u]] - oiu;
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            dx += ex[u] * uj[u];
            dy += ey[u] * uj[u];
            dz += ez[u] * uj[u];
          }
        }
      }
    }
    kx = group_sum<real, LPR>(kx);
    ky = group_sum<real, LPR>(ky);
    kz = group_sum<real, LPR>(kz);
    dx = group_sum<real, LPR>(dx);
    dy = group_sum<real, LPR>(dy);
    dz = group_sum<real, LPR>(dz);
    if (valid && lane == 0) {
      const real m0 = mx[i], m1 = my[i], m2 = mz[i];
      real ax = 0, ay = 0, az = 0;
      if (anis) {
        ax = P.Q[0][i] * m0 + P.Q[3][i] * m1 + P.Q[4][i] * m2;
        ay = P.Q[3][i] * m0 + P.Q[1][i] * m1 + P.Q[5][i] * m2;
        az = P.Q[4][i] * m0 + P.Q[5][i] * m1 + P.Q[2][i] * m2;
      }
      const real hx = -kx - dx + ax + bzx;
      const real hy = -ky - dy + ay + bzy;
      const real hz = -kz - dz + az + bzz;
      const real Hx = m1 * hz - m2 * hy, Hy = m2 * hx - m0 * hz, Hz = m0 * hy - m1 * hx;
      P.H[tr][0][i] = Hx;
      P.H[tr][1][i] = Hy;
      P.H[tr][2][i] = Hz;
      if (C->store_h) {
        P.h[0][i] = hx;
        P.h[1][i] = hy;
        P.h[2][i] = hz;
      }
      const double V = (double)P.V[i];
      fa[FP_EEX] += 0.5 * V * (double)(m0 * kx + m1 * ky + m2 * kz);
      if constexpr (kDiff) {
        // FP32: the anisotropy energy sum_e V_e K1_e - m.Q m cancels for m
        // near the easy axis; for unit m it equals m.(tr(Q) I - Q) m, whose
        // matrix has no large entries along the axis
        if (anis) {
          const real t0 = P.Q[1][i] + P.Q[2][i], t1 = P.Q[0][i] + P.Q[2][i], t2 = P.Q[0][i] + P.Q[1][i];
          const real q = t0 * m0 * m0 + t1 * m1 * m1 + t2 * m2 * m2 -
                         real(2) * (P.Q[3][i] * m0 * m1 + P.Q[4][i] * m0 * m2 + P.Q[5][i] * m1 * m2);
          fa[FP_EAN] += 0.5 * V * (double)q;
        }
      } else {
        fa[FP_EAN] -= 0.5 * V * (double)(m0 * ax + m1 * ay + m2 * az);
      }
      // with the applied field in FP64 (rounding it to FP32 would bias every node alike)
      if (zeem) fa[FP_EZ] -= V * ((double)m0 * C->bz[0] + (double)m1 * C->bz[1] + (double)m2 * C->bz[2]);
      fa[FP_ED] += 0.5 * V * (double)(m0 * dx + m1 * dy + m2 * dz);
      const double H2 = (double)Hx * Hx + (double)Hy * Hy + (double)Hz * Hz;
      fa[FP_TMAX] = fmax(fa[FP_TMAX], sqrt(H2));
      fa[FP_D] += V * H2;
      fa[FP_H2] += H2;
      // BB differences against the accepted state: s = m_t - m, y = g_t - g, g = m x H
      const real n0 = P.m[a][0][i], n1 = P.m[a][1][i], n2 = P.m[a][2][i];
      const real G0 = P.H[a][0][i], G1 = P.H[a][1][i], G2 = P.H[a][2][i];
      const double s0 = (double)m0 - n0, s1 = (double)m1 - n1, s2 = (double)m2 - n2;
      const double y0 = (double)(m1 * Hz - m2 * Hy) - (double)(n1 * G2 - n2 * G1);
      const double y1 = (double)(m2 * Hx - m0 * Hz) - (double)(n2 * G0 - n0 * G2);
      const double y2 = (double)(m0 * Hy - m1 * Hx) - (double)(n0 * G1 - n1 * G0);
      fa[FP_SS] += V * (s0 * s0 + s1 * s1 + s2 * s2);
      // the next step goes along H_t x m_t (first order): its overlap with this one
      fa[FP_SD] += V * (s0 * ((double)Hy * m2 - (double)Hz * m1) + s1 * ((double)Hz * m0 - (double)Hx * m2) +
                        s2 * ((double)Hx * m1 - (double)Hy * m0));
      fa[FP_SY] += V * (s0 * y0 + s1 * y1 + s2 * y2);
      fa[FP_YY] += V * (y0 * y0 + y1 * y1 + y2 * y2);
      fa[FP_MX] += V * (double)m0;
      fa[FP_MY] += V * (double)m1;
      fa[FP_MZ] += V * (double)m2;
      if constexpr (kDiff) {
        // energy change from the accepted state.  Every term of the energy is
        // quadratic or linear in m, so e(m_t) - e(m) = -1/2 sum V s.(h_t + h)
        // exactly, with s = m_t - m: small products of s, accurate relative
        // to the change itself, where the difference of two FP32 energies
        // would lose it.  The accepted field is h = (m.h) m + H x m.
        const double mha = (double)P.mh[a][i];
        const double ha0 = mha * n0 + ((double)G1 * n2 - (double)G2 * n1);
        const double ha1 = mha * n1 + ((double)G2 * n0 - (double)G0 * n2);
        const double ha2 = mha * n2 + ((double)G0 * n1 - (double)G1 * n0);
        const double sh = s0 * ((double)hx + ha0) + s1 * ((double)hy + ha1) + s2 * ((double)hz + ha2);
        fa[FP_DE] -= 0.5 * V * sh;
        P.mh[tr][i] = m0 * hx + m1 * hy + m2 * hz;
      }
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kNPart; ++k) acc[k] = fa[k];
  }
}

__device__ __forceinline__ int n_parts(int phase, int mg_op = 0, int mg_lev = 0) {
  switch (phase) {
    case PH_PREP: return 3;
    case PH_CG0: return 2;
    case PH_CG: return 4;
    case PH_FIELD: return kNPart;
    case PH_MG: return (mg_op == MG_POST && mg_lev == 0) ? 1 : 0;
    case PH_PCG_A: return 1;
    case PH_PCG_B: return 2;
    default: return 0;
  }
}

__device__ __forceinline__ bool is_work(int phase) {
  return (phase >= PH_PREP && phase <= PH_FIELD) || phase == PH_MG || phase == PH_PCG_A || phase == PH_PCG_B;
}

__device__ void push_hist(Ctrl* C, double e) {
  const int M = C->nonmono_M;
  C->hist[C->hist_pos] = e;
  C->hist_pos = (C->hist_pos + 1) % M;
  if (C->hist_n < M) C->hist_n++;
}

__device__ void accept_trial(Ctrl* C, const double* v, double e_t, const double* eterm) {
  C->acc = 1 - C->acc;
  C->e_acc = e_t;
  C->e_chain = e_t;
  C->halvings = 0;
  C->T_acc = v[FP_TMAX];
  C->d_acc = v[FP_D];
  C->h2_acc = v[FP_H2];
  for (int k = 0; k < 4; ++k) C->eterm_acc[k] = eterm[k];
  C->mavg_acc[0] = v[FP_MX] / C->vol;
  C->mavg_acc[1] = v[FP_MY] / C->vol;
  C->mavg_acc[2] = v[FP_MZ] / C->vol;
  push_hist(C, e_t);
}

constexpr int kStall = 50;   // accepted steps without progress that end a mixed run

// Stopping test on the accepted state: the largest torque (default), or the
// sum of the squared torques against tol^2 (the paper's test on the squared
// projected gradient, Results section).
__device__ __forceinline__ bool converged(const Ctrl* C) {
  return C->stop_sum2 ? C->h2_acc < C->tol * C->tol : C->T_acc < C->tol;
}

__device__ void finish_done(Ctrl* C, int status) {
  C->status = status;
  C->phase = PH_DONE;
}

template <typename real>
__device__ __forceinline__ void signal_done(const ProbDev<real>& P, const Ctrl* C) {
  if (P.ndone && C->phase == PH_DONE) {
    const unsigned k = atomicAdd((unsigned*)P.ndone, 1u);
    if (P.done_list) P.done_list[k] = P.slot;
  }
}

// Step-length logic after an evaluated trial (Method section, step length
// selection): acceptance against the nonmonotone reference, Armijo
// backtracking for the first step and for rejected BB steps, then the BB
// step lengths tau1 = s.s/s.y, tau2 = s.y/y.y (eq. (10)) chosen by the rule.
__device__ void step_logic(Ctrl* C, const double* v) {
  const bool anis = C->terms & MMSD_ANIS;
  double eterm[4] = {v[FP_EEX], v[FP_EAN] + (anis ? C->c_an : 0.0), v[FP_EZ],
                     v[FP_ED] + (C->demag ? 0.5 * C->ru : 0.0)};
  const double e_direct = eterm[0] + eterm[1] + eterm[2] + eterm[3];
  // the energy the decisions use: direct, or (chain mode, after the first
  // evaluation) the accepted energy plus the change the FIELD phase summed
  const double e_t = (C->chain && C->stage == ST_RUN) ? C->e_chain + v[FP_DE] : e_direct;
  C->evals++;
  if (!isfinite(e_t) || !isfinite(e_direct) || !isfinite(v[FP_TMAX])) {
    finish_done(C, MMSD_E_NONFINITE);
    return;
  }
  if (C->stage == ST_EVAL) {
    accept_trial(C, v, e_t, eterm);
    finish_done(C, MMSD_OK);
    return;
  }
  if (C->stage == ST_INIT) {
    accept_trial(C, v, e_t, eterm);
    if (converged(C)) {
      finish_done(C, MMSD_OK);
      return;
    }
    C->stall = 0;
    C->prog_e = C->e_chain;
    C->prog_T = C->T_acc;
    C->tau = C->theta0 / C->T_acc;
    C->first = 1;
    C->backtrack = 0;
    C->kappa = C->kappa0;
    C->win_n = 0;
    C->win_pos = 0;
    C->alt = 0;
    C->stage = ST_RUN;
    C->phase = PH_PREP;
    return;
  }
  double e_ref = C->hist[0];
  for (int k = 1; k < C->hist_n; ++k) e_ref = fmax(e_ref, C->hist[k]);
  const bool armijo = C->first || C->backtrack;
  const bool ok = armijo ? (e_t <= e_ref - C->c1 * C->tau * C->d_acc) : (e_t <= e_ref);
  if (!ok) {
    if (C->evals >= C->max_evals) {
      finish_done(C, MMSD_W_MAXEVALS);
      return;
    }
    C->tau *= C->rho;
    C->backtrack = 1;
    // stop also after max_halvings failed trials of one line search (mixed
    // form: once the torque reaches the FP32 fields' error, the trials'
    // energy changes are no longer resolved, and halving does not help)
    if (C->tau < C->tau_floor || (C->max_halvings > 0 && ++C->halvings > C->max_halvings)) {
      finish_done(C, MMSD_W_FLOOR);
      return;
    }
    C->phase = PH_PREP;
    return;
  }
  const double ss = v[FP_SS], sy = v[FP_SY], yy = v[FP_YY];
  accept_trial(C, v, e_t, eterm);
  C->iters++;
  if (converged(C)) {
    finish_done(C, MMSD_OK);
    return;
  }
  if (C->evals >= C->max_evals) {
    finish_done(C, MMSD_W_MAXEVALS);
    return;
  }
  if (C->chain) {
    // mixed form: once the torque reaches the error of the FP32 fields the
    // accepted steps only shuffle noise.  Progress is a torque 10% below the
    // best so far or an energy below the one at the last progress by more
    // than its FP32 resolution (a reversal near a switching field lowers the
    // energy while its torque grows); kStall accepted steps without progress
    // end the run (FLOOR).
    const double e_scale = fabs(eterm[0]) + fabs(eterm[1]) + fabs(eterm[2]) + fabs(eterm[3]);
    if (C->T_acc < 0.9 * C->prog_T || C->e_chain < C->prog_e - C->e_res * e_scale) {
      C->prog_T = fmin(C->prog_T, C->T_acc);
      C->prog_e = fmin(C->prog_e, C->e_chain);
      C->stall = 0;
    } else if (++C->stall >= kStall) {
      finish_done(C, MMSD_W_FLOOR);
      return;
    }
  }
  C->first = 0;
  C->backtrack = 0;
  double tau = C->tau;
  if (sy <= 0.0) {
    tau = fmin(10.0 * tau, C->tau_max);
  } else {
    const double t1 = ss / sy, t2 = sy / yy;
    switch (C->step_rule) {
      case MMSD_STEP_BB1:
        tau = t1;
        break;
      case MMSD_STEP_BB2:
        tau = t2;
        break;
      case MMSD_STEP_ALTERNATE:
        tau = (C->alt & 1) ? t2 : t1;
        C->alt ^= 1;
        break;
      default: {
        // adaptive switching (min of the last 3 tau2 when tau2/tau1 < kappa)
        const int W = 3;
        C->win[C->win_pos] = t2;
        C->win_pos = (C->win_pos + 1) % W;
        if (C->win_n < W) C->win_n++;
        if (t2 / t1 < C->kappa) {
          double mn = C->win[0];
          for (int k = 1; k < C->win_n; ++k) mn = fmin(mn, C->win[k]);
          tau = mn;
          C->kappa *= 0.9;
        } else {
          tau = t1;
          C->kappa *= 1.1;
        }
      }
    }
  }
  C->tau = fmin(fmax(tau, C->tau_min), C->tau_max);
  // first-order overlap of the next step (tau (H x m) at the new state) with the last
  C->step_proj = ss > 0.0 ? C->tau * v[FP_SD] / ss : 0.0;
  C->phase = PH_PREP;
}


// Potential buffers of the solve a PREP starts: after an accepted state
// (or at the start) the working buffer holds its potential, which becomes
// the accepted one and is copied into the next working buffer; after a
// rejected trial the start is interpolated between the accepted and the
// rejected trial's potentials into the third buffer.
__device__ void enter_prep(Ctrl* C) {
  if (!C->demag) return;
  if (C->backtrack) {
    C->u_src = C->uacc;
    C->u_src2 = C->ucur;
    C->u_w = C->rho;
    C->ucur = 3 - C->uacc - C->ucur;
  } else if (C->iters > 0 && C->ucur != C->uacc) {
    // after an accepted step s: the next step's potential change is about
    // (s_new.s / s.s) times this step's, u_acc - u_prev
    C->u_src = C->ucur;
    C->u_src2 = C->uacc;
    C->u_w = -C->step_proj;
    const int w = 3 - C->uacc - C->ucur;
    C->uacc = C->ucur;
    C->ucur = w;
  } else {
    C->u_src = C->ucur;
    C->u_src2 = -1;
    C->u_w = 0.0;
    C->uacc = C->ucur;
    C->ucur = (C->ucur + 1) % 3;
  }
}

// Advance the state by the outcome of the phase it records (v: the finished
// reductions of that phase's partials); the phases of the potential solve's
// iterations are advanced by transition_fast() below.
__device__ void transition_phase(Ctrl* C, const double* v, const double* btab, int n_lev, int fused, bool folded) {
  C->seq++;
  const int phase = C->phase;
  if (phase == PH_IDLE || phase == PH_DONE) return;
  if (phase == PH_START) {
    C->phase = PH_PREP;
    return;
  }
  C->launches_done++;
  if (btab) C->alg_bytes += btab[byte_slot(phase, C->mg_op, C->mg_lev)];   // block 0 only: it publishes C
  C->nphase[phase == PH_FIELD ? 3 : phase == PH_PREP ? 0 : (phase == PH_CG0 || phase == PH_MG) ? 1 : 2]++;
  switch (phase) {
    case PH_PREP:
      if (!C->demag) {
        C->ru = 0;
        C->phase = PH_FIELD;
        return;
      }
      C->bb = v[0];
      C->rr = v[1];
      C->ru = v[2];
      C->pcg_it = 0;
      if (C->rr <= C->pcg_rtol2 * C->bb) {
        C->phase = PH_FIELD;
      } else if (C->precond == PC_AMG) {
        C->phase = PH_MG;
        C->mg_op = MG_DOWN;
        C->mg_lev = 0;
        C->mg_first = 1;
      } else {
        C->phase = PH_CG0;
      }
      return;
    case PH_CG0:
      C->gam = v[0];
      C->dlt = v[1];
      C->alpha = C->gam / C->dlt;
      C->beta = 0.0;
      C->phase = PH_CG;
      return;
    case PH_CG: {
      // gamma = r.D^-1 r, delta = (L D^-1 r).D^-1 r of the new residual
      const double gam = v[0], dlt = v[1];
      const double beta = gam / C->gam;
      C->alpha = gam / (dlt - beta * gam / C->alpha);
      C->beta = beta;
      C->gam = gam;
      C->dlt = dlt;
      C->rr = v[2];
      C->ru = v[3];
      C->pcur ^= 1;
      C->pcg_it++;
      C->pcg_total++;
      C->phase = (C->rr <= C->pcg_rtol2 * C->bb || C->pcg_it >= C->pcg_maxit) ? PH_FIELD : PH_CG;
      return;
    }
    case PH_FIELD:
      step_logic(C, v);
      return;
  }
}

// The V-cycle operation after (op, lev), in (nop, nlev); false after the
// post-smoothing of level 0, which completes z = M r.
__device__ __forceinline__ bool mg_next(int op, int lev, int n_lev, int fused, bool folded, int& nop, int& nlev) {
  nop = op;
  nlev = lev;
  if (op == MG_DOWN && !((fused >> lev) & 1)) {
    nop = MG_REST;
    return true;
  }
  if (op == MG_DOWN || op == MG_REST) {   // a fused DOWN also restricted
    if (lev + 1 < n_lev) {
      nlev = lev + 1;
      nop = MG_DOWN;
    } else if (folded) {   // the last DOWN also solved the coarsest level
      nop = MG_POST;
    } else {
      nop = MG_SOLVE;
      nlev = 0;
    }
    return true;
  }
  if (op == MG_SOLVE) {
    nlev = n_lev - 1;
    nop = MG_POST;
    return true;
  }
  if (lev > 0) {
    nlev = lev - 1;
    return true;
  }
  return false;
}

// The transitions inside the potential solve (after a V-cycle operation or
// one of the two PCG phases: every launch of a PCG iteration), in a short
// inline path of their own: the general transition is long, and each launch
// starts with a cold instruction cache.  Returns false for every other
// phase.
__device__ __forceinline__ bool transition_fast(Ctrl* C, const double* v, const double* btab, int n_lev, int fused,
                                                bool folded) {
  const int phase = C->phase;
  if (phase != PH_MG && phase != PH_PCG_A && phase != PH_PCG_B) return false;
  C->seq++;
  C->launches_done++;
  if (btab) C->alg_bytes += btab[byte_slot(phase, C->mg_op, C->mg_lev)];
  if (phase == PH_MG) {
    C->nphase[1]++;
    int nop, nlev;
    if (mg_next(C->mg_op, C->mg_lev, n_lev, fused, folded, nop, nlev)) {
      C->mg_op = nop;
      C->mg_lev = nlev;
    } else {   // z = M r is complete: next search direction
      C->beta = C->mg_first ? 0.0 : v[0] / C->gam;
      C->gam = v[0];
      C->mg_first = 0;
      C->phase = PH_PCG_A;
    }
    return true;
  }
  C->nphase[2]++;
  if (phase == PH_PCG_A) {
    C->alpha = C->gam / v[0];
    C->pcur ^= 1;
    C->phase = PH_PCG_B;
    return true;
  }
  C->rr = v[0];
  C->ru = v[1];
  C->rcur ^= 1;
  C->pcg_it++;
  C->pcg_total++;
  if (C->rr <= C->pcg_rtol2 * C->bb || C->pcg_it >= C->pcg_maxit) {
    C->phase = PH_FIELD;
  } else {
    C->phase = PH_MG;
    C->mg_op = MG_REST;
    C->mg_lev = 0;
  }
  return true;
}

// Every other transition (PREP, the Jacobi-CG phases, FIELD's step logic).
__device__ void transition(Ctrl* C, const double* v, const double* btab, int n_lev, int fused, bool folded) {
  transition_phase(C, v, btab, n_lev, fused, folded);
  if (C->phase == PH_PREP) enter_prep(C);
}

// out[k] = sum (max for the torque slot) over the G block partials of slot k
// (stored slot-major: the G partials of one slot are contiguous).
// Wavefront w takes slots w, w + 8, ...; lanes stride over the blocks, then a
// butterfly combines them: the same fixed order in every block.  Slots 0 and
// 1 were already fetched (`pre`, by waves 0 and 1) together with the control
// block.
constexpr int kPreParts = 8;   // partials per lane fetched early: G <= 64 * kPreParts
__device__ __forceinline__ void reduce_partials(DevPtr<const double> src, int G, int np, int phase, const double* pre, double* out) {
  const int wid = threadIdx.x >> 6, lid = threadIdx.x & 63;
  for (int k = wid; k < np; k += kBlock / 64) {
    const bool mx = (phase == PH_FIELD && k == FP_TMAX);
    double v = 0.0;
    if (k < 2 && G <= 64 * kPreParts) {
#pragma unroll
      for (int u = 0; u < kPreParts; ++u) {
        const double x = pre[u];
        v = (lid + 64 * u < G) ? (mx ? fmax(v, x) : v + x) : v;
      }
    } else {
      for (int q = lid; q < G; q += 64) {
        const double x = src[(size_t)k * G + q];
        v = mx ? fmax(v, x) : v + x;
      }
    }
    v = mx ? wave_max(v) : wave_sum(v);
    if (lid == 0) out[k] = v;
  }
}

// One phase on this block's rows, then its block partials: butterfly in each
// wave, then the waves in order; plain stores, published to the next launch
// by the kernel boundary.  The accumulators live only inside one phase, so
// each phase is register-allocated on its own.
template <typename real, int LPR, int PHASE>
__device__ __forceinline__ void run_phase(const ProbDev<real>& P, const Ctrl* C, int lb, int parity,
                                          double (*s_red)[kNPart], int mop = 0, int mlev = 0) {
  constexpr int NA = PHASE == PH_FIELD ? kNPart : PHASE == PH_PREP ? 3 : PHASE == PH_MG ? 1 : 4;
  double acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k] = 0.0;
  if constexpr (PHASE == PH_PREP) phase_prep<real, LPR>(P, C, lb, acc);
  else if constexpr (PHASE == PH_CG0) phase_cg0<real, LPR>(P, C, lb, acc);
  else if constexpr (PHASE == PH_CG) phase_cg<real, LPR>(P, C, lb, acc);
  else if constexpr (PHASE == PH_FIELD) phase_field<real, LPR>(P, C, lb, acc);
  else if constexpr (PHASE == PH_MG) phase_mg<real, LPR>(P, C, mop, mlev, lb, acc);
  else if constexpr (PHASE == PH_PCG_A) phase_pcg_a<real, LPR>(P, C, lb, acc);
  else phase_pcg_b<real, LPR>(P, C, lb, acc);

  const int np = n_parts(PHASE, mop, mlev);
  if (np == 0) return;
  const int wid = threadIdx.x >> 6, lid = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    if (k < np) {
      const double v = (PHASE == PH_FIELD && k == FP_TMAX) ? wave_max(acc[k]) : wave_sum(acc[k]);
      if (lid == 0) s_red[wid][k] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < np) {
    const int k = threadIdx.x;
    const bool mx = (PHASE == PH_FIELD && k == FP_TMAX);
    double v = s_red[0][k];
    for (int w = 1; w < kBlock / 64; ++w) v = mx ? fmax(v, s_red[w][k]) : v + s_red[w][k];
    P.part[((size_t)parity * kNPart + k) * P.G + lb] = v;
  }
}

// At most 128 VGPRs (4 wavefronts per SIMD): two 512-thread blocks per CU
// stay resident (as they would at 5), with no register spills.  512 blocks
// of 512 threads measured fastest overall: 768 blocks slowed the sweep by
// 16%; 256 blocks of 1024 threads (the same wavefronts per CU) took 1.5% off
// a PCG iteration of the 80 nm cube but slowed the small grain problems by
// 6-10%.
template <typename real, int LPR>
__global__ void __launch_bounds__(kBlock, 4) k_step(const ProbDev<real>* __restrict__ probs, int nprob,
                                                    const int* __restrict__ blk_start, int parity) {
  __shared__ Ctrl s_c;
  __shared__ double s_red[kBlock / 64][kNPart];
  __shared__ double s_tot[kNPart];
  __shared__ double s_btab[kByteSlots];
  __shared__ int s_newly_done;
  const int b = blockIdx.x;
  int lo = 0, hi = nprob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (blk_start[mid] <= b) lo = mid;
    else hi = mid;
  }
  const ProbDev<real>& P = probs[lo];
  const int lb = b - P.blk0;
  const int prev = parity ^ 1;

  // prologue: the previous launch's state and the reductions of its phase.
  // The control block, block 0's byte table and partial slots 0 and 1 are
  // fetched in one round trip; the phase decides later what is used.
  DevPtr<const double> part_prev = P.part + (size_t)prev * P.G * kNPart;
  // The control block, the level descriptors and block 0's byte table (one
  // word per thread each) are loaded before the partials and stored to LDS
  // after them: loads complete in order, so the stores, and the barrier,
  // wait only for those words, and the partials stay in flight through the
  // transition of the V-cycle launches, which do not use them.
  static_assert(sizeof(Ctrl) / 8 <= kBlock && kByteSlots <= kBlock &&
                    kMaxLevels * sizeof(MgLevelDev<double>) / 8 <= kBlock,
                "one word per thread");
  double pre[kPreParts];
  {
    const int wid = threadIdx.x >> 6, lid = threadIdx.x & 63, t = threadIdx.x;
    const int cwords = (int)(sizeof(Ctrl) / 8);
    const int lwords = P.n_lev * (int)(sizeof(MgLevelDev<real>) / 8);
    DevPtr<const long long> csrc = reinterpret_cast<DevPtr<const long long>>(P.ctrl + prev);
    DevPtr<const long long> lsrc = reinterpret_cast<DevPtr<const long long>>(P.lev);
    const long long cw = t < cwords ? csrc[t] : 0;
    const long long lw = t < lwords ? lsrc[t] : 0;
    const double bw = (lb == 0 && t < kByteSlots) ? P.btab[t] : 0.0;
#pragma unroll
    for (int u = 0; u < kPreParts; ++u) {
      const int q = lid + 64 * u;
      pre[u] = (wid < 2 && q < P.G) ? part_prev[(size_t)wid * P.G + q] : 0.0;
    }
    if (t < cwords) reinterpret_cast<long long*>(&s_c)[t] = cw;
    if (t < lwords) reinterpret_cast<long long*>(s_lev_raw)[t] = lw;
    if (lb == 0 && t < kByteSlots) s_btab[t] = bw;
  }
  __syncthreads();
  const int ran = s_c.phase;
  auto publish = [&] {   // block 0: the new control state into slot `parity`
    const long long* src = reinterpret_cast<const long long*>(&s_c);
    DevPtr<long long> dst = reinterpret_cast<DevPtr<long long>>(P.ctrl + parity);
    for (int w = threadIdx.x; w < (int)(sizeof(Ctrl) / 8); w += kBlock) dst[w] = src[w];
  };
  // From one V-cycle operation to the next nothing is reduced and only the
  // cycle position changes: every thread derives the next operation from the
  // position it read after the barrier above, and only block 0 records the
  // transition, at the end, once every wavefront of the block has passed a
  // second barrier.  Recording it here would race with wavefronts that have
  // not yet read the position: a late one would run the operation after the
  // next (or take the other branch, with its own barriers).
  int mop = 0, mlev = 0;
  const bool in_cycle =
      ran == PH_MG && mg_next(s_c.mg_op, s_c.mg_lev, P.n_lev, P.mg_fused, P.AinvM != nullptr, mop, mlev);
  int phase = PH_MG;
  if (!in_cycle) {
    const int np_prev = n_parts(ran, s_c.mg_op, s_c.mg_lev);
    if (np_prev > 0) reduce_partials(part_prev, P.G, np_prev, ran, pre, s_tot);
    __syncthreads();
    if (threadIdx.x == 0) {
      if (!transition_fast(&s_c, s_tot, lb == 0 ? s_btab : nullptr, P.n_lev, P.mg_fused, P.AinvM != nullptr))
        transition(&s_c, s_tot, lb == 0 ? s_btab : nullptr, P.n_lev, P.mg_fused, P.AinvM != nullptr);
      s_newly_done = (ran != PH_DONE && s_c.phase == PH_DONE);
    }
    __syncthreads();
    if (lb == 0) {
      publish();
      if (threadIdx.x == 0 && s_newly_done) signal_done<real>(P, &s_c);
    }
    phase = s_c.phase;
    mop = s_c.mg_op;
    mlev = s_c.mg_lev;
    if (!is_work(phase)) return;
  }

  switch (phase) {
    case PH_PREP:
      run_phase<real, LPR, PH_PREP>(P, &s_c, lb, parity, s_red);
      break;
    case PH_CG0:
      run_phase<real, LPR, PH_CG0>(P, &s_c, lb, parity, s_red);
      break;
    case PH_CG:
      run_phase<real, LPR, PH_CG>(P, &s_c, lb, parity, s_red);
      break;
    case PH_FIELD:
      run_phase<real, LPR, PH_FIELD>(P, &s_c, lb, parity, s_red);
      break;
    case PH_MG:
      run_phase<real, LPR, PH_MG>(P, &s_c, lb, parity, s_red, mop, mlev);
      break;
    case PH_PCG_A:
      run_phase<real, LPR, PH_PCG_A>(P, &s_c, lb, parity, s_red);
      break;
    case PH_PCG_B:
      run_phase<real, LPR, PH_PCG_B>(P, &s_c, lb, parity, s_red);
      break;
  }
  if (in_cycle && lb == 0) {
    __syncthreads();   // every wavefront has read the cycle position
    if (threadIdx.x == 0) transition_fast(&s_c, s_tot, s_btab, P.n_lev, P.mg_fused, P.AinvM != nullptr);
    __syncthreads();   // thread 0's record of the transition
    publish();
  }
}

// Arm a problem for a new minimization or evaluation: the state goes into
// slot `slot` (the one the next step launch reads), with a sequence number
// above both slots' so the host always picks the newest.
struct CtrlInit {
  int stage, terms, nonmono_M, step_rule, pcg_maxit, store_h, demag, acc, precond, chain, max_halvings, stop_sum2;
  int ucur, pad;
  long long max_evals;
  double tol, pcg_rtol2, c1, rho, kappa0, theta0, tau_min, tau_max, tau_floor, e_res;
  double bz[3], c_an, vol;
};

__global__ void k_ctrl_init(Ctrl* ctrl, int slot, CtrlInit a) {
  if (threadIdx.x != 0) return;
  const long long seq = ctrl[0].seq > ctrl[1].seq ? ctrl[0].seq : ctrl[1].seq;
  Ctrl* C = &ctrl[slot];
  C->seq = seq + 1;
  C->phase = PH_START;
  C->stage = a.stage;
  C->acc = a.acc;
  C->pcur = 0;
  C->first = 0;
  C->backtrack = 0;
  C->status = 0;
  C->pcg_it = 0;
  C->hist_n = 0;
  C->hist_pos = 0;
  C->win_n = 0;
  C->win_pos = 0;
  C->terms = a.terms;
  C->nonmono_M = a.nonmono_M;
  C->step_rule = a.step_rule;
  C->alt = 0;
  C->pcg_maxit = a.pcg_maxit;
  C->store_h = a.store_h;
  C->demag = a.demag;
  C->stop_sum2 = a.stop_sum2;
  C->ucur = C->uacc = C->u_src = a.ucur;
  C->u_src2 = -1;
  C->u_w = 0.0;
  C->step_proj = 0.0;
  C->evals = 0;
  C->iters = 0;
  C->pcg_total = 0;
  C->max_evals = a.max_evals;
  C->launches_done = 0;
  for (int k = 0; k < 4; ++k) C->nphase[k] = 0;
  C->precond = a.precond;
  C->mg_op = 0;
  C->mg_lev = 0;
  C->rcur = 0;
  C->mg_first = 0;
  C->chain = a.chain;
  C->max_halvings = a.max_halvings;
  C->halvings = 0;
  C->e_chain = 0.0;
  C->alg_bytes = 0.0;
  C->tol = a.tol;
  C->pcg_rtol2 = a.pcg_rtol2;
  C->c1 = a.c1;
  C->rho = a.rho;
  C->kappa0 = a.kappa0;
  C->theta0 = a.theta0;
  C->tau_min = a.tau_min;
  C->tau_max = a.tau_max;
  C->tau_floor = a.tau_floor;
  C->e_res = a.e_res;
  C->stall = 0;
  C->prog_e = C->prog_T = 0.0;
  for (int k = 0; k < 3; ++k) C->bz[k] = a.bz[k];
  C->c_an = a.c_an;
  C->vol = a.vol;
  C->tau = 0.0;
  C->kappa = a.kappa0;
  C->gam = C->dlt = C->bb = C->rr = C->ru = C->alpha = C->beta = 0.0;
}

// Plain streaming copy, 16 bytes per thread per step: the reference kernel
// for calibrating hardware traffic counters against a known byte count.
__global__ void __launch_bounds__(256) k_copy_probe(const double2* __restrict__ src, double2* __restrict__ dst,
                                                    long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 16);
  hipLaunchKernelGGL(k_copy_probe, dim3(2048), dim3(256), 0, s, (const double2*)src, (double2*)dst, n);
  return hipGetLastError();
}

// ---- host-side launch wrappers -------------------------------------------
template <typename real>
hipError_t launch_step(int lpr, const Prob<real>* probs, int nprob, const int* blk_start, int grid, int parity,
                       hipStream_t s) {
  const ProbDev<real>* dprobs = reinterpret_cast<const ProbDev<real>*>(probs);
  switch (lpr) {
    case 4:
      hipLaunchKernelGGL((k_step<real, 4>), dim3(grid), dim3(kBlock), 0, s, dprobs, nprob, blk_start, parity);
      break;
    case 16:
      hipLaunchKernelGGL((k_step<real, 16>), dim3(grid), dim3(kBlock), 0, s, dprobs, nprob, blk_start, parity);
      break;
    default:
      hipLaunchKernelGGL((k_step<real, 8>), dim3(grid), dim3(kBlock), 0, s, dprobs, nprob, blk_start, parity);
      break;
  }
  return hipGetLastError();
}

template hipError_t launch_step<double>(int, const Prob<double>*, int, const int*, int, int, hipStream_t);
template hipError_t launch_step<float>(int, const Prob<float>*, int, const int*, int, int, hipStream_t);

hipError_t launch_ctrl_init(Ctrl* ctrl, int slot, int stage, int terms, int nonmono_M, int step_rule,
                            int pcg_maxit, int store_h, int demag, int acc, int precond, int chain,
                            int max_halvings, int stop_sum2, int ucur, long long max_evals,
                            const double* dparams, hipStream_t s) {
  CtrlInit a;
  a.ucur = ucur;
  a.pad = 0;
  a.precond = precond;
  a.chain = chain;
  a.max_halvings = max_halvings;
  a.stop_sum2 = stop_sum2;
  a.stage = stage;
  a.terms = terms;
  a.nonmono_M = nonmono_M;
  a.step_rule = step_rule;
  a.pcg_maxit = pcg_maxit;
  a.store_h = store_h;
  a.demag = demag;
  a.acc = acc;
  a.max_evals = max_evals;
  a.tol = dparams[0];
  a.pcg_rtol2 = dparams[1];
  a.c1 = dparams[2];
  a.rho = dparams[3];
  a.kappa0 = dparams[4];
  a.theta0 = dparams[5];
  a.tau_min = dparams[6];
  a.tau_max = dparams[7];
  a.tau_floor = dparams[8];
  a.bz[0] = dparams[9];
  a.bz[1] = dparams[10];
  a.bz[2] = dparams[11];
  a.c_an = dparams[12];
  a.vol = dparams[13];
  a.e_res = dparams[14];
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, s, ctrl, slot, a);
  return hipGetLastError();
}

}  // namespace mmsd
