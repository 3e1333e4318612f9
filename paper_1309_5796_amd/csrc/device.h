// Device-side data of one minimization problem and the phase machine that
// drives it.  Shared by the kernels and the host runtime of the library.
//
// One evaluation of the energy gradient (Method section; the paper's Table 2
// lists its linear-algebra parts) is a sequence of phases; every launch of
// the step kernel advances every unfinished problem of its table by exactly
// one phase, and the last block of a problem to finish decides the next phase:
//
//   PREP   trial m_t = Cayley(m, h, tau) (eq. (7), explicit form) on magnet
//          rows; b = G m_t; r = b - L u (warm start); z = D^-1 r
//   PCG_A  p = z + beta p_old (recomputed at every gathered neighbour);
//          q = L p; partial p.q
//   PCG_B  u += alpha p; r -= alpha q; z = D^-1 r; partial r.z, r.r, r.u
//   FIELD  h = -K m - D2 u + Q m + b_ext/Js; H = m x h; fused reductions of
//          the energy, max|H|, sum V|H|^2 and the BB dots s.s, s.y, y.y
//          (eq. (9)); the last block then runs the step-length logic
//          (acceptance, BB / adaptive switching, line search, stopping test).
//
// Internal units: lengths in nm, energies in mu0 Ms^2 nm^3, fields in Ms,
// potential in Ms nm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmsd {

enum Phase : int { PH_IDLE = 0, PH_PREP = 1, PH_PCG_A = 2, PH_PCG_B = 3, PH_FIELD = 4, PH_DONE = 5 };
enum Stage : int { ST_INIT = 0, ST_RUN = 1, ST_EVAL = 2 };

constexpr int kBlock = 256;        // threads per block (4 wavefronts of 64)
constexpr int kGroup = 64;         // blocks per first-level reduction group
constexpr int kNPart = 13;         // partial sums per block (FIELD needs 13)
constexpr int kMaxHist = 64;       // nonmonotone memory capacity
constexpr int kMaxBlocks = 1 << 16;  // per problem
constexpr int kMaxGroups = kMaxBlocks / kGroup;

// FIELD partial slots
enum FieldPart : int {
  FP_EEX = 0, FP_EAN = 1, FP_EZ = 2, FP_ED = 3, FP_TMAX = 4, FP_D = 5,
  FP_SS = 6, FP_SY = 7, FP_YY = 8, FP_MX = 9, FP_MY = 10, FP_MZ = 11, FP_H2 = 12
};

// Control block of one problem.  Written only by the finishing block of a
// launch (thread 0) and by the host-side init kernel; read by every block at
// the start of a launch.
struct Ctrl {
  // phase machine
  int phase, stage, acc, pcur;
  int first, backtrack, status, pcg_it;
  int hist_n, hist_pos, win_n, win_pos;
  int terms, nonmono_M, step_rule, alt;
  int pcg_maxit, store_h, demag, pad0;
  long long evals, iters, pcg_total, max_evals;
  long long launches_done;       // phases executed
  long long nphase[4];           // executed PREP, PCG_A, PCG_B, FIELD phases
  // options and constants
  double tol, pcg_rtol2, c1, rho, kappa0, theta0, tau_min, tau_max, tau_floor;
  double bz[3];                  // applied field / Js
  double c_an;                   // sum_e V_e K1_e / (mu0 Ms^2)
  double vol;                    // sum_i V_i
  // step state
  double tau, kappa;
  double win[4];
  double hist[kMaxHist];
  double e_acc, T_acc, d_acc, h2_acc;
  double eterm_acc[4];
  double mavg_acc[3];
  // PCG scalars
  double rz, pq, bb, rr, ru, alpha, beta;
  double pad1[4];
};

template <typename real>
struct Prob {
  int N, Nt, G, blk0;
  // magnet rows: CSR pattern shared by K, D1 (b = D1 m) and D2 (h_d = -D2 u)
  const int* mrp;
  const int* mci;
  const real* K;          // 2 K_ij / V_i
  const real* D1[3];      // sum_e V_e/4 grad(phi_i)|_e
  const real* D2[3];      // sum_e V_e/4 grad(phi_j)|_e / V_i
  const real* Q[6];       // 2 Q_i / V_i: xx yy zz xy xz yz
  const real* V;          // lumped nodal volume
  real* m[2][3];          // accepted / trial slots, SoA
  real* H[2][3];          // torque m x h per slot
  real* h[3];             // effective field (written when store_h)
  // potential rows (magnet rows first): transformed Laplacian
  const int* lrp;
  const int* lci;
  const real* L;
  const real* invd;       // 1 / diag(L)
  real* u;
  real* r;
  real* z;
  real* p[2];
  real* q;
  // reductions
  unsigned* ndone;        // nullable: incremented once when the problem finishes
  int* done_list;         // nullable: receives `slot` at position ndone - 1
  int slot;
  double* part;           // [G][kNPart]
  double* gpart;          // [G/kGroup][kNPart]
  unsigned* cnt;          // [0] top level, [1 + g] group g
  Ctrl* ctrl;
};

}  // namespace mmsd
