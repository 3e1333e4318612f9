// Device-side data of one minimization problem and the phase machine that
// drives it.  Shared by the kernels and the host runtime of the library.
//
// One evaluation of the energy gradient (Method section; the paper's Table 2
// lists its linear-algebra parts) is a sequence of phases, one per launch of
// the step kernel:
//
//   PREP   trial m_t = Cayley(m, h, tau) (eq. (8), explicit form) on magnet
//          rows; b = G m_t; r = b - L u (warm start from the last solve)
//   CG0    w = L D^-1 r; partial r.D^-1 r and w.D^-1 r
//   CG     one Jacobi-preconditioned CG iteration in the single-reduction
//          (Chronopoulos-Gear) arrangement: p = D^-1 r + beta p,
//          s = w + beta s, u += alpha p, r -= alpha s, w = L D^-1 r, with both
//          dot products of the next step from the same sweep; neighbour
//          values of r, s, w are recomputed where they are gathered
//   FIELD  h = -K m - D2 u + Q m + b_ext/Js; H = m x h; fused reductions of
//          the energy, max|H|, sum V|H|^2 and the BB dots s.s, s.y, y.y
//          (eq. (10)).
// With the multigrid preconditioner the potential solve runs PH_MG
// operations (one V-cycle operation on one level per launch; a DOWN may
// also restrict, and on the last level also solve the coarsest level),
// PH_PCG_A and PH_PCG_B instead of CG0 / CG.
//
// Launches alternate a parity bit.  A launch of parity p reads the control
// state and the per-block partial sums that the previous launch (parity
// 1 - p) left in slot 1 - p, and every block runs the same deterministic
// transition on them (finishing the reductions, PCG scalars, and after a
// FIELD phase the step-length logic: acceptance, BB / adaptive switching,
// line search, stopping test).  Block 0 stores the new state in slot p; all
// blocks then execute the new phase and leave their partials in slot p.
// The kernel boundary publishes them, so no atomics or fences are needed.
//
// Internal units: lengths in nm, energies in mu0 Ms^2 nm^3, fields in Ms,
// potential in Ms nm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmsd {

enum Phase : int {
  PH_IDLE = 0, PH_PREP = 1, PH_CG0 = 2, PH_CG = 3, PH_FIELD = 4, PH_DONE = 5, PH_START = 6,
  PH_MG = 7,     // one multigrid V-cycle operation (sub-op and level in Ctrl)
  PH_PCG_A = 8,  // AMG-preconditioned CG: p = z + beta p, q = L p, p.q
  PH_PCG_B = 9   // u += alpha p, r -= alpha q, and the finest pre-smoothing residual
};
enum MgOp : int { MG_DOWN = 0, MG_REST = 1, MG_SOLVE = 2, MG_POST = 3,
                  MG_RESTM = 4 };   // inside a DOWN launch: the blocks that sweep M
enum Precond : int { PC_AUTO = 0, PC_JACOBI = 1, PC_AMG = 2 };
constexpr int kMaxLevels = 12;
enum Stage : int { ST_INIT = 0, ST_RUN = 1, ST_EVAL = 2 };

constexpr int kBlock = 512;        // threads per block (8 wavefronts of 64)
constexpr int kNPart = 15;         // partial sums per block (FIELD needs 15)
constexpr int kMaxHist = 64;       // nonmonotone memory capacity
constexpr int kMaxBlocks = 2048;   // per problem (every block reads all partials)

// FIELD partial slots
enum FieldPart : int {
  FP_EEX = 0, FP_EAN = 1, FP_EZ = 2, FP_ED = 3, FP_TMAX = 4, FP_D = 5,
  FP_SS = 6, FP_SY = 7, FP_YY = 8, FP_MX = 9, FP_MY = 10, FP_MZ = 11, FP_H2 = 12,
  FP_DE = 13,  // mixed form: energy change from the accepted state, -1/2 sum V s.(h_t + h)
  FP_SD = 14   // sum V s.(H_t x m_t): the step against the next descent direction
};

// Control state of one problem (two slots, one per launch parity).  `phase`
// is the phase the launch that wrote the slot executes.
struct Ctrl {
  long long seq;                 // launches since the state was armed (newest slot wins)
  // phase machine
  int phase, stage, acc, pcur;
  int first, backtrack, status, pcg_it;
  int hist_n, hist_pos, win_n, win_pos;
  int terms, nonmono_M, step_rule, alt;
  int pcg_maxit, store_h, demag, stop_sum2;   // stop_sum2: test sum |H|^2 < tol^2, else max |H| < tol
  long long evals, iters, pcg_total, max_evals;
  long long launches_done;       // phases executed
  long long nphase[4];           // executed PREP, CG0 / MG, CG / PCG_A + PCG_B, FIELD phases
  int precond, mg_op, mg_lev, rcur;   // preconditioner in use; V-cycle position; residual parity
  int mg_first, chain;           // chain: trial energies = accepted energy + the FIELD phase's change
  int max_halvings, halvings;    // line-search halvings allowed (0: down to tau_floor) and taken
  double alg_bytes;              // algorithmic bytes of the executed phases (roofline accounting)
  // options and constants
  double tol, pcg_rtol2, c1, rho, kappa0, theta0, tau_min, tau_max, tau_floor;
  double e_chain;                // accepted energy of the chain (chain mode)
  // stagnation test of the chain mode: energy and torque at the last
  // progress, FP32 resolution of the energy, accepted steps since
  double prog_e, prog_T, e_res;
  int stall, pad3;
  // potential buffers (indices into u3): the working one, the accepted
  // state's, and the two a PREP starts from (u_src2 < 0: u_src alone; else
  // the interpolation u_src + rho (u_src2 - u_src) after a rejected trial)
  int ucur, uacc, u_src, u_src2;
  double u_w;                    // weight of u_src2 - u_src in the start of the solve
  double step_proj;              // projection of the next step on the last one (s_new.s / s.s, first order)
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
  double gam, dlt, bb, rr, ru, alpha, beta;
  double pad1[4];
};
static_assert(sizeof(Ctrl) % 8 == 0, "Ctrl is copied as 8-byte words");

// One level of the multigrid hierarchy (level 0 is the potential matrix).
// wd = w / diag, w the V-cycle smoother's damped-Jacobi weight.
// Two node values gathered together: one 16-byte (8-byte in FP32) load per
// neighbour instead of two.
template <typename real>
struct alignas(2 * sizeof(real)) Pair {
  real a, b;
};

// The descriptors below are filled by the host with plain pointers and read
// by the kernels through global-address-space pointers of the same size and
// value, so that their loads compile to global (not flat) memory
// instructions.
template <typename T>
using HostPtr = T*;
template <typename T>
using DevPtr = __attribute__((address_space(1))) T*;
template <typename T>
using DevRef = __attribute__((address_space(1))) T&;

template <typename real, template <typename> class Ptr>
struct MgLevelT {
  int n, n_next;
  int lanes_a, lanes_q, lanes_r, lanes_m;   // lanes per row for A, Q, R, M in CSR: 4, 8, 16 or 32
  int m_blocks;            // blocks of 512 (scaled to the launch's) that sweep M in DOWN; 0: no M,
                           // the level restricts in a REST operation of its own
  int pad;
  Ptr<const int> arp;
  Ptr<const int> aci;
  Ptr<const real> av;
  Ptr<const real> wd;
  Ptr<const int> qrp;          // Q: n x n_next, the pattern of A P with value pairs {(A P)_ik, P_ik}
  Ptr<const int> qci;
  Ptr<const Pair<real>> qv;
  Ptr<const int> rrp;          // R = P^T: n_next x n
  Ptr<const int> rci;
  Ptr<const real> rv;
  Ptr<const int> mrp;          // M = R (I - A wd): n_next x n, b_{l+1} = M b
  Ptr<const int> mci;
  Ptr<const real> mv;
  // sliced copies (64-row slices, as the potential matrix) of A, Q and R;
  // null when the matrix has too few rows to fill the GPU one row per thread
  Ptr<const int> aso;
  Ptr<const int> asc;
  Ptr<const real> asv;
  Ptr<const int> qso;          // Q sliced: the (A P) values; P's values of the row
  Ptr<const int> qsc;          // fronts (each row lists P's columns first) in
  Ptr<const real> qsv;         // slices of their own (offsets qpo)
  Ptr<const int> qpo;
  Ptr<const real> qpv;
  Ptr<const int> rso;
  Ptr<const int> rsc;
  Ptr<const real> rsv;
  // sliced rows are held in a windowed order (rows sorted by length inside
  // windows of 512, which cuts the slices' padding): the row at each
  // position of A's, Q's and R's sliced copies (null: position = row)
  Ptr<const int> aord;
  Ptr<const int> qord;
  Ptr<const int> rord;
  Ptr<real> b;                 // right-hand side (level 0 uses the CG residual)
  Ptr<real> wb;                // wd b (levels >= 1), written with b
  Ptr<real> res;               // residual after pre-smoothing
  Ptr<real> xb;                // after post-smoothing (level 0: the preconditioned residual z)
};

// Per-node state of the potential solve, packed so that one gathered
// neighbour costs one 4-wide load: residual r, L p (s), L D^-1 r (w) and the
// Jacobi factor d = 1/diag(L).
template <typename real>
struct __align__(4 * sizeof(real)) Rec {
  real r, s, w, d;
};

// Index of a phase in the per-problem byte table: plain phases by number,
// V-cycle operations by (op, level).
constexpr int kByteSlots = 16 + 4 * kMaxLevels;
__host__ __device__ inline int byte_slot(int phase, int op, int lev) {
  return phase == PH_MG ? 16 + op * kMaxLevels + lev : phase;
}

template <typename real, template <typename> class Ptr>
struct ProbT {
  int N, Nt, G, blk0;
  int stream, pad_s;          // 1: sliced matrices too large for the Infinity Cache are read non-temporally
  // magnet rows: CSR pattern shared by K, D1 (b = D1 m) and D2 (h_d = -D2 u)
  Ptr<const int> mrp;
  Ptr<const int> mci;
  Ptr<const real> K;          // 2 K_ij / V_i
  Ptr<const real> D1[3];      // sum_e V_e/4 grad(phi_i)|_e
  Ptr<const real> D2[3];      // sum_e V_e/4 grad(phi_j)|_e / V_i
  Ptr<const real> Q[6];       // 2 Q_i / V_i: xx yy zz xy xz yz
  Ptr<const real> V;          // lumped nodal volume
  Ptr<real> m[2][3];          // accepted / trial slots, SoA
  Ptr<real> H[2][3];          // torque m x h per slot
  Ptr<real> h[3];             // effective field (written when store_h)
  Ptr<real> mh[2];            // m.h per slot (FP32 form: with H = m x h it gives h = (m.h) m + H x m)
  // potential rows (magnet rows first): transformed Laplacian in 64-row
  // slices (entry k of row i at lso[i/64] + 64 k + i mod 64, short rows
  // padded with their own column and a zero value)
  Ptr<const int> lso;
  Ptr<const int> lsc;
  Ptr<const real> lsv;
  Ptr<const real> lsum;       // row sums of the potential matrix (zero but on rows next to the
                              // Dirichlet boundary); the FP32 form takes L u as
                              // sum_j L_ij (u_j - u_i) + lsum_i u_i
  Ptr<real> u3[3];            // potential buffers: the CG iterate (Ctrl::ucur) and the accepted
                              // state's potential (Ctrl::uacc), the warm starts across solves
  Ptr<real> p;                // search direction (row-local)
  Ptr<Rec<real>> rec[2];      // CG state by buffer parity (pcur)
  // multigrid-preconditioned CG (absent when n_lev == 0)
  int n_lev;              // levels with a coarser level below them
  int mg_fused;           // bit l: level l's DOWN also restricts (MgLevel::m_blocks > 0)
  int nc;                 // size of the coarsest level
  Ptr<const MgLevelT<real, Ptr>> lev;
  Ptr<const real> Ainv;       // dense inverse of the coarsest operator, row-major nc x nc
  Ptr<const real> AinvM;      // nullable: Ainv M of the last level, row-major nc x n_last; the
                              // last DOWN then forms x_c = Ainv M b itself and SOLVE is skipped
  Ptr<real> bc;               // coarsest right-hand side and solution
  Ptr<real> xc;
  Ptr<real> r2[2];            // residual by parity (rcur)
  Ptr<Pair<real>> zp;         // {z, p}: preconditioned residual and search direction
  Ptr<Pair<real>> rq;         // {wd r, wd q} of the current iteration
  Ptr<real> q;                // L p
  Ptr<const double> btab;     // algorithmic bytes per executed phase, indexed by byte_slot()
  // reductions and control
  Ptr<unsigned> ndone;        // nullable: incremented once when the problem finishes
  Ptr<int> done_list;         // nullable: receives `slot` at position ndone - 1
  int slot;
  Ptr<double> part;           // [2][kNPart][G] per-block partials (slot-major), by launch parity
  Ptr<Ctrl> ctrl;             // [2] control state, by launch parity
};

template <typename real>
using MgLevel = MgLevelT<real, HostPtr>;
template <typename real>
using MgLevelDev = MgLevelT<real, DevPtr>;
template <typename real>
using Prob = ProbT<real, HostPtr>;
template <typename real>
using ProbDev = ProbT<real, DevPtr>;
static_assert(sizeof(ProbDev<double>) == sizeof(Prob<double>) && sizeof(MgLevelDev<float>) == sizeof(MgLevel<float>),
              "device views must match the host layout");

}  // namespace mmsd
