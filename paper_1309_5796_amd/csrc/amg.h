// Host setup of the algebraic multigrid preconditioner for the scalar-potential
// solve: smoothed aggregation (Jacobi-smoothed prolongation on the first
// `smooth_levels` levels, plain aggregation below), Galerkin coarse
// operators, dense inverse on the coarsest level.
#pragma once
#include <atomic>
#include <cstdint>
#include <functional>
#include <vector>

namespace mmsd {

struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
};

struct AmgLevel {
  Csr A;                   // operator of this level
  std::vector<double> dinv;
  double omega = 0;        // prolongation smoothing weight 4 / (3 rho(D^-1 A))
  double wsmooth = 0;      // the V-cycle smoother's damped-Jacobi weight (amg_setup)
  Csr P;                   // prolongation to this level from the next coarser one
  Csr R;                   // restriction, the transpose of P
  Csr AP;                  // A P (formed for the Galerkin product; post-smoothing sweeps it)
};

struct AmgHierarchy {
  std::vector<AmgLevel> lv;      // levels 0 .. L-1 (each with P/R to level l+1)
  int nc = 0;                    // size of the coarsest level L
  std::vector<double> Ainv;      // dense inverse of the coarsest operator, row-major
  double complexity = 0;         // total nonzeros of all operators / nonzeros of A_0
};

struct AmgParams {
  double theta = 0.04;           // strength of connection |a_ij| >= theta sqrt(a_ii a_jj)
  int smooth_levels = 10;        // levels whose prolongation is Jacobi-smoothed (all, with p_drop)
  int coarse_max = 600;          // stop coarsening at or below this size
  int max_levels = 10;
  double p_drop = 0.1;           // drop smoothed-P entries below this fraction of the row's largest
  // The V-cycle smoother's weight: smooth_scale x omega, capped at 1.9 / g
  // with g a Gershgorin bound of rho(D^-1 A) (the smaller of those of D^-1 A
  // and of D^-1/2 A D^-1/2), so that the damped Jacobi sweep stays
  // convergent whatever the power iteration's estimate of rho.  In a CPU
  // model of the preconditioned CG (to 1e-10 from zero), 1.2 x omega took 24
  // instead of 26 iterations on the 80 nm cube and 27 instead of 28 on the
  // polycrystal (where the cap binds on the two coarsest levels); 1.3 x was
  // no better and 1.45 x diverged.
  double smooth_scale = 1.2;
};

// Runs f(a, b) over [0, n) cut into contiguous ranges, on up to 16 threads
// (one for n < 2048), and on the calling thread's share of the cores when a
// sharing counter is set (below).
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& f);

// Threads that share the cores: while `active` is set on a thread, its
// parallel_for calls use at most cores / *active threads (the server's setup
// workers set it to their count of busy workers).  nullptr: no sharing.
void share_cores(const std::atomic<int>* active);

// M = R (I - A W) with W = wsmooth D^-1: the restriction of the residual left
// by one damped-Jacobi sweep from zero, b_{l+1} = M b_l.  For symmetric A,
// R A = (A P)^T, so M = R - (A P)^T W, with the pattern of (A P)^T (which
// holds R's, A's diagonal being stored); rows with ascending columns.
Csr residual_restriction(const AmgLevel& L);

// Build the hierarchy for the symmetric positive definite CSR matrix A
// (taken by value: pass a moved copy to spare one).  Returns false (and
// leaves h empty) when the matrix does not coarsen.
bool amg_setup(Csr A, const AmgParams& prm, AmgHierarchy* h);

}  // namespace mmsd
