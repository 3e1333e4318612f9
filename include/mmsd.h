/*
 * mmsd.h -- C ABI of the MI355X (gfx950) curvilinear steepest-descent
 * micromagnetic energy minimizer.
 *
 * Method: Exl, Bance, Reichel, Schrefl, Stimming, Mauser, "LaBonte's method
 * revisited: an effective steepest descent method for micromagnetic energy
 * minimization" (arXiv:1309.5796).  The library minimizes the total Gibbs
 * free energy (stray field + exchange + anisotropy + Zeeman) of a P1
 * tetrahedral mesh under |m_i| = 1 (Method section, eq. (1)) by the
 * curvilinear search on the sphere (eq. (8)) with Barzilai-Borwein step
 * lengths (eq. (10)) selected by the adaptive rule the paper adopts, a
 * 20-energy nonmonotone line search, and the stopping test on the torque.
 * The stray field comes from a magnetic scalar potential with an open
 * boundary handled by a space transformation (Results, comparison section);
 * the potential is solved on the device by CG preconditioned with an
 * algebraic multigrid V-cycle (built on the host at problem creation) or by
 * Jacobi.
 *
 * Conventions
 *  - Every function returns int: 0 = OK, > 0 = warning (result valid),
 *    < 0 = error (the object is left as it was).  mmsd_last_error() gives a
 *    thread-local message for the last error on the calling thread.
 *  - Host arrays passed in are copied during the call; the caller keeps
 *    ownership and may free them on return.  Host output arrays are written
 *    during the call and are owned by the caller.
 *  - Device memory is owned by the library (allocated through the context's
 *    allocator, default hipMalloc) and released by the matching destroy call.
 *  - SI units at the boundary: metres, tesla (mu0 H and Js), J/m^3, J/m, J.
 *    Fields h returned by mmsd_get_field are in units of Ms (dimensionless).
 *  - A problem handle is used by one host thread at a time.  A server handle
 *    is internally synchronized.
 *  - All work of a context is issued on the context's stream.
 */
#ifndef MMSD_H
#define MMSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MMSD_OK 0
#define MMSD_W_MAXEVALS 1     /* evaluation budget reached before the stopping test */
#define MMSD_W_FLOOR 2        /* backtracking step fell below the floor (in the mixed form
                                 also: the next trial's energy change is below the FP32
                                 resolution of the energy); torque reported */
#define MMSD_E_INVALID (-1)   /* bad argument */
#define MMSD_E_MESH (-2)      /* degenerate/inverted tetrahedron, bad index, bad Dirichlet set */
#define MMSD_E_NOMEM (-3)     /* device or host allocation failed */
#define MMSD_E_HIP (-4)       /* HIP runtime error (the context should be recreated) */
#define MMSD_E_NONFINITE (-5) /* non-finite energy or torque */
#define MMSD_E_BUSY (-6)      /* server: result not ready yet */
#define MMSD_E_CANCELLED (-7) /* server: request was cancelled */

/* precision of a problem */
#define MMSD_FP64 0           /* all storage and arithmetic in FP64 */
#define MMSD_MIXED 1          /* FP32 matrices/vectors/SpMV/updates; FP64 reductions,
                                 energy, step logic and PCG scalars */

/* energy terms (bit mask) */
#define MMSD_EXCH 1
#define MMSD_ANIS 2
#define MMSD_ZEEM 4
#define MMSD_DEMAG 8
#define MMSD_ALL 15

/* preconditioner of the scalar-potential solve */
#define MMSD_PRECOND_AUTO 0   /* multigrid when its setup succeeded, else Jacobi */
#define MMSD_PRECOND_JACOBI 1 /* Jacobi, single-reduction CG: one launch per iteration */
#define MMSD_PRECOND_AMG 2    /* smoothed-aggregation multigrid V(1,1) cycle, PCG */

/* stopping tests (tol = mmsd_options.tol_torque) */
#define MMSD_STOP_MAX_TORQUE 0 /* max_i |m_i x h_i| < tol */
#define MMSD_STOP_SUM_SQ 1     /* sum_i |m_i x h_i|^2 < tol^2: the paper's test on the squared
                                  projected gradient (Results, comparison with the LLG solver) */

/* step-length rules (eq. (10)); ADAPTIVE is the rule the paper uses */
#define MMSD_STEP_ADAPTIVE 0  /* adaptive tau1/tau2 switching with a min-window */
#define MMSD_STEP_ALTERNATE 1 /* plain alternation of tau1 and tau2 */
#define MMSD_STEP_BB1 2
#define MMSD_STEP_BB2 3

typedef struct mmsd_ctx_s* mmsd_ctx;
typedef struct mmsd_problem_s* mmsd_problem;
typedef struct mmsd_server_s* mmsd_server;

/* Device allocator hooks; both NULL selects hipMalloc/hipFree.  alloc returns
 * NULL on failure.  Called only from the thread that calls into the library. */
typedef void* (*mmsd_alloc_fn)(size_t bytes, void* user);
typedef void (*mmsd_free_fn)(void* ptr, void* user);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to
 * issue all work on (e.g. torch.cuda.current_stream().cuda_stream), or NULL
 * for a stream the library creates.  The stream must outlive the context. */
int mmsd_ctx_create(int device, void* hip_stream, mmsd_alloc_fn alloc, mmsd_free_fn free_fn,
                    void* user, mmsd_ctx* out);
int mmsd_ctx_destroy(mmsd_ctx ctx);

/* ---- mesh and materials ------------------------------------------------ */
/* A full potential mesh: magnet + air + transformation shell, P1 tetrahedra
 * (Abstract: standard linear tetrahedral elements). */
typedef struct {
  int64_t n_nodes;
  const double* xyz;          /* [n_nodes*3] node coordinates, metres, AoS */
  int64_t n_tets;
  const int32_t* tets;        /* [n_tets*4] 0-based node ids, either orientation */
  const int32_t* tet_region;  /* [n_tets] >= 1 magnetic region id, 0 = non-magnetic */
  const uint8_t* dirichlet;   /* [n_nodes] 1 = potential fixed to 0 (outer box); may be
                                 NULL when the stray field is never requested */
  const double* shell;        /* [9] open-boundary space transformation: centre c[3],
                                 inner half-extent a[3] (identity for |x_k - c_k| <= a_k),
                                 outer half-extent b[3] (mapped to infinity); NULL = none */
} mmsd_mesh;

typedef struct {
  int32_t region;   /* region id >= 1 */
  double Js_T;      /* saturation polarization mu0 Ms (must be equal for all regions) */
  double K1_Jm3;    /* uniaxial anisotropy constant */
  double A_Jm;      /* exchange constant */
  double easy_axis[3];
} mmsd_material;

/* Bytes of device memory a problem on this mesh will hold, for admission:
 * exact for the first arena (operators, node state, control), plus an
 * allowance for the multigrid hierarchy, whose size is known only after its
 * setup ((24 + 2 s) bytes per potential-matrix entry and 8 s per potential
 * node, s = 8 for FP64, 4 for mixed). */
int mmsd_footprint(const mmsd_mesh* mesh, int precision, size_t* bytes_out);

/* The minimization problem of the Method section, eq. (1): the total Gibbs
 * free energy (stray field + exchange + anisotropy + external) of a mesh of
 * standard linear tetrahedral elements (Abstract), with the stray field from
 * a magnetic scalar potential on the transformed open domain (Results,
 * comparison with the LLG solver).
 * Validate the mesh, assemble the FE operators on the host and upload them.
 * Magnetic nodes are the nodes of region >= 1 tetrahedra, in ascending input
 * order; every magnetic region needs a material.  Errors: MMSD_E_MESH for an
 * index out of range, a degenerate tetrahedron, no magnetic tetrahedra or a
 * magnetic node on the Dirichlet set; MMSD_E_INVALID for a missing material or
 * unequal Js; MMSD_E_NOMEM / MMSD_E_HIP for device failures.  The initial
 * state is m = +z, b_ext = 0, potential 0. */
int mmsd_problem_create(mmsd_ctx ctx, const mmsd_mesh* mesh, const mmsd_material* mats,
                        int n_mats, int precision, mmsd_problem* out);
int mmsd_problem_destroy(mmsd_problem p);
/* Wall seconds of the problem's creation: t[4] = {assembly (host, or device
 * with the copies the host keeps), multigrid setup (host), device build
 * (arena, conversions, uploads, the hierarchy's layout; includes waiting for
 * the context's lock), total}. */
int mmsd_problem_setup_times(mmsd_problem p, double t[4]);

int mmsd_n_magnetic(mmsd_problem p, int64_t* n);   /* N: magnetic nodes */
int mmsd_n_potential(mmsd_problem p, int64_t* n);  /* free (non-Dirichlet) nodes, 0 if none */
/* Operator sizes: sizes[4] = {N, entries of the magnet-row pattern (shared by
 * the exchange and the two gradient operators), N_t, entries of the
 * potential matrix (CSR, before any padding)}.  The measurement of the
 * algorithmic bytes per evaluation uses the average row lengths. */
int mmsd_problem_sizes(mmsd_problem p, int64_t sizes[4]);

/* Material constants of the exchange and anisotropy terms of eq. (1) for one
 * region (re-assembles exchange and anisotropy).  Errors: MMSD_E_INVALID for
 * region < 1, a zero easy axis, Js <= 0, A < 0 or a non-finite K1; the
 * problem keeps its previous material then. */
int mmsd_set_material(mmsd_problem p, const mmsd_material* mat);
/* Applied field b = mu0 H_ext (T), uniform: the external-energy term of
 * eq. (1).  MMSD_E_INVALID for a non-finite component. */
int mmsd_set_field(mmsd_problem p, const double b_ext_T[3]);
/* Magnetization, which eq. (1) constrains to unit length at every node.
 * m: [N*3] AoS, magnetic-node order, host memory copied during the call;
 * each vector is normalized on entry; a zero or non-finite vector gives
 * MMSD_E_INVALID (m unchanged).  mmsd_get_m writes the current accepted
 * state into the caller's [N*3] array. */
int mmsd_set_m(mmsd_problem p, const double* m);
int mmsd_get_m(mmsd_problem p, double* m_out);

/* ---- minimization ------------------------------------------------------ */
typedef struct {
  double tol_torque;    /* stop when max_i |m_i x h_i| < tol (h in units of Ms); default 1e-6 */
  int64_t max_evals;    /* energy-gradient evaluation budget; default 100000 */
  int terms;            /* MMSD_* mask; default MMSD_ALL */
  int nonmono_M;        /* nonmonotone memory (1..64); default 20 (end of Method section) */
  double pcg_rtol;      /* potential solve: stop at |r| <= rtol |b|; default 1e-10 (FP64),
                           1e-6 (mixed) */
  int pcg_maxit;        /* default 5000 */
  int step_rule;        /* MMSD_STEP_*; default adaptive */
  double refine_tol_T;  /* hysteresis: > 0 bisects each switching field to this width (T) */
  int precond;          /* MMSD_PRECOND_*; default AUTO */
  int stop_rule;        /* MMSD_STOP_*; default MMSD_STOP_MAX_TORQUE */
} mmsd_options;

/* Defaults: every field zero selects its default. */
void mmsd_options_default(mmsd_options* o);

typedef struct {
  int status;                 /* MMSD_OK or a warning */
  double energy_J;            /* total energy */
  double e_exch_J, e_anis_J, e_zeem_J, e_demag_J;
  double max_torque;          /* max_i |m_i x h_i| */
  double sum_V_torque2;       /* sum_i V_i |m_i x h_i|^2, m^3 */
  double sum_torque2;         /* sum_i |m_i x h_i|^2, the paper's stopping quantity */
  double m_avg[3];            /* volume average of m */
  int64_t iterations;         /* accepted steps */
  int64_t evals;              /* energy-gradient evaluations, line-search trials included */
  int64_t pcg_iters;          /* potential-solver iterations, summed */
  int64_t launches;           /* device step launches issued */
  double seconds;             /* wall time of the call */
} mmsd_result;

/* Minimize eq. (1) from the current m at the current field by the Method
 * section's scheme: projected gradient (eqs. (2)-(5)), curvilinear step
 * (eqs. (7)-(8), solved in closed form), Barzilai-Borwein step lengths
 * (eq. (10)) with the adaptive switch, first step by an inexact line search
 * and a line search whenever the energy exceeds the last 20 (step length
 * selection); stop when max_i |m_i x h_i| < tol (the paper's Results use
 * the sum of the squared gradient, reported as sum_torque2).  Returns the status
 * (also in out->status): MMSD_OK, MMSD_W_MAXEVALS, MMSD_W_FLOOR, or an error
 * (MMSD_E_NONFINITE when the energy or torque became non-finite; m is then
 * the last accepted state).  The potential is warm-started from the last
 * solve. */
int mmsd_minimize(mmsd_problem p, const mmsd_options* o, mmsd_result* out);

/* One evaluation of eq. (1) and its gradient (no step; the effective field
 * h = -dphi/dm defined below eq. (9), lumped per node; the potential by the
 * preconditioned CG solve) at the current m: energies and torque in *out;
 * the field is then available from mmsd_get_field and the potential from
 * mmsd_get_potential. */
int mmsd_evaluate(mmsd_problem p, const mmsd_options* o, mmsd_result* out);
int mmsd_get_field(mmsd_problem p, double* h_out);        /* [N*3] AoS, units of Ms */
int mmsd_get_potential(mmsd_problem p, double* u_out);    /* [n_nodes] input node order, A;
                                                             Dirichlet and unused nodes 0 */

/* Hysteresis (Introduction: continuation of local minima): for each field
 * b_T[k] (n x 3, T) minimize starting from the previous minimum, with a fresh
 * step-length state.  per_step[k] receives each result.  Switching is a sign
 * change of <m>.u between consecutive steps, u = b_T[k]/|b_T[k]| for the
 * first nonzero field (a sweep may start at zero field).  If
 * o->refine_tol_T > 0 each switching field is bisected from the last
 * unswitched minimum.  b_switch_out (nullable, capacity n) receives the
 * switching fields projected on u (T); *n_switch_out (nullable) their count. */
int mmsd_hysteresis(mmsd_problem p, const double* b_T, int64_t n, const mmsd_options* o,
                    mmsd_result* per_step, double* b_switch_out, int64_t* n_switch_out);

/* Batched form (not in the paper; each problem follows the same Method
 * section scheme as mmsd_minimize, eqs. (1)-(10)).
 * Minimize n independent problems of one context together: every device
 * launch advances all unfinished problems by one phase (one persistent
 * kernel over a problem table; a captured launch graph is replayed until all
 * are done, and finished problems are dropped from the table as they
 * accumulate).  Inside the shared launch a problem runs on
 * min(its own block count, a multiple of 8 covering its rows with about four
 * passes of a 512-thread block) blocks; its result equals its own
 * mmsd_minimize result at that block count bit for bit.  out: [n]. */
int mmsd_minimize_batch(mmsd_problem* probs, int n, const mmsd_options* o, mmsd_result* out);

/* Checkpoint (not in the paper): the state a hysteresis continuation
 * carries from one field point to the next (Introduction).
 * Checkpoint: m, potential warm start and field.  bytes: in = capacity, out =
 * size; buf NULL queries the size.  set_state restores a state taken from a
 * problem on the same mesh and precision. */
int mmsd_get_state(mmsd_problem p, void* buf, size_t* bytes);
int mmsd_set_state(mmsd_problem p, const void* buf, size_t bytes);

/* Kernel timing (measurement aid): when stride > 0 the library brackets every
 * batch of step launches it issues with a pair of HIP events on the context
 * stream (kernels back to back plus the gaps between them).  stats:
 * [0] summed milliseconds, [1] step launches inside the timed batches,
 * [2] algorithmic bytes of the phases those launches executed. */
int mmsd_timing_enable(mmsd_ctx ctx, int stride);
int mmsd_timing_read(mmsd_ctx ctx, double stats[3], int reset);

/* Launch configuration of the step kernel: lanes per CSR row (4, 8 or 16)
 * and maximum blocks per problem (multiple of 8).  0 keeps the current
 * value.  Applies to problems created afterwards. */
int mmsd_set_launch_config(mmsd_ctx ctx, int lanes_per_row, int max_blocks);

/* Forms of the multigrid V(1,1) cycle for problems created afterwards on
 * this context (rearrangements of the same cycle, equal up to rounding):
 *   MMSD_VC_FUSE_REST   on coarse levels where the library's cost model
 *                       finds it pays, the restriction runs inside the
 *                       down-sweep's launch, b_{l+1} = R (I - A wd) b;
 *   MMSD_VC_FOLD_SOLVE  with the last level fused, the coarsest solve too,
 *                       x_c = Ainv R (I - A wd) b.
 *   MMSD_VC_SLICE_ALL   hold every matrix of the hierarchy (the level
 *                       operators, restrictions and fused prolongation
 *                       matrices) in the 64-row sliced layout and sweep it
 *                       one row per thread, whatever its size and row
 *                       length.  By default only matrices of at least
 *                       65,536 rows and at most 24 entries per row on
 *                       average are sliced, which only meshes of about a
 *                       million nodes reach; the option runs those code
 *                       paths on small meshes (tests).
 * Default: MMSD_VC_FUSE_REST | MMSD_VC_FOLD_SOLVE.  0 gives the plain order
 * (REST and SOLVE launches of their own).  Returns MMSD_E_INVALID for other
 * bits. */
#define MMSD_VC_FUSE_REST 1
#define MMSD_VC_FOLD_SOLVE 2
#define MMSD_VC_SLICE_ALL 4
int mmsd_set_vcycle(mmsd_ctx ctx, int flags);

/* Where problems created through this context (and the requests of a server
 * created on it) assemble their operators (Abstract: linear tetrahedral
 * elements; Results, comparison section: the transformed open-boundary
 * Laplacian).  MMSD_ASSEMBLE_HOST (default): the host assembly, uploaded.
 * MMSD_ASSEMBLE_DEVICE: mmsd_assemble_device's kernels build the operators
 * on the device and the problem's sliced potential matrix, row sums and
 * Jacobi factors are formed there too; the host keeps only what later calls
 * need (numbering, the magnet pattern, lumped volumes, the magnetic tets'
 * geometry for mmsd_set_material, and a copy of the potential matrix for the
 * multigrid setup).  The two give the same operators up to the rounding of
 * fused multiply-adds (relative 1e-15); errors are those of
 * mmsd_assemble_device (a node in more than 3,276 tets is MMSD_E_INVALID).
 * Device temporaries of up to ~190 bytes per tet are held during creation.
 * MMSD_E_INVALID for any other value. */
#define MMSD_ASSEMBLE_HOST 0
#define MMSD_ASSEMBLE_DEVICE 1
int mmsd_set_assembly(mmsd_ctx ctx, int where);

/* Measurement aid: `reps` launches of a plain device-to-device copy kernel
 * (k_copy_probe) of `bytes` bytes each; *ms_out (nullable) gets the mean
 * time per launch.  Used to calibrate hardware traffic counters against a
 * known byte count. */
int mmsd_copy_probe(mmsd_ctx ctx, size_t bytes, int reps, double* ms_out);

/* Launch shape of one problem: lanes per CSR row (4, 8, 16) and the block
 * cap (multiple of 8, <= 2048).  Takes effect at the next run. */
int mmsd_set_problem_launch(mmsd_problem p, int lanes_per_row, int max_blocks);

/* Autotuner: times a fixed slice of this problem's potential solve for every
 * lanes-per-row x block-cap shape, keeps the fastest on the problem and in a
 * per-context cache keyed by (precision, log2 N, log2 N_t) (a cached class
 * is applied without timing; *us_out is then -1).  The problem's state (m,
 * potential) is unchanged.  Outputs are nullable. */
int mmsd_autotune(mmsd_problem p, int* lanes_out, int* blocks_out, double* us_out);

/* The autotuner's per-context cache as plain records, so that a caller can
 * keep it across processes (a file, a service) and hand it to a new context
 * instead of timing again.  A record is 5 int32: {precision (MMSD_FP64 or
 * MMSD_MIXED), floor(log2(N + 1)), floor(log2(N_t + 1)), lanes per row,
 * block cap}, the class key and the shape mmsd_autotune keeps.
 * mmsd_autotune_cache_get writes min(cap, count) records to rec (host
 * memory the caller owns, 5 * cap int32; NULL with cap 0 for the count
 * only) in ascending key order and the cache's record count to *n.
 * mmsd_autotune_cache_put adds n records (a class already cached takes the
 * new shape); it checks every record first and adds none if one is invalid
 * (unknown precision, a log2 outside [0, 62], lanes not 4, 8 or 16, blocks
 * not a multiple of 8 in [8, 2048]): MMSD_E_INVALID.  Cached shapes apply
 * to the problems autotuned afterwards, not to existing ones.  Both are
 * host-only and take the context's lock. */
int mmsd_autotune_cache_get(mmsd_ctx ctx, int32_t* rec, int cap, int* n);
int mmsd_autotune_cache_put(mmsd_ctx ctx, const int32_t* rec, int n);

/* Host-side assembly only (no device): sizes[4] = {N, nnz of the magnet
 * pattern, N_t, nnz of the potential matrix}; every array pointer may be
 * NULL (query sizes first).  Values are in the library's internal units
 * (nm, mu0 Ms^2 nm^3): mrp[N+1], mci[nnzM], K[nnzM] (= 2 K_ij / V_i),
 * D1[3*nnzM] and D2[3*nnzM] (component-major), Q[6*N] (xx yy zz xy xz yz,
 * = 2 Q_i / V_i), V[N], pot_global[N_t] (input node of each potential row),
 * lrp[N_t+1], lci[nnzL], L[nnzL], scalars[4] = {sum V_e K1_e / (mu0 Ms^2),
 * sum V_i, Ms, mu0 Ms^2}.  For inspection and tests of the assembly. */
int mmsd_assembly_export(const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, int64_t sizes[4],
                         int32_t* mrp, int32_t* mci, double* K, double* D1, double* D2, double* Q, double* V,
                         int32_t* pot_global, int32_t* lrp, int32_t* lci, double* L, double* scalars);

/* Device-side assembly of the same operators (Abstract: linear tetrahedral
 * elements; Results, comparison section: the transformed open-boundary
 * Laplacian).  The host validates the mesh and materials and numbers the
 * nodes; HIP kernels on ctx's stream build the node-to-tet adjacency and
 * the sparsity patterns and compute the tet geometry, the shell metric and
 * every value.  Arguments and layouts are those of mmsd_assembly_export
 * without scalars, but every array is DEVICE memory the caller owns: all
 * eleven NULL = size query (writes sizes[4]; runs the pattern kernels), all
 * eleven set = assemble, with sizes[4] holding what the query returned (the
 * buffers' sizes; a mismatch is MMSD_E_INVALID before anything is written);
 * a mix of NULL and set is MMSD_E_INVALID.  A node in more than 3,276 tets
 * is MMSD_E_INVALID (a row's candidate columns are held in 64 KB of LDS; the
 * host assembly has no such limit).
 * With N_t = 0, lrp[1] = {0} and lci, L, pot_global are untouched.
 * Temporaries (up to ~190 B per tet: a 128-B geometry record, vertex ids,
 * the node-to-tet adjacencies) come from ctx's allocator and are freed before
 * return; the call returns once the values are written.  Errors: the host
 * checks of mmsd_assembly_export (MMSD_E_MESH / MMSD_E_INVALID), degenerate
 * tets, tets outside the shell and non-positive diagonals found by the
 * kernels (MMSD_E_MESH), more than 2^26 magnetic or potential rows
 * (MMSD_E_INVALID), MMSD_E_NOMEM, MMSD_E_HIP. */
int mmsd_assemble_device(mmsd_ctx ctx, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                         int64_t sizes[4], int32_t* mrp, int32_t* mci, double* K, double* D1, double* D2,
                         double* Q, double* V, int32_t* pot_global, int32_t* lrp, int32_t* lci, double* L);

/* For callers that cannot allocate device memory (a harness that forbids
 * hipMalloc, a tight serving loop): mmsd_assemble_device with the same
 * arguments, layouts, outputs and errors, but its device temporaries come
 * from a fixed 64 MiB region the library holds on each GPU for the life of
 * the process, never from an allocator (no hipMalloc, hipFree or allocating
 * library routine is called).  A mesh whose temporaries need more (about
 * 161 bytes per tetrahedron, 40 per magnetic tetrahedron and 48 per node:
 * some 300,000 tetrahedra) gives MMSD_E_INVALID before any device work.  The
 * region is shared by every call on one GPU and keeps the last call's
 * contents; the call clears what must start at zero.  Calls through one
 * context are serialized; calls through two contexts on the same GPU that
 * overlap race on the region and must not be made.  Host staging (pageable
 * copies, the host-side numbering) is as in mmsd_assemble_device. */
int mmsd_assemble_device_noalloc(mmsd_ctx ctx, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                                 int64_t sizes[4], int32_t* mrp, int32_t* mci, double* K, double* D1,
                                 double* D2, double* Q, double* V, int32_t* pot_global, int32_t* lrp,
                                 int32_t* lci, double* L);

/* ---- serving ----------------------------------------------------------- */
/* Served form (not in the paper; every request is one mmsd_minimize of
 * eq. (1) by the Method section's scheme).
 * A server owns a worker thread that admits submitted minimizations while
 * their device footprint fits in hbm_budget bytes and a slot is free (at
 * most max_slots resident), assembles and uploads them off the critical
 * path, advances every resident problem by one phase per device launch
 * (continuous batching), and releases a slot as soon as its problem is done.
 * A request runs with the block count mmsd_minimize_batch would give it.
 * mmsd_submit copies the request and returns at once; its footprint is sized
 * (mmsd_footprint) by an idle setup worker, in queue order, so a mesh that
 * fails validation is reported by mmsd_poll, not by mmsd_submit. */
int mmsd_server_create(mmsd_ctx ctx, size_t hbm_budget, int max_slots, mmsd_server* out);
int mmsd_submit(mmsd_server s, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                const double b_T[3], int precision, const double* m0 /* nullable: +z */,
                const mmsd_options* o, uint64_t* ticket);
/* MMSD_E_BUSY until done; then the result (and m if m_out != NULL, [N*3]). */
int mmsd_poll(mmsd_server s, uint64_t ticket, mmsd_result* out, double* m_out);
int mmsd_cancel(mmsd_server s, uint64_t ticket);
/* stats: [0] submitted, [1] completed, [2] resident, [3] queued, [4] bytes resident,
 * [5] device launches, [6] node-evaluations completed, [7] seconds spent in request
 * setup (assembly, multigrid setup, upload; summed over the setup workers),
 * [8] seconds the device loop spent in launch batches */
int mmsd_server_stats(mmsd_server s, double stats[9]);
int mmsd_server_destroy(mmsd_server s);

const char* mmsd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MMSD_H */
