// Host runtime objects behind the C ABI: contexts, problems, batched runs.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "amg.h"
#include "assemble.h"
#include "device.h"
#include "mmsd.h"

struct mmsd_ctx_s;

namespace mmsd {

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define MMSD_HIP(call)                         \
  do {                                         \
    hipError_t _e = (call);                    \
    if (_e != hipSuccess) return hip_fail(_e, #call); \
  } while (0)

template <typename real>
hipError_t launch_step(int lpr, const Prob<real>* probs, int nprob, const int* blk_start, int grid, int parity,
                       hipStream_t s);
hipError_t launch_ctrl_init(Ctrl* ctrl, int slot, int stage, int terms, int nonmono_M, int step_rule,
                            int pcg_maxit, int store_h, int demag, int acc, int precond, int chain,
                            int max_halvings, int stop_sum2, int ucur, long long max_evals,
                            const double* dparams, hipStream_t s);

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t s);

// Operators assembled on the device into buffers the library allocated from
// a context's allocator (FP64 values; the layouts of mmsd_assembly_export).
struct DeviceAssembly {
  int64_t N = 0, nnzM = 0, Nt = 0, nnzL = 0;
  int32_t *mrp = nullptr, *mci = nullptr, *pot_global = nullptr, *lrp = nullptr, *lci = nullptr;
  double *K = nullptr, *D1 = nullptr, *D2 = nullptr, *Q = nullptr, *V = nullptr, *L = nullptr;
  std::vector<void*> owned;
  void release(mmsd_ctx_s* c);   // waits for the context's stream, frees every owned buffer
};
// Validate, number and assemble on the device (mmsd_assemble_device's
// kernels) into owned buffers; S receives the host structure.  Takes the
// context's lock.  On failure nothing stays allocated.
int assemble_device_owned(mmsd_ctx_s* c, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats,
                          DeviceAssembly* out, AssemblyStructure* S);
// FP64 -> real copy of n values (device to device).
template <typename real>
hipError_t launch_to_real(const double* src, real* dst, int64_t n, hipStream_t s);
// CSR (rp, ci, v) of n rows into the 64-row sliced layout with the slice
// offsets so[(n + 63) / 64 + 1] (every slice as wide as its longest row),
// plus the FP64 row sums (lsum) and the diagonal's reciprocal in the d field
// of the two CG record buffers (rec0, rec1: 4 reals per row).
template <typename real>
hipError_t launch_slice_rows(const int32_t* rp, const int32_t* ci, const double* v, const int32_t* so, int64_t n,
                             int32_t* sc, real* sv, real* lsum, real* rec0, real* rec1, hipStream_t s);

// Every batch of step launches starts with parity 0 and has an even length,
// so the state a run is armed with goes into slot 1.
constexpr int kArmSlot = 1;

// The newer of the two control slots.
inline const Ctrl& latest(const Ctrl* two) { return two[1].seq > two[0].seq ? two[1] : two[0]; }

struct Resolved {
  double tol, rtol;
  int64_t max_evals;
  int terms, M, rule, maxit, precond, stop;
  double refine;
};

// One launch table: nprob problems of one precision.
struct Table {
  int precision;
  const void* dprobs;
  const int* dblk;
  int nprob, grid, lpr;
};

struct TimingState {
  int stride = 0;                      // 0 = off
  double ms = 0, count = 0, bytes = 0;
  std::vector<hipEvent_t> pool;        // free events
  std::vector<hipEvent_t> pending;     // recorded (start, end) pairs not yet read
  std::vector<double> pending_launches;  // step launches inside each pair
};

}  // namespace mmsd

struct mmsd_ctx_s;
struct mmsd_problem_s;

namespace mmsd {
int resolve(mmsd_problem_s* p, const mmsd_options* o, Resolved* r);
int arm(mmsd_problem_s* p, const Resolved& r, int stage, int store_h);
int launch_table(const Table& t, int parity, hipStream_t st);
void fill_result(mmsd_problem_s* p, const Ctrl& C, mmsd_result* out, double secs, int64_t launches);
int ensure_pinned(mmsd_problem_s* p);
int issue(mmsd_ctx_s* c, const std::vector<Table>& tabs, int B, std::map<int, hipGraphExec_t>* graphs);
int batch_blocks(mmsd_problem_s* p, bool demag);
double run_bytes(mmsd_problem_s* p, const Ctrl& C);
}  // namespace mmsd

struct mmsd_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  mmsd_alloc_fn alloc = nullptr;
  mmsd_free_fn free_fn = nullptr;
  void* user = nullptr;
  int lpr = 4;
  int max_blocks = 512;
  int vcycle = MMSD_VC_FUSE_REST | MMSD_VC_FOLD_SOLVE;   // V-cycle forms for new problems
  int assembly = MMSD_ASSEMBLE_HOST;                     // where new problems' operators are assembled
  bool use_graph = true;
  mmsd::TimingState timing;
  std::map<int64_t, std::pair<int, int>> tuned;   // autotuner results by problem class
  std::mutex mu;            // serializes device work issued through this context
  void* dalloc(size_t bytes);
  void dfree(void* p);
};

struct mmsd_problem_s {
  mmsd_ctx ctx = nullptr;
  int precision = MMSD_FP64;
  mmsd::Assembly A;
  // device arena
  char* arena = nullptr;
  size_t arena_bytes = 0;
  // descriptor (host copy; device copy at dprob) and launch table
  alignas(16) unsigned char desc[sizeof(mmsd::Prob<double>)];
  void* dprob = nullptr;     // device Prob<real>
  int* dblk = nullptr;       // device blk_start [2]
  mmsd::Ctrl* dctrl = nullptr;            // [2] slots
  void* snap[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [set][m | u]
  int G = 0, lpr = 4;
  int acc = 0;
  int ucur = 0;                           // potential buffer holding the current potential
  bool h_valid = false;
  double b_ext[3] = {0, 0, 0};
  double btab[mmsd::kByteSlots] = {};     // algorithmic bytes per executed phase (also on the device)
  double phase_bytes_h = 0;               // extra FIELD bytes when h is stored
  double prep_bytes_nodemag = 0;
  // multigrid preconditioner of the potential solve
  bool has_amg = false;
  mmsd::AmgHierarchy amg;                 // host copy (sizes; values uploaded)
  std::vector<int64_t> amg_q_nnz;         // entries of each level's fused prolongation/smoothing matrix
  std::vector<int64_t> amg_m_nnz;         // entries of each level's residual restriction (levels >= 1)
  std::vector<int> amg_q_sliced;          // 1: the level's Q is swept from its sliced form
  bool amg_folded = false;                // the last DOWN forms the coarsest solution (Ainv M)
  char* amg_arena = nullptr;
  size_t amg_bytes = 0;
  mmsd::Ctrl* hctrl = nullptr;            // pinned mirrors [2 polls][2 slots]
  std::map<int, hipGraphExec_t> graphs;   // batch size -> instantiated graph
  int64_t last_launches = 0;
  double setup_t[4] = {0, 0, 0, 0};       // creation: assembly, multigrid setup, device build, total (s)
};
