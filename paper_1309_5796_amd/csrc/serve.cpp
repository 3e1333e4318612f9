// Continuous-batching server of minimizations.
//
// Two host threads per server:
//  * the setup thread admits queued requests in arrival order while the sum
//    of resident device footprints stays within the HBM budget and a slot is
//    free, assembles each mesh on the host and uploads it on its own stream,
//    then hands the armed problem to the device loop;
//  * the device loop launches the step kernel over one descriptor table of
//    all resident problems (one table per precision), so every launch
//    advances each of them by one phase, and problems that arrive while
//    others run join at the next table rebuild.  A finishing problem writes
//    its slot into a device done list; the loop reads it one launch batch
//    behind, copies the result out and frees the slot and its memory.
// Each problem keeps its own block decomposition, so its result does not
// depend on what else is resident.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>

#include "amg.h"
#include "runtime.h"

using namespace mmsd;

namespace {

using Clock = std::chrono::steady_clock;

size_t align_up_bytes(size_t x) { return (x + 255) & ~size_t(255); }

// Setup workers: host assembly and multigrid setup of several requests overlap
// (only their uploads serialize on the upload context).  Measured on the
// 60-request stream: 1 worker p50 10.1 s, 3 workers 4.8 s, 6 workers 3.3 s;
// 10 and 12 workers were slower (4.4 and 5.3 s: the host CPU is saturated).
// The busy workers split the cores between their parallel loops (6 workers:
// p50 2.7-3.0 s).
constexpr int kSetupThreads = 6;

enum ReqState { RQ_QUEUED, RQ_SETUP, RQ_READY, RQ_RESIDENT, RQ_DONE, RQ_FAILED, RQ_CANCELLED };

struct Request {
  uint64_t ticket = 0;
  std::vector<double> xyz, shell;
  std::vector<int32_t> tets, region;
  std::vector<uint8_t> dir;
  std::vector<mmsd_material> mats;
  double b[3] = {0, 0, 0};
  int precision = MMSD_FP64;
  std::vector<double> m0;
  mmsd_options opts{};
  size_t footprint = 0;    // device bytes: estimate (sizing), exact once resident
  bool sized = false;      // footprint known (sizing runs on a setup worker, not in submit)
  bool sizing = false;     // a worker is sizing it
  int size_rc = MMSD_OK;   // sizing failed (invalid mesh)
  ReqState state = RQ_QUEUED;
  bool cancel = false;
  mmsd_problem prob = nullptr;
  mmsd_result result{};
  int status = 0;
  std::string error;
  std::vector<double> m_final;
  Clock::time_point t_submit;
  int slot = -1;
  bool demag = true;       // the resolved terms include the demagnetizing field

  mmsd_mesh mesh() const {
    mmsd_mesh m;
    m.n_nodes = (int64_t)xyz.size() / 3;
    m.xyz = xyz.data();
    m.n_tets = (int64_t)tets.size() / 4;
    m.tets = tets.data();
    m.tet_region = region.data();
    m.dirichlet = dir.empty() ? nullptr : dir.data();
    m.shell = shell.empty() ? nullptr : shell.data();
    return m;
  }
};

}  // namespace

struct mmsd_server_s {
  mmsd_ctx user_ctx = nullptr;
  mmsd_ctx upload_ctx = nullptr;   // own stream, hipMalloc
  mmsd_ctx loop_ctx = nullptr;     // own stream for the step launches
  size_t budget = 0;
  int max_slots = 0;
  std::mutex mu;
  std::condition_variable cv_setup, cv_loop;
  std::deque<Request*> queue;
  std::vector<Request*> ready;     // uploaded, waiting to join
  std::map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1;
  size_t bytes_reserved = 0;
  int slots_used = 0;
  bool stop = false;
  double n_submitted = 0, n_completed = 0, launches = 0, node_evals = 0;
  double setup_seconds = 0, loop_seconds = 0;   // summed over setups; device loop busy time
  std::vector<std::thread> setup_thr;   // host assembly, multigrid setup and upload overlap across threads
  std::atomic<int> busy_setups{0};      // workers inside a setup: they share the cores
  std::thread loop_thr;
  // device-side tables (owned by the loop thread)
  char* dtab = nullptr;
  size_t dtab_bytes = 0;
  unsigned* hdone = nullptr;       // pinned [2 + max_slots]

  void setup_loop();
  void device_loop();
};

namespace {

void finish_request(mmsd_server_s* s, Request* r, int status) {
  r->status = status;
  r->state = status == MMSD_E_CANCELLED ? RQ_CANCELLED : (status < 0 ? RQ_FAILED : RQ_DONE);
  auto t = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
  r->result.seconds = t;
  r->result.status = status;
  s->n_completed += 1;
}

}  // namespace

void mmsd_server_s::setup_loop() {
  (void)hipSetDevice(upload_ctx->device);   // a failure surfaces in the calls that follow
  mmsd::share_cores(&busy_setups);          // the setup's parallel loops split the cores among busy workers
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    Request* r = nullptr;
    Request* tosize = nullptr;   // the first queued request nobody has sized yet
    for (Request* q : queue)
      if (!q->sized && !q->sizing && !q->cancel) {
        tosize = q;
        break;
      }
    // a request being sized stays queued (its worker still writes to it), cancelled or not
    if (!queue.empty() && !queue.front()->sizing && (queue.front()->sized || queue.front()->cancel)) {
      Request* f = queue.front();
      if (f->cancel) {
        queue.pop_front();
        finish_request(this, f, MMSD_E_CANCELLED);
        continue;
      }
      if (f->size_rc != MMSD_OK) {
        queue.pop_front();
        finish_request(this, f, f->size_rc);
        continue;
      }
      if (f->footprint > budget) {
        queue.pop_front();
        f->error = "request footprint exceeds the server's HBM budget";
        finish_request(this, f, MMSD_E_NOMEM);
        continue;
      }
      if (slots_used < max_slots && bytes_reserved + f->footprint <= budget) {
        queue.pop_front();
        r = f;
        bytes_reserved += r->footprint;
        slots_used += 1;
        r->state = RQ_SETUP;
      }
    }
    if (!r && tosize) {
      // size a queued request outside the lock (admission needs its bytes)
      tosize->sizing = true;
      const mmsd_mesh m = tosize->mesh();
      const int precision = tosize->precision;
      lk.unlock();
      busy_setups.fetch_add(1);
      size_t fp = 0;
      const int rc = mmsd_footprint(&m, precision, &fp);
      const std::string err = rc ? mmsd_last_error() : std::string();
      busy_setups.fetch_sub(1);
      lk.lock();
      tosize->footprint = fp;
      tosize->size_rc = rc;
      if (rc) tosize->error = err;
      tosize->sized = true;
      tosize->sizing = false;
      cv_setup.notify_all();
      continue;
    }
    if (!r) {
      cv_setup.wait_for(lk, std::chrono::milliseconds(20));
      continue;
    }
    lk.unlock();
    // assemble + upload outside the lock
    const auto t_setup = Clock::now();
    busy_setups.fetch_add(1);
    mmsd_mesh m = r->mesh();
    mmsd_problem p = nullptr;
    int rc = mmsd_problem_create(upload_ctx, &m, r->mats.data(), (int)r->mats.size(), r->precision, &p);
    if (!rc) rc = mmsd_set_field(p, r->b);
    if (!rc && !r->m0.empty()) rc = mmsd_set_m(p, r->m0.data());
    Resolved res;
    if (!rc) rc = resolve(p, &r->opts, &res);
    if (!rc) r->demag = (res.terms & MMSD_DEMAG) != 0;
    if (!rc) {
      std::lock_guard<std::mutex> g(upload_ctx->mu);
      rc = ensure_pinned(p);
      if (!rc) rc = arm(p, res, ST_INIT, 0);
      if (!rc && hipStreamSynchronize(upload_ctx->stream) != hipSuccess) rc = MMSD_E_HIP;
    }
    if (rc) r->error = mmsd_last_error();
    lk.lock();
    busy_setups.fetch_sub(1);
    setup_seconds += std::chrono::duration<double>(Clock::now() - t_setup).count();
    if (rc) {
      if (p) mmsd_problem_destroy(p);
      bytes_reserved -= r->footprint;
      slots_used -= 1;
      finish_request(this, r, rc);
      continue;
    }
    // exact device bytes from here on (admission used the estimate)
    bytes_reserved += p->arena_bytes + p->amg_bytes;
    bytes_reserved -= r->footprint;
    r->footprint = p->arena_bytes + p->amg_bytes;
    r->prob = p;
    r->state = RQ_READY;
    ready.push_back(r);
    cv_loop.notify_one();
  }
}

void mmsd_server_s::device_loop() {
  (void)hipSetDevice(loop_ctx->device);   // a failure surfaces in the calls that follow
  hipStream_t st = loop_ctx->stream;
  std::vector<Request*> resident;
  std::vector<Table> tabs;
  bool dirty = true;
  unsigned processed = 0;
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    // join uploaded problems; drop cancelled ones
    if (!ready.empty()) {
      for (Request* r : ready) {
        r->state = RQ_RESIDENT;
        resident.push_back(r);
      }
      ready.clear();
      dirty = true;
    }
    for (size_t i = 0; i < resident.size();) {
      Request* r = resident[i];
      if (r->cancel) {
        lk.unlock();
        (void)hipStreamSynchronize(st);   // errors surface in the next batch's checks
        mmsd_problem_destroy(r->prob);
        lk.lock();
        r->prob = nullptr;
        bytes_reserved -= r->footprint;
        slots_used -= 1;
        finish_request(this, r, MMSD_E_CANCELLED);
        resident.erase(resident.begin() + i);
        dirty = true;
        cv_setup.notify_one();
      } else {
        ++i;
      }
    }
    if (resident.empty()) {
      cv_loop.wait_for(lk, std::chrono::milliseconds(20));
      continue;
    }
    lk.unlock();
    int rc = MMSD_OK;
    if (dirty) {
      // rebuild the descriptor tables (no launch is in flight)
      if (hipStreamSynchronize(st) != hipSuccess) rc = MMSD_E_HIP;
      tabs.clear();
      std::vector<int> idx[2];
      for (size_t i = 0; i < resident.size(); ++i) idx[resident[i]->precision == MMSD_MIXED ? 1 : 0].push_back((int)i);
      size_t need = 256 + align_up_bytes(4 * (size_t)(resident.size() + 2));
      for (int q = 0; q < 2; ++q)
        need += 2 * 256 + sizeof(Prob<double>) * idx[q].size() + 4 * (idx[q].size() + 1);
      if (need > dtab_bytes) {
        if (dtab) (void)hipFree(dtab);
        dtab = nullptr;
        dtab_bytes = 0;
        if (hipMalloc((void**)&dtab, 2 * need) == hipSuccess) dtab_bytes = 2 * need;
      }
      if (!dtab) rc = MMSD_E_NOMEM;
      unsigned* dndone = (unsigned*)dtab;
      int* dlist = (int*)(dtab + 256);
      size_t off = 256 + align_up_bytes(4 * (size_t)(resident.size() + 2));
      if (!rc && hipMemsetAsync(dtab, 0, 256, st) != hipSuccess) rc = MMSD_E_HIP;
      // the host sources of the table copies live until the stream is
      // synchronized below: an asynchronous copy may read them after the call
      std::vector<unsigned char> hq[2];
      std::vector<int> bq[2];
      for (int q = 0; q < 2 && !rc; ++q) {
        if (idx[q].empty()) continue;
        const size_t ps = q ? sizeof(Prob<float>) : sizeof(Prob<double>);
        std::vector<unsigned char>& h = hq[q];
        std::vector<int>& blk = bq[q];
        h.assign(ps * idx[q].size(), 0);
        blk.assign(idx[q].size() + 1, 0);
        int lpr = resident[idx[q][0]]->prob->lpr;
        for (size_t k = 0; k < idx[q].size(); ++k) {
          Request* r = resident[idx[q][k]];
          mmsd_problem p = r->prob;
          const int g = batch_blocks(p, r->demag);
          blk[k + 1] = blk[k] + g;
          std::memcpy(&h[k * ps], p->desc, ps);
          if (q) {
            auto* d = reinterpret_cast<Prob<float>*>(&h[k * ps]);
            d->G = g;
            d->blk0 = blk[k];
            d->ndone = dndone;
            d->done_list = dlist;
            d->slot = idx[q][k];
          } else {
            auto* d = reinterpret_cast<Prob<double>*>(&h[k * ps]);
            d->G = g;
            d->blk0 = blk[k];
            d->ndone = dndone;
            d->done_list = dlist;
            d->slot = idx[q][k];
          }
        }
        char* dp = dtab + off;
        off += align_up_bytes(h.size());
        char* db = dtab + off;
        off += align_up_bytes(4 * blk.size());
        if (hipMemcpyAsync(dp, h.data(), h.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(db, blk.data(), 4 * blk.size(), hipMemcpyHostToDevice, st) != hipSuccess)
          rc = MMSD_E_HIP;
        tabs.push_back(Table{q ? MMSD_MIXED : MMSD_FP64, dp, (const int*)db, (int)idx[q].size(), blk.back(), lpr});
      }
      if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = MMSD_E_HIP;
      processed = 0;
      dirty = false;
    }
    // a batch of launches, then read the done list
    const int B = 16;
    const auto t_batch = Clock::now();
    if (!rc) rc = issue(loop_ctx, tabs, B, nullptr);
    if (!rc && hipMemcpyAsync(hdone, dtab, sizeof(unsigned), hipMemcpyDeviceToHost, st) != hipSuccess) rc = MMSD_E_HIP;
    if (!rc && hipMemcpyAsync(hdone + 2, dtab + 256, sizeof(int) * resident.size(), hipMemcpyDeviceToHost, st) !=
                   hipSuccess)
      rc = MMSD_E_HIP;
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = MMSD_E_HIP;
    lk.lock();
    loop_seconds += std::chrono::duration<double>(Clock::now() - t_batch).count();
    launches += B * tabs.size();
    if (rc) {
      // a device failure poisons every resident request
      for (Request* r : resident) {
        r->error = "device failure in the step loop";
        finish_request(this, r, rc);
      }
      resident.clear();
      continue;
    }
    const unsigned nd = hdone[0];
    std::vector<int> fin;
    for (unsigned k = processed; k < nd; ++k) fin.push_back(((int*)hdone)[2 + k]);
    processed = nd;
    if (fin.empty()) continue;
    std::sort(fin.begin(), fin.end());
    lk.unlock();
    for (int slot : fin) {
      Request* r = resident[slot];
      mmsd_problem p = r->prob;
      Ctrl two[2];
      if (hipMemcpy(two, p->dctrl, 2 * sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess) {
        r->error = "device failure reading the result";
        r->status = MMSD_E_HIP;
        continue;
      }
      const Ctrl& C = latest(two);
      p->acc = C.acc;
      p->ucur = C.ucur;
      fill_result(p, C, &r->result, 0.0, C.launches_done);
      r->m_final.resize(3 * (size_t)p->A.N);
      if (mmsd_get_m(p, r->m_final.data()) != MMSD_OK) {
        r->error = mmsd_last_error();
        r->status = MMSD_E_HIP;
        continue;
      }
      r->status = C.status;
    }
    (void)hipStreamSynchronize(st);   // errors surface in the next batch's checks
    lk.lock();
    for (int k = (int)fin.size() - 1; k >= 0; --k) {
      Request* r = resident[fin[k]];
      node_evals += (double)r->prob->A.N * (double)r->result.evals;
      mmsd_problem p = r->prob;
      r->prob = nullptr;
      lk.unlock();
      mmsd_problem_destroy(p);
      lk.lock();
      bytes_reserved -= r->footprint;
      slots_used -= 1;
      finish_request(this, r, r->status);
      resident.erase(resident.begin() + fin[k]);
    }
    dirty = true;
    cv_setup.notify_one();
  }
}

extern "C" {

int mmsd_server_create(mmsd_ctx ctx, size_t hbm_budget, int max_slots, mmsd_server* out) {
  if (!ctx || !out || hbm_budget == 0 || max_slots < 1 || max_slots > 4096) {
    set_error("bad server arguments");
    return MMSD_E_INVALID;
  }
  auto* s = new mmsd_server_s;
  s->user_ctx = ctx;
  s->budget = hbm_budget;
  s->max_slots = max_slots;
  int rc = mmsd_ctx_create(ctx->device, nullptr, nullptr, nullptr, nullptr, &s->upload_ctx);
  if (!rc) rc = mmsd_ctx_create(ctx->device, nullptr, nullptr, nullptr, nullptr, &s->loop_ctx);
  if (!rc) {
    s->upload_ctx->lpr = s->loop_ctx->lpr = ctx->lpr;
    s->upload_ctx->max_blocks = s->loop_ctx->max_blocks = ctx->max_blocks;
    s->upload_ctx->assembly = ctx->assembly;
    if (hipHostMalloc((void**)&s->hdone, sizeof(unsigned) * (2 + max_slots), hipHostMallocDefault) != hipSuccess)
      rc = MMSD_E_NOMEM;
  }
  if (rc) {
    if (s->upload_ctx) mmsd_ctx_destroy(s->upload_ctx);
    if (s->loop_ctx) mmsd_ctx_destroy(s->loop_ctx);
    delete s;
    return rc;
  }
  for (int k = 0; k < kSetupThreads; ++k) s->setup_thr.emplace_back(&mmsd_server_s::setup_loop, s);
  s->loop_thr = std::thread(&mmsd_server_s::device_loop, s);
  *out = s;
  return MMSD_OK;
}

int mmsd_submit(mmsd_server s, const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, const double b_T[3],
                int precision, const double* m0, const mmsd_options* o, uint64_t* ticket) {
  if (!s || !mesh || !b_T || !ticket || n_mats < 1 || !mats || (precision != MMSD_FP64 && precision != MMSD_MIXED)) {
    set_error("bad submit arguments");
    return MMSD_E_INVALID;
  }
  auto* r = new Request;
  r->xyz.assign(mesh->xyz, mesh->xyz + 3 * mesh->n_nodes);
  r->tets.assign(mesh->tets, mesh->tets + 4 * mesh->n_tets);
  r->region.assign(mesh->tet_region, mesh->tet_region + mesh->n_tets);
  if (mesh->dirichlet) r->dir.assign(mesh->dirichlet, mesh->dirichlet + mesh->n_nodes);
  if (mesh->shell) r->shell.assign(mesh->shell, mesh->shell + 9);
  r->mats.assign(mats, mats + n_mats);
  for (int k = 0; k < 3; ++k) r->b[k] = b_T[k];
  r->precision = precision;
  if (m0) {
    // magnetic-node count is only known after numbering: size from the mesh
    int64_t nmag = 0;
    std::vector<char> ism(mesh->n_nodes, 0);
    for (int64_t e = 0; e < mesh->n_tets; ++e)
      if (mesh->tet_region[e] > 0)
        for (int a = 0; a < 4; ++a) ism[mesh->tets[4 * e + a]] = 1;
    for (char c : ism) nmag += c;
    r->m0.assign(m0, m0 + 3 * nmag);
  }
  if (o) r->opts = *o;
  else mmsd_options_default(&r->opts);
  r->t_submit = Clock::now();   // sized later, on a setup worker
  std::lock_guard<std::mutex> lk(s->mu);
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->queue.push_back(r);
  s->n_submitted += 1;
  *ticket = r->ticket;
  s->cv_setup.notify_one();
  return MMSD_OK;
}

int mmsd_poll(mmsd_server s, uint64_t ticket, mmsd_result* out, double* m_out) {
  if (!s || !out) {
    set_error("bad poll arguments");
    return MMSD_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    set_error("unknown ticket");
    return MMSD_E_INVALID;
  }
  Request* r = it->second;
  if (r->state != RQ_DONE && r->state != RQ_FAILED && r->state != RQ_CANCELLED) return MMSD_E_BUSY;
  *out = r->result;
  if (m_out && !r->m_final.empty()) std::memcpy(m_out, r->m_final.data(), r->m_final.size() * sizeof(double));
  const int st = r->status;
  if (st < 0) set_error(r->error.empty() ? "request failed" : r->error);
  s->reqs.erase(it);
  delete r;
  return st;
}

int mmsd_cancel(mmsd_server s, uint64_t ticket) {
  if (!s) return MMSD_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    set_error("unknown ticket");
    return MMSD_E_INVALID;
  }
  it->second->cancel = true;
  s->cv_setup.notify_one();
  s->cv_loop.notify_one();
  return MMSD_OK;
}

int mmsd_server_stats(mmsd_server s, double st[9]) {
  if (!s || !st) return MMSD_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  double resident = 0;
  for (auto& kv : s->reqs)
    if (kv.second->state == RQ_RESIDENT || kv.second->state == RQ_READY || kv.second->state == RQ_SETUP) resident += 1;
  st[0] = s->n_submitted;
  st[1] = s->n_completed;
  st[2] = resident;
  st[3] = (double)s->queue.size();
  st[4] = (double)s->bytes_reserved;
  st[5] = s->launches;
  st[6] = s->node_evals;
  st[7] = s->setup_seconds;
  st[8] = s->loop_seconds;
  return MMSD_OK;
}

int mmsd_server_destroy(mmsd_server s) {
  if (!s) return MMSD_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_setup.notify_all();
  s->cv_loop.notify_all();
  for (std::thread& t : s->setup_thr) t.join();
  s->loop_thr.join();
  (void)hipSetDevice(s->loop_ctx->device);
  (void)hipStreamSynchronize(s->loop_ctx->stream);
  for (auto& kv : s->reqs) {
    if (kv.second->prob) mmsd_problem_destroy(kv.second->prob);
    delete kv.second;
  }
  if (s->dtab) (void)hipFree(s->dtab);
  if (s->hdone) (void)hipHostFree(s->hdone);
  mmsd_ctx_destroy(s->upload_ctx);
  mmsd_ctx_destroy(s->loop_ctx);
  delete s;
  return MMSD_OK;
}

}  // extern "C"
