// Request server: continuous batching of independent solves on one GPU.
//
// One worker thread owns the GPU side: a range pool over one device arena
// (the HBM budget), a copy stream for uploads of admitted solves and
// downloads of finished ones, and up to six lanes.  A lane is one
// gmunu_batch (each solve one block in its own group) whose stream carries
// all of the lane's work; solves go to a lane by integrator and by kind: 1D
// solves, other small solves (at most kSmallCells interior cells) and large
// ones.  A 1D tube needs thousands of cheap steps, so its lane is not paced
// by the multi-dimensional solves, and replays several steps per captured
// graph (a step of such a lane costs little more than its launches).  The
// lanes' kernels run concurrently on the device.  A lane and its stream are
// made when its first solve arrives, so an unused integrator holds no
// hardware queue.  Callers only touch the pending queue and the result
// queue, both under one mutex.
//
// Loop: admit pending solves in arrival order while a slot, list capacity
// and arena space are free (upload on the copy stream) -> for every lane
// whose round of replays has finished: read each group's (t, dt, steps),
// start the download of finished solves and drop them from the lane -> every
// idle lane takes in its uploaded solves, commits, initialises the new ones
// and launches its next round of replays -> finished downloads return their
// memory.  A batch is only changed while its lane is idle.  Each lane sizes
// its rounds to about kRoundSeconds of device work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/gmunu.h"
#include "batch_internal.hpp"
#include "gmunu_host.hpp"
#include "gmunu_pool.hpp"

using namespace gm;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kAlign = 256;
constexpr long kSmallCells = 1L << 16;  // interior cells of a "small" solve
constexpr double kRoundSeconds = 2e-3;  // device time per round of replays
constexpr int kMaxRound = 64;           // replays per round, at most
constexpr int NLANE = 6;                // (SSPRK2, SSPRK3) x (1D, small, large)
constexpr int kLaneSteps[3] = {8, 2, 1};  // steps per replay: 1D, small, large

struct Req {
  unsigned long long id = 0;
  gmunu_request r;
  double t_submit = 0.0, t_admit = 0.0;
  size_t nv = 0, arr8 = 0, arr5 = 0, bytes = 0, off = RangePool::npos;
  double *qn = nullptr, *qs = nullptr, *prim = nullptr, *met = nullptr;
  int lane = 0, slot = -1;
  BatchItems items{};
  hipEvent_t ev = nullptr;
  int steps = 0, status = GMUNU_OK;
  unsigned int nfatal = 0;
  double t = 0.0;
  bool in_batch = false;
};

// One batch, its stream and its slots.
struct Lane {
  gmunu_batch *b = nullptr;
  hipStream_t st = nullptr;  // the batch's own stream
  hipEvent_t ev = nullptr;
  bool inflight = false;
  int steps = 1;  // steps per replay
  int round = 1;  // replays per round
  double t_launch = 0.0;
  std::vector<Req *> slot;  // resident or uploading, by slot
  std::vector<int> free_slots;
  long stage[kMaxVariants] = {};
  long cells = 0, ghosts = 0;
  std::vector<Req *> joining;  // uploaded, to be added when the lane is idle
  std::vector<int> newly;
  bool dirty = false;
  int resident = 0;
  std::vector<double> t, dt;
  std::vector<int> ns;
  std::vector<unsigned int> nf;

  bool fits(const Req *r, long maxi) const {
    return !free_slots.empty() && stage[r->items.variant] + r->items.stage <= maxi && cells + r->items.cells <= maxi &&
           ghosts + r->items.ghosts <= maxi;
  }
  void take(Req *r) {
    r->slot = free_slots.back();
    free_slots.pop_back();
    slot[r->slot] = r;
    stage[r->items.variant] += r->items.stage;
    cells += r->items.cells;
    ghosts += r->items.ghosts;
  }
  void give_back(Req *r) {
    slot[r->slot] = nullptr;
    free_slots.push_back(r->slot);
    stage[r->items.variant] -= r->items.stage;
    cells -= r->items.cells;
    ghosts -= r->items.ghosts;
  }
};

}  // namespace

struct gmunu_server {
  // fixed at create
  int device = 0;
  double cfl = 0.4;
  int spsync = 1;
  int max_slots = 0;
  long maxi = 0;
  char *arena = nullptr;
  hipStream_t xs = nullptr;
  Lane lane[NLANE];

  // shared with callers (under mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> pending;
  std::deque<gmunu_result> results;
  bool stop = false;
  int error = GMUNU_OK;
  unsigned long long next_id = 1;
  gmunu_server_info info{};

  // worker only
  RangePool pool;
  std::vector<Req *> loading, unloading;
  std::thread worker;

  static int lane_index(const gmunu_grid_desc &d) {
    const long cells = (long)d.n[0] * d.n[1] * d.n[2];
    const int kind = cells > kSmallCells ? 2 : d.ndim == 1 ? 0 : 1;
    return (d.rk == 3 ? 3 : 0) + kind;
  }

  // Make lane k's batch, stream and event on first use.
  bool ensure_lane(int k) {
    Lane &L = lane[k];
    if (L.b) return true;
    if (gmunu_batch_create(max_slots, max_slots, maxi, &L.b) != GMUNU_OK) {
      L.b = nullptr;
      return false;
    }
    L.st = batch_stream(L.b);
    L.steps = kLaneSteps[k % 3];
    L.round = std::max(1, (spsync + L.steps - 1) / L.steps);
    return hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) == hipSuccess;
  }
  Lane &lane_of(const Req *r) { return lane[r->lane]; }
  int resident_total() const {
    int n = 0;
    for (const Lane &L : lane) n += L.resident;
    return n;
  }
  bool any_inflight() const {
    for (const Lane &L : lane)
      if (L.inflight) return true;
    return false;
  }

  void finish(Req *r, int status) {
    gmunu_result res{};
    res.id = r->id;
    res.tag = r->r.tag;
    res.status = status;
    res.steps = r->steps;
    res.nfatal = r->nfatal;
    res.t = r->t;
    res.t_submit = r->t_submit;
    res.t_admit = r->t_admit;
    res.t_done = now_s();
    res.bytes = r->bytes;
    if (r->ev) (void)hipEventDestroy(r->ev);
    delete r;
    std::lock_guard<std::mutex> lk(mu);
    results.push_back(res);
    info.completed++;
    cv_done.notify_all();
  }

  void publish() {
    std::lock_guard<std::mutex> lk(mu);
    info.pending = (long)pending.size();
    info.resident = resident_total();
    info.pool_bytes = pool.capacity();
    info.pool_used = pool.used();
    info.pool_peak = pool.peak();
  }

  bool start_load(Req *r) {
    r->t_admit = now_s();
    char *base = arena + r->off;
    r->qn = reinterpret_cast<double *>(base);
    r->qs = reinterpret_cast<double *>(base + r->arr8);
    r->prim = reinterpret_cast<double *>(base + 2 * r->arr8);
    r->met = reinterpret_cast<double *>(base + 3 * r->arr8);
    loading.push_back(r);
    if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) return false;
    bool ok = hipMemcpyAsync(r->prim, r->r.prim, sizeof(double) * 8 * r->nv, hipMemcpyDefault, xs) == hipSuccess;
    ok = ok && hipMemcpyAsync(r->met, r->r.metric, sizeof(double) * 5 * r->nv, hipMemcpyDefault, xs) == hipSuccess;
    return ok && hipEventRecord(r->ev, xs) == hipSuccess;
  }

  // Solves whose upload finished wait for their lane to be idle.
  bool finish_loads(bool &progress) {
    size_t k = 0;
    for (; k < loading.size(); k++) {
      Req *r = loading[k];
      const hipError_t q = hipEventQuery(r->ev);
      if (q == hipErrorNotReady) break;  // uploads complete in order
      if (q != hipSuccess) return false;
      lane_of(r).joining.push_back(r);
      progress = true;
    }
    loading.erase(loading.begin(), loading.begin() + k);
    return true;
  }

  // An idle lane takes its uploaded solves into its batch.  A solve the
  // batch rejects ends alone with the batch's error code (its slot and memory
  // return); only a HIP error stops the server.
  bool join(Lane &L) {
    for (Req *r : L.joining) {
      gmunu_block blk;
      blk.desc = r->r.desc;
      blk.q_n = r->qn;
      blk.q_s = r->qs;
      blk.prim = r->prim;
      blk.metric = r->met;
      blk.flags = nullptr;
      blk.group = r->slot;
      int rc = gmunu_batch_set_block(L.b, r->slot, &blk);
      if (rc == GMUNU_OK) {
        rc = gmunu_batch_set_group(L.b, r->slot, 0.0, r->r.t_end, r->r.max_steps);
        if (rc != GMUNU_OK && gmunu_batch_clear_block(L.b, r->slot) != GMUNU_OK) return false;
      }
      if (rc == GMUNU_EHIP) return false;
      if (rc != GMUNU_OK) {
        L.give_back(r);
        pool.release(r->off, r->bytes);
        finish(r, rc);
        continue;
      }
      L.newly.push_back(r->slot);
      L.dirty = true;
      L.resident++;
      r->in_batch = true;
    }
    L.joining.clear();
    return true;
  }

  bool start_unload(Lane &L, Req *r, int status) {
    r->status = status;
    bool ok = true;
    if (r->r.q_out)
      ok = hipMemcpyAsync(r->r.q_out, r->qn, sizeof(double) * 8 * r->nv, hipMemcpyDefault, xs) == hipSuccess;
    if (r->r.prim_out)
      ok = ok &&
           hipMemcpyAsync(r->r.prim_out, r->prim, sizeof(double) * 8 * r->nv, hipMemcpyDefault, xs) == hipSuccess;
    ok = ok && hipEventRecord(r->ev, xs) == hipSuccess;
    ok = ok && gmunu_batch_clear_block(L.b, r->slot) == GMUNU_OK;
    L.give_back(r);
    L.resident--;
    L.dirty = true;
    unloading.push_back(r);
    return ok;
  }

  // Finished downloads: return the memory and publish the result.  A solve
  // leaves its lane (commit) before its memory returns, so no later round
  // reads it.
  bool finish_unloads(bool &progress) {
    size_t k = 0;
    for (; k < unloading.size(); k++) {
      Req *r = unloading[k];
      const hipError_t q = hipEventQuery(r->ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return false;
      pool.release(r->off, r->bytes);
      finish(r, r->status);
      progress = true;
    }
    unloading.erase(unloading.begin(), unloading.begin() + k);
    return true;
  }

  // A lane's round finished: solves at their end (or stalled) leave it.
  bool check_lane(Lane &L) {
    if (gmunu_batch_times(L.b, L.t.data(), L.dt.data(), L.ns.data(), L.nf.data(), L.st) != GMUNU_OK) return false;
    for (int s = 0; s < max_slots; s++) {
      Req *r = L.slot[s];
      if (!r || !r->in_batch) continue;  // empty, or still uploading
      r->t = L.t[s];
      r->steps = L.ns[s];
      r->nfatal = L.nf[s];
      const bool done = r->t >= r->r.t_end || (r->r.max_steps > 0 && r->steps >= r->r.max_steps);
      if (done) {
        if (!start_unload(L, r, GMUNU_OK)) return false;
      } else if (!(L.dt[s] > 0.0)) {
        if (!start_unload(L, r, GMUNU_ESTALL)) return false;
      }
    }
    return true;
  }

  // Rounds that finished: adapt the round length, retire finished solves.
  bool poll_lanes(bool &progress) {
    for (Lane &L : lane) {
      if (!L.inflight) continue;
      const hipError_t q = hipEventQuery(L.ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return false;
      L.inflight = false;
      const double dur = now_s() - L.t_launch;
      {
        std::lock_guard<std::mutex> lk(mu);
        info.busy_s += dur;
      }
      const double per = dur / L.round;
      const int want = per > 0.0 ? (int)std::lround(kRoundSeconds / per) : kMaxRound;
      L.round = std::max((spsync + L.steps - 1) / L.steps, std::min(kMaxRound, want));
      if (!check_lane(L)) return false;
      progress = true;
    }
    return true;
  }

  // Idle lanes: commit changes, initialise new solves, launch a round.
  bool launch_lanes(bool &progress) {
    for (Lane &L : lane) {
      if (L.inflight) continue;
      if (!L.joining.empty() && !join(L)) return false;
      if (L.dirty) {
        if (gmunu_batch_commit(L.b, L.st) != GMUNU_OK) return false;
        if (!L.newly.empty() && gmunu_batch_init(L.b, L.newly.data(), (int)L.newly.size(), L.st) != GMUNU_OK)
          return false;
        L.newly.clear();
        L.dirty = false;
      }
      if (!L.resident) continue;
      L.t_launch = now_s();
      for (int k = 0; k < L.round; k++)
        if (batch_step_graph(L.b, cfl, nullptr, L.steps, L.st) != GMUNU_OK) return false;
      if (hipEventRecord(L.ev, L.st) != hipSuccess) return false;
      L.inflight = true;
      progress = true;
      std::lock_guard<std::mutex> lk(mu);
      info.replays += (long)L.round * L.steps;
    }
    return true;
  }

  void fail_all() {
    std::vector<Req *> all;
    {
      std::lock_guard<std::mutex> lk(mu);
      error = GMUNU_ESTOP;
      all.assign(pending.begin(), pending.end());
      pending.clear();
    }
    for (Lane &L : lane)
      for (Req *&r : L.slot)
        if (r) {
          all.push_back(r);
          r = nullptr;
        }
    for (Req *r : unloading)
      if (std::find(all.begin(), all.end(), r) == all.end()) all.push_back(r);
    loading.clear();
    unloading.clear();
    for (Req *r : all) finish(r, GMUNU_ESTOP);
  }

  void run() {
    if (hipSetDevice(device) != hipSuccess) {
      fail_all();
      return;
    }
    for (;;) {
      std::vector<Req *> adm;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (stop) break;
        if (resident_total() == 0 && loading.empty() && unloading.empty() && pending.empty() && !any_inflight())
          cv_work.wait(lk, [&] { return stop || !pending.empty(); });
        if (stop) break;
        while (!pending.empty()) {
          Req *r = pending.front();
          Lane &L = lane_of(r);
          if (!L.fits(r, maxi)) break;
          const size_t off = pool.alloc(r->bytes);
          if (off == RangePool::npos) break;
          pending.pop_front();
          r->off = off;
          L.take(r);
          info.admitted++;
          adm.push_back(r);
        }
      }
      bool ok = true, progress = !adm.empty();
      for (Req *r : adm) ok = ok && ensure_lane(r->lane) && start_load(r);
      ok = ok && finish_loads(progress) && poll_lanes(progress) && launch_lanes(progress) &&
           finish_unloads(progress);
      if (!ok) {
        fail_all();
        break;
      }
      publish();
      if (!progress) {
        if (any_inflight() || !loading.empty() || !unloading.empty())
          std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
    }
    for (Lane &L : lane)
      if (L.b) (void)hipStreamSynchronize(L.st);
    (void)hipStreamSynchronize(xs);
  }
};

extern "C" {

double gmunu_server_clock(void) { return now_s(); }

int gmunu_server_create(size_t hbm_bytes, int max_slots, double cfl, int steps_per_sync, gmunu_server **out) {
  if (!out) return GMUNU_ENULL;
  if (hbm_bytes < (1u << 20) || max_slots < 1 || max_slots > (1 << 20) || !(cfl > 0.0) || steps_per_sync < 1)
    return GMUNU_EINVAL;
  gmunu_server *s = new (std::nothrow) gmunu_server();
  if (!s) return GMUNU_ENOMEM;
  s->cfl = cfl;
  s->spsync = std::min(steps_per_sync, kMaxRound);
  s->max_slots = max_slots;
  // list capacity: a solve needs at most ~4 tiles per 256 of its cells
  // (ragged tiles), plus one per block for the remainders
  const long max_cells = (long)(hbm_bytes / 232);
  s->maxi = std::min(1L << 30, 4 * (max_cells / 256) + 64L * max_slots + 1024);
  bool ok = hipGetDevice(&s->device) == hipSuccess;
  ok = ok && hipMalloc(&s->arena, hbm_bytes) == hipSuccess;
  if (!ok) {
    delete s;
    return GMUNU_ENOMEM;
  }
  s->pool.reset(hbm_bytes);
  ok = hipStreamCreateWithFlags(&s->xs, hipStreamNonBlocking) == hipSuccess;
  for (Lane &L : s->lane) {
    L.slot.assign(max_slots, nullptr);
    for (int k = max_slots - 1; k >= 0; k--) L.free_slots.push_back(k);
    L.t.assign(max_slots, 0.0);
    L.dt.assign(max_slots, 0.0);
    L.ns.assign(max_slots, 0);
    L.nf.assign(max_slots, 0u);
  }
  if (!ok) {
    if (s->xs) (void)hipStreamDestroy(s->xs);
    (void)hipFree(s->arena);
    delete s;
    return GMUNU_EHIP;
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return GMUNU_OK;
}

int gmunu_server_submit(gmunu_server *s, const gmunu_request *req, unsigned long long *id_out) {
  if (!s || !req) return GMUNU_ENULL;
  if (!req->prim || !req->metric) return GMUNU_ENULL;
  const int rc = validate_desc(req->desc);
  if (rc) return rc;
  if (req->desc.pp_limiter) return GMUNU_EINVAL;  // solves run in a batch
  // the batch's rule for a group's end (t_end >= t = 0; NaN fails it), and
  // some end: a finite t_end or a step limit
  if (!(req->t_end >= 0.0)) return GMUNU_EINVAL;
  if (std::isinf(req->t_end) && req->max_steps <= 0) return GMUNU_EINVAL;
  Req *r = new (std::nothrow) Req();
  if (!r) return GMUNU_ENOMEM;
  r->r = *req;
  long nv = 1;
  for (int a = 0; a < 3; a++) nv *= req->desc.n[a] + (a < req->desc.ndim ? 2L * req->desc.ng : 0L);
  r->nv = (size_t)nv;
  r->arr8 = RangePool::round_up(sizeof(double) * 8 * r->nv, kAlign);
  r->arr5 = RangePool::round_up(sizeof(double) * 5 * r->nv, kAlign);
  r->bytes = 3 * r->arr8 + r->arr5;
  r->lane = gmunu_server::lane_index(req->desc);
  r->items = batch_items_for(nullptr, req->desc);  // the server never tunes its batches
  if (r->bytes > s->pool.capacity() || r->items.stage > s->maxi || r->items.cells > s->maxi ||
      r->items.ghosts > s->maxi) {
    delete r;
    return GMUNU_EINVAL;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error || s->stop) {
      delete r;
      return GMUNU_ESTOP;
    }
    r->id = s->next_id++;
    r->t_submit = now_s();
    s->pending.push_back(r);
    s->info.submitted++;
    if (id_out) *id_out = r->id;
  }
  s->cv_work.notify_one();
  return GMUNU_OK;
}

int gmunu_server_poll(gmunu_server *s, gmunu_result *out, int max, int timeout_ms) {
  if (!s || (!out && max > 0)) return GMUNU_ENULL;
  if (max < 0) return GMUNU_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->results.empty() && timeout_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !s->results.empty() || s->error; });
  int n = 0;
  while (n < max && !s->results.empty()) {
    out[n++] = s->results.front();
    s->results.pop_front();
  }
  return n;
}

int gmunu_server_status(gmunu_server *s, gmunu_server_info *out) {
  if (!s || !out) return GMUNU_ENULL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->info;
  out->pending = (long)s->pending.size();
  return s->error;
}

int gmunu_server_destroy(gmunu_server *s) {
  if (!s) return GMUNU_ENULL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Req *r : s->pending) {
    if (r->ev) (void)hipEventDestroy(r->ev);
    delete r;
  }
  std::vector<Req *> left(s->unloading.begin(), s->unloading.end());
  for (Lane &L : s->lane)
    for (Req *r : L.slot)
      if (r && std::find(left.begin(), left.end(), r) == left.end()) left.push_back(r);
  for (Req *r : left) {
    if (r->ev) (void)hipEventDestroy(r->ev);
    delete r;
  }
  for (Lane &L : s->lane) {
    if (L.ev) (void)hipEventDestroy(L.ev);
    if (L.b) gmunu_batch_destroy(L.b);  // also the lane's stream
  }
  (void)hipStreamDestroy(s->xs);
  const int rc = hipFree(s->arena) == hipSuccess ? GMUNU_OK : GMUNU_EHIP;
  delete s;
  return rc;
}

}  // extern "C"
