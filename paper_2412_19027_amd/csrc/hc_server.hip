// Served form: continuous batching of many independent problems on one GPU.
//
// Requests are validated and analysed on the submitting thread (hc_setup),
// queued first-in first-out, and admitted into active slots while their
// device workspace fits the HBM budget; the workspace is carved from one
// device pool allocated at creation, and the pinned read-back staging is one
// block per slot allocated when a worker starts, so admission and retirement
// never allocate or free memory.  Worker threads each own a stream (default priority)
// and a share of the slots; every tick advances each of a worker's active
// problems by one pass of the loop body of Algorithm 1, so short and long
// solves interleave and a finished problem frees its slot and memory for the
// next request at the following tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hc_steps.h"
#include "hc_wave.h"
#include "hipcone.h"

namespace {

// pinned read-back block per slot: enough for the reduction partials and
// step masks of problems with a few dozen cone segments; a problem that
// needs more allocates its own at bind
constexpr size_t kStageBytes = (size_t)1 << 20;

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Job {
  uint64_t ticket = 0, tag = 0;
  hc_solver* h = nullptr;
  size_t bytes = 0, offset = 0;
  int stage = -1;                  // the worker's pinned read-back block it uses
  int64_t n = 0, m = 0;
  double t_submit = 0, t_start = 0, t_end = 0;
  int32_t status = HC_STATUS_UNSOLVED;
  int32_t error = HC_OK;
  hc_info info{};
  std::vector<double> x, s, z;
  bool finished = false;
  // batched engine
  std::unique_ptr<hc::WavePlan> plan;
  int slot = -1;
  int32_t first_iterations = 0;    // iterations of a mixed-precision attempt run again in FP64
};

// first-fit allocator over [0, size) with coalescing, 256-byte granules
struct Pool {
  size_t size = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
  void init(size_t bytes) {
    size = bytes;
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  static size_t round(size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; }
  bool take(size_t bytes, size_t* off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t o = it->first + bytes;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = round(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct hc_server {
  hc_server_config cfg{};
  char* pool_base = nullptr;
  bool own_pool = false;            // allocated here (else the caller's hc_server_config.pool)
  Pool pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<std::shared_ptr<Job>> pending;
  std::deque<std::shared_ptr<Job>> pending_wave;            // for the batched engine
  std::deque<std::shared_ptr<Job>> to_plan;                 // set up, waiting for a planner thread
  std::condition_variable cv_plan;
  std::vector<std::thread> planners;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;   // submitted, not yet collected
  std::vector<std::thread> workers;
  std::thread wave_thread;
  int64_t ticks = 0;
  // statistics
  size_t in_use = 0, peak = 0;
  int64_t submitted = 0, completed = 0, rejected = 0, cancelled = 0, iterations = 0, active = 0;
  std::vector<double> latencies;
  double t_first = -1, t_last = 0, busy_ms = 0;

  void worker(int w, int cap);
  void wave_worker(int cap);
  void planner();
  void finish(const std::shared_ptr<Job>& j, int32_t rc, hipStream_t st);
  void retire(const std::shared_ptr<Job>& j);   // bookkeeping of a finished job (lock held)
};

void hc_server::retire(const std::shared_ptr<Job>& j) {
  j->t_end = now_ms();
  j->finished = true;
  pool.give(j->offset, j->bytes);
  in_use -= Pool::round(j->bytes);
  active--;
  completed++;
  iterations += j->info.iterations;
  latencies.push_back(j->t_end - j->t_submit);
  t_last = j->t_end;
  cv_done.notify_all();
  cv_work.notify_all();
}

void hc_server::finish(const std::shared_ptr<Job>& j, int32_t rc, hipStream_t st) {
  (void)st;
  if (j->h) {
    if (rc == HC_OK) rc = hc::solver_finish(j->h);
    hc_get_info(j->h, &j->info);
    if (rc == HC_OK) {
      j->x.resize(j->n);
      j->s.resize(j->m);
      j->z.resize(j->m);
      rc = hc_get_solution(j->h, j->x.data(), j->s.data(), j->z.data(), 0);
    }
    hc_destroy(j->h);
    j->h = nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  j->error = rc;
  j->status = rc == HC_OK ? j->info.status : HC_STATUS_NUMERICAL_ERROR;
  retire(j);
}

// Planner threads: the batched engine's plan of a set-up problem (ordering,
// band layout, gather plan) is made off the submitting thread; a problem the
// engine does not take goes to the per-slot workers.
void hc_server::planner() {
  for (;;) {
    std::shared_ptr<Job> j;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_plan.wait(lk, [&] { return stop || !to_plan.empty(); });
      if (stop) return;
      j = to_plan.front();
      to_plan.pop_front();
    }
    std::unique_ptr<hc::WavePlan> plan(new hc::WavePlan());
    std::string why;
    bool take = hc::wave_plan(j->h, plan.get(), &why);
    size_t wb = take ? plan->blob_bytes() : 0;
    if (take && Pool::round(wb) > pool.size) take = false;
    if (take) {
      hc_destroy(j->h);
      j->h = nullptr;
      j->plan = std::move(plan);
      j->bytes = wb;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (j->plan) pending_wave.push_back(j);
    else pending.push_back(j);
    cv_work.notify_all();
  }
}

// The batched engine: every tick is one graph launch (interior-point
// iterations of all slots in one kernel, then the slots' phase words copied to
// pinned host memory); between ticks finished problems are read out and
// retired and queued ones admitted into free slots and pool memory.  A tick
// lasts about one iteration of its largest problem; the smaller ones run as
// many iterations as fit in that time (the budget is 0.9 of the last tick's
// length), so a small problem does not wait a whole tick per iteration.
void hc_server::wave_worker(int cap) {
  using namespace hc;
  (void)hipSetDevice(cfg.device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
  WaveDesc* hdesc = nullptr;
  int32_t *hact = nullptr, *hstat = nullptr;
  int64_t* hbudget = nullptr;
  void* dtab = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipHostMalloc((void**)&hdesc, (size_t)cap * sizeof(WaveDesc), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&hact, (size_t)cap * sizeof(int32_t), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&hstat, (size_t)cap * sizeof(int32_t), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&hbudget, sizeof(int64_t), hipHostMallocDefault) == hipSuccess &&
            hipMalloc(&dtab, (size_t)cap * (sizeof(WaveDesc) + 2 * sizeof(int32_t)) + 64) == hipSuccess;
  WaveDesc* ddesc = (WaveDesc*)dtab;
  int32_t* dact = ok ? (int32_t*)((char*)dtab + (size_t)cap * sizeof(WaveDesc)) : nullptr;
  int32_t* dstat = ok ? dact + cap : nullptr;
  int64_t* dbudget = ok ? (int64_t*)(((uintptr_t)(dstat + cap) + 15) / 16 * 16) : nullptr;
  if (ok) {
    std::memset(hact, 0, (size_t)cap * sizeof(int32_t));
    *hbudget = 0;
    ok = hipMemcpyAsync(dact, hact, (size_t)cap * sizeof(int32_t), hipMemcpyHostToDevice, st) == hipSuccess &&
         hipMemcpyAsync(dbudget, hbudget, sizeof(int64_t), hipMemcpyHostToDevice, st) == hipSuccess &&
         hipStreamSynchronize(st) == hipSuccess;
  }
  if (ok) {   // the tick, captured once
    ok = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      wave_tick(ddesc, dact, cap, dstat, dbudget, st);
      (void)hipMemcpyAsync(hstat, dstat, (size_t)cap * sizeof(int32_t), hipMemcpyDeviceToHost, st);
      ok = hipStreamEndCapture(st, &graph) == hipSuccess &&
           hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    }
  }
  std::vector<std::shared_ptr<Job>> slot(cap);
  std::vector<int> free_slots;
  for (int i = cap - 1; i >= 0; --i) free_slots.push_back(i);
  int nact = 0;
  for (;;) {
    std::vector<std::shared_ptr<Job>> fresh;
    {
      std::unique_lock<std::mutex> lk(mu);
      auto admissible = [&]() {
        if (pending_wave.empty() || free_slots.empty()) return false;
        size_t off = 0;
        if (!pool.take(pending_wave.front()->bytes, &off)) return false;
        pool.give(off, pending_wave.front()->bytes);
        return true;
      };
      while (!stop && nact == 0 && !admissible()) cv_work.wait(lk);
      if (stop) break;
      while (!free_slots.empty() && !pending_wave.empty()) {
        auto j = pending_wave.front();
        size_t off = 0;
        if (!pool.take(j->bytes, &off)) break;   // first in, first out: wait for memory
        pending_wave.pop_front();
        j->offset = off;
        j->slot = free_slots.back();
        free_slots.pop_back();
        in_use += Pool::round(j->bytes);
        peak = std::max(peak, in_use);
        active++;
        fresh.push_back(j);
      }
    }
    if (!ok) {   // no engine on this device: fail what was admitted
      for (auto& j : fresh) {
        std::lock_guard<std::mutex> lk(mu);
        j->error = HC_ERR_DEVICE;
        j->status = HC_STATUS_NUMERICAL_ERROR;
        free_slots.push_back(j->slot);
        retire(j);
      }
      continue;
    }
    for (auto& j : fresh) {
      j->t_start = now_ms();
      wave_upload(*j->plan, pool_base + j->offset, &hdesc[j->slot], st);
      hact[j->slot] = 1;
      slot[j->slot] = j;
      ++nact;
    }
    if (!fresh.empty()) {
      (void)hipMemcpyAsync(ddesc, hdesc, (size_t)cap * sizeof(WaveDesc), hipMemcpyHostToDevice, st);
      (void)hipMemcpyAsync(dact, hact, (size_t)cap * sizeof(int32_t), hipMemcpyHostToDevice, st);
    }
    if (nact == 0) continue;
    const double t0 = now_ms();
    const bool launched = hipGraphLaunch(exec, st) == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
    const double tick_ms = now_ms() - t0;
    bool changed = false, restarted = false;
    for (int i = 0; i < cap; ++i) {
      if (!hact[i]) continue;
      auto& j = slot[i];
      if (launched && hstat[i] != PH_DONE) continue;
      hc_info inf{};
      j->x.resize(j->n);
      j->s.resize(j->m);
      j->z.resize(j->m);
      if (launched) wave_result(hdesc[i], *j->plan, &inf, j->x.data(), j->s.data(), j->z.data(), st);
      // a mixed-precision solve that broke down runs again in FP64, in the same
      // slot and pool block (the FP64 layout is the mixed one without its FP32
      // buffers), with the regularisation of the mixed mode's FP64 fallback
      // factorisation; its iterations and one fallback are added to the report
      if (launched && j->plan->mixed &&
          (inf.status == HC_STATUS_NUMERICAL_ERROR || inf.status == HC_STATUS_INSUFFICIENT_PROGRESS)) {
        j->plan->mixed = false;
        j->plan->st.static_reg = 1e-8;
        j->plan->st.dyn_reg = std::ldexp(1.0, -104);
        j->plan->st.ir_mu_frac = 0.0;
        j->first_iterations = inf.iterations;
        wave_upload(*j->plan, pool_base + j->offset, &hdesc[i], st);
        restarted = true;
        continue;
      }
      inf.iterations += j->first_iterations;
      if (j->first_iterations) inf.fp64_fallbacks += 1;
      hact[i] = 0;
      changed = true;
      --nact;
      std::lock_guard<std::mutex> lk(mu);
      j->info = inf;
      j->error = launched ? HC_OK : HC_ERR_DEVICE;
      j->status = launched ? inf.status : HC_STATUS_NUMERICAL_ERROR;
      j->plan.reset();
      free_slots.push_back(i);
      retire(j);
      slot[i].reset();
    }
    if (changed) (void)hipMemcpyAsync(dact, hact, (size_t)cap * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (restarted) (void)hipMemcpyAsync(ddesc, hdesc, (size_t)cap * sizeof(WaveDesc), hipMemcpyHostToDevice, st);
    // next tick's budget: 0.9 of this tick's length (10 ns clock ticks)
    *hbudget = (int64_t)(0.9 * tick_ms * 1e5);
    (void)hipMemcpyAsync(dbudget, hbudget, sizeof(int64_t), hipMemcpyHostToDevice, st);
    std::lock_guard<std::mutex> lk(mu);
    busy_ms += now_ms() - t0;
    ticks++;
  }
  // shutting down: cancel the active problems
  (void)hipStreamSynchronize(st);
  for (int i = 0; i < cap; ++i) {
    if (!hact || !hact[i] || !slot[i]) continue;
    std::lock_guard<std::mutex> lk(mu);
    auto& j = slot[i];
    j->status = HC_STATUS_CANCELLED;
    j->finished = true;
    j->t_end = now_ms();
    pool.give(j->offset, j->bytes);
    in_use -= Pool::round(j->bytes);
    active--;
    cancelled++;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (dtab) (void)hipFree(dtab);
  if (hdesc) (void)hipHostFree(hdesc);
  if (hact) (void)hipHostFree(hact);
  if (hstat) (void)hipHostFree(hstat);
  if (hbudget) (void)hipHostFree(hbudget);
  (void)hipStreamDestroy(st);
}

void hc_server::worker(int w, int cap) {
  (void)w;
  (void)hipSetDevice(cfg.device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
  // one pinned read-back block per slot, allocated once: binding a problem
  // then allocates no pinned memory, and retiring it frees none (hipHostFree
  // would synchronise the whole device, stalling the other workers' streams)
  std::vector<void*> stage(cap, nullptr);
  std::vector<int> stage_free;
  for (int i = cap - 1; i >= 0; --i)
    if (hipHostMalloc(&stage[i], kStageBytes, hipHostMallocDefault) == hipSuccess) stage_free.push_back(i);
  std::vector<std::shared_ptr<Job>> mine, fresh;
  for (;;) {
    fresh.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      auto admissible = [&]() {
        if (pending.empty() || (int)mine.size() >= cap) return false;
        size_t off = 0;
        if (!pool.take(pending.front()->bytes, &off)) return false;
        pool.give(off, pending.front()->bytes);
        return true;
      };
      while (!stop && mine.empty() && !admissible()) cv_work.wait(lk);
      if (stop) break;
      while ((int)mine.size() < cap && !pending.empty()) {
        auto j = pending.front();
        size_t off = 0;
        if (!pool.take(j->bytes, &off)) break;   // first in, first out: wait for memory
        pending.pop_front();
        j->offset = off;
        in_use += Pool::round(j->bytes);
        peak = std::max(peak, in_use);
        active++;
        mine.push_back(j);
        fresh.push_back(j);
      }
    }
    for (auto& j : fresh) {
      hc_device dev{pool_base + j->offset, Pool::round(j->bytes), st, cfg.device, nullptr, 0};
      if (!stage_free.empty()) {
        j->stage = stage_free.back();
        stage_free.pop_back();
        dev.host_stage = stage[j->stage];
        dev.host_stage_bytes = kStageBytes;
      }
      j->t_start = now_ms();
      int32_t rc = hc_bind(j->h, &dev);
      if (rc == HC_OK) rc = hc::solver_begin(j->h);
      if (rc != HC_OK) {
        if (j->stage >= 0) stage_free.push_back(j->stage);
        finish(j, rc, st);
        mine.erase(std::find(mine.begin(), mine.end(), j));
      }
    }
    // one tick: every active problem advances by one iteration
    const double t0 = now_ms();
    for (size_t i = 0; i < mine.size();) {
      int done = 0;
      const int32_t rc = hc::solver_step(mine[i]->h, &done);
      if (rc != HC_OK || done) {
        if (mine[i]->stage >= 0) stage_free.push_back(mine[i]->stage);
        finish(mine[i], rc, st);
        mine.erase(mine.begin() + (long)i);
      } else {
        ++i;
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      busy_ms += now_ms() - t0;
    }
  }
  // shutting down: cancel what this worker still holds
  for (auto& j : mine) {
    (void)hipStreamSynchronize(st);
    hc_destroy(j->h);
    j->h = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    j->status = HC_STATUS_CANCELLED;
    j->finished = true;
    j->t_end = now_ms();
    pool.give(j->offset, j->bytes);
    in_use -= Pool::round(j->bytes);
    active--;
    cancelled++;
  }
  (void)hipStreamSynchronize(st);
  for (void* b : stage)
    if (b) (void)hipHostFree(b);
  (void)hipStreamDestroy(st);
}

namespace {

void fill_result(const Job& j, hc_result* out) {
  out->tag = j.tag;
  out->status = j.status;
  out->error = j.error;
  out->iterations = j.info.iterations;
  out->obj_primal = j.info.obj_primal;
  out->obj_dual = j.info.obj_dual;
  out->res_primal = j.info.res_primal;
  out->res_dual = j.info.res_dual;
  out->queue_ms = j.t_start > 0 ? j.t_start - j.t_submit : j.t_end - j.t_submit;
  out->solve_ms = j.t_start > 0 ? j.t_end - j.t_start : 0.0;
  out->latency_ms = j.t_end - j.t_submit;
  out->n = j.n;
  out->m = j.m;
  if (out->x && !j.x.empty()) std::memcpy(out->x, j.x.data(), j.x.size() * sizeof(double));
  if (out->s && !j.s.empty()) std::memcpy(out->s, j.s.data(), j.s.size() * sizeof(double));
  if (out->z && !j.z.empty()) std::memcpy(out->z, j.z.data(), j.z.size() * sizeof(double));
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double r = p * (double)(v.size() - 1);
  const size_t i = (size_t)r;
  const double f = r - (double)i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

int32_t hc_server_config_default(hc_server_config* c) {
  if (!c) return HC_ERR_INVALID_ARG;
  std::memset(c, 0, sizeof(*c));
  c->hbm_budget_bytes = (size_t)64 << 30;
  c->max_slots = 64;
  c->workers = 4;
  c->device = 0;
  c->batched = 1;
  c->batch_slots = 1024;
  return hc_settings_default(&c->settings);
}

int32_t hc_server_create(hc_server** out, const hc_server_config* cfg) {
  if (!out || !cfg) return HC_ERR_INVALID_ARG;
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->workers < 1 || cfg->workers > 16 || cfg->hbm_budget_bytes < 4096 ||
      (cfg->batched && (cfg->batch_slots < 1 || cfg->batch_slots > 65536)))
    return HC_ERR_INVALID_ARG;
  std::unique_ptr<hc_server> s(new hc_server());
  s->cfg = *cfg;
  if (hipSetDevice(cfg->device) != hipSuccess) return HC_ERR_DEVICE;
  void* p = cfg->pool;
  if (p) {
    if ((uintptr_t)p % 256 != 0) return HC_ERR_INVALID_ARG;
  } else {
    if (hipMalloc(&p, cfg->hbm_budget_bytes) != hipSuccess) return HC_ERR_OOM;
    s->own_pool = true;
  }
  s->pool_base = (char*)p;
  s->pool.init(cfg->hbm_budget_bytes / 256 * 256);
  const int nw = std::min(cfg->workers, cfg->max_slots);
  for (int w = 0; w < nw; ++w) {
    const int cap = cfg->max_slots / nw + (w < cfg->max_slots % nw ? 1 : 0);
    s->workers.emplace_back(&hc_server::worker, s.get(), w, cap);
  }
  if (cfg->batched) {
    s->wave_thread = std::thread(&hc_server::wave_worker, s.get(), cfg->batch_slots);
    // planning takes 1-3 ms per MPC request on the host: two planners per worker
    for (int i = 0; i < 2 * std::max(2, cfg->workers); ++i) s->planners.emplace_back(&hc_server::planner, s.get());
  }
  *out = s.release();
  return HC_OK;
}

int32_t hc_server_submit(hc_server* s, const hc_problem* p, uint64_t tag, uint64_t* ticket) {
  if (!s || !p || !ticket) return HC_ERR_INVALID_ARG;
  const double t = now_ms();
  hc_solver* h = nullptr;
  int32_t rc = hc_setup(&h, p, &s->cfg.settings);
  size_t bytes = 0;
  if (rc == HC_OK) rc = hc_workspace_bytes(h, &bytes);
  if (rc == HC_OK && Pool::round(bytes) > s->pool.size) rc = HC_ERR_TOO_LARGE;
  if (rc != HC_OK) {
    hc_destroy(h);
    std::lock_guard<std::mutex> lk(s->mu);
    s->rejected++;
    return rc;
  }
  auto j = std::make_shared<Job>();
  j->tag = tag;
  j->h = h;
  j->bytes = bytes;
  j->n = p->n;
  j->m = p->m;
  j->t_submit = t;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    if (h) hc_destroy(h);
    return HC_ERR_STATE;
  }
  j->ticket = s->next_ticket++;
  *ticket = j->ticket;
  s->jobs[j->ticket] = j;
  if (s->cfg.batched) {
    s->to_plan.push_back(j);   // a planner thread decides where it runs
    s->cv_plan.notify_one();
  } else {
    s->pending.push_back(j);
  }
  s->submitted++;
  if (s->t_first < 0) s->t_first = t;
  s->cv_work.notify_all();
  return HC_OK;
}

int32_t hc_server_poll(hc_server* s, uint64_t ticket, hc_result* out) {
  if (!s || !out) return HC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return HC_ERR_INVALID_ARG;
  if (!it->second->finished) return HC_PENDING;
  fill_result(*it->second, out);
  s->jobs.erase(it);
  return HC_OK;
}

int32_t hc_server_wait(hc_server* s, uint64_t ticket, hc_result* out) {
  if (!s || !out) return HC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return HC_ERR_INVALID_ARG;
  std::shared_ptr<Job> j = it->second;
  s->cv_done.wait(lk, [&] { return j->finished || s->stop; });
  if (!j->finished) return HC_ERR_STATE;
  fill_result(*j, out);
  s->jobs.erase(ticket);
  return HC_OK;
}

int32_t hc_server_stats(hc_server* s, hc_server_report* out) {
  if (!s || !out) return HC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->rejected = s->rejected;
  out->cancelled = s->cancelled;
  out->active = s->active;
  out->pending = (int64_t)(s->pending.size() + s->pending_wave.size() + s->to_plan.size());
  out->iterations = s->iterations;
  out->hbm_in_use = s->in_use;
  out->hbm_peak = s->peak;
  out->p50_latency_ms = percentile(s->latencies, 0.50);
  out->p99_latency_ms = percentile(s->latencies, 0.99);
  double sum = 0;
  for (double v : s->latencies) sum += v;
  out->mean_latency_ms = s->latencies.empty() ? 0.0 : sum / (double)s->latencies.size();
  const double span = s->t_last - s->t_first;
  out->solves_per_s = (s->completed > 0 && span > 0) ? 1e3 * (double)s->completed / span : 0.0;
  out->busy_ms = s->busy_ms;
  return HC_OK;
}

void hc_server_destroy(hc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    s->cv_plan.notify_all();
  }
  for (auto& t : s->planners) t.join();
  for (auto& t : s->workers) t.join();
  if (s->wave_thread.joinable()) s->wave_thread.join();
  for (auto& j : s->pending) {
    hc_destroy(j->h);
    j->h = nullptr;
  }
  for (auto& j : s->pending_wave) {
    j->status = HC_STATUS_CANCELLED;
    j->finished = true;
  }
  for (auto& j : s->to_plan) {
    hc_destroy(j->h);
    j->h = nullptr;
    j->status = HC_STATUS_CANCELLED;
    j->finished = true;
  }
  if (s->own_pool) (void)hipFree(s->pool_base);
  delete s;
}

}  // extern "C"
