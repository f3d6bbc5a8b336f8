// Continuous-batching reconstruction server.
//
// Requests wait in a FIFO queue and are admitted, first fit, between engine
// steps: as soon as fewer than max_slots requests are active and a request's
// device footprint fits the remaining HBM budget.  A request's footprint is
// its plan's buffers plus its share of the engine's eigen-decomposition
// buffers; the budget covers every device byte the server holds (running
// plans, idle plans kept for reuse, and the engine buffers, which are trimmed
// back to the running requests' needs when an admission would not fit
// otherwise).  One scheduler thread drives
// the lock-step engine: each step advances every active request by one outer
// IRLS iteration, with one launch sequence of the eigen-decomposition per
// group of equal Gram size and all other kernels on each request's own stream.  A request
// that arrives while others run joins at the next step, with its own iteration
// count and epsilon schedule.  The scheduler keeps one step in flight ahead of
// the device, so admissions take effect within about one step.  When a request
// finishes, its images are copied to host memory and its budget share is
// released at once; its plan is kept idle for the next request of the same
// shape and evicted when the budget is needed.  A result depends only on the
// request, not on what runs beside it (bit-identical to running it alone).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "engine.h"
#include "plan.h"

using namespace slrx;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t id = 0;
  slrx_plan* plan = nullptr;
  bool owned = false;       // plan created by the server at admission
  size_t bytes = 0;         // plan footprint + engine share, charged while running
  size_t eig = 0;           // engine share (part of bytes)
  int s = 0;                // Gram size
  int state = 0;            // 0 queued, 1 running, 2 done
  bool holds_budget = false;
  slrx_status status = SLRX_OK;
  std::string err;
  double t_submit = 0, t_admit = 0, t_done = 0;
  slrx_dims dims{};
  slrx_params prm{};
  std::vector<float2> b;
  std::vector<uint8_t> S;
  std::vector<float2> result;  // images of a finished server-owned request
};

}  // namespace

typedef std::tuple<int, int, int, int, int, int> ShapeKey;
static ShapeKey key_of(const slrx_dims& d) { return ShapeKey(d.P, d.Q, d.T, d.N1, d.N2, d.M); }

struct slrx_server {
  size_t budget = 0;
  int max_slots = 1;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  size_t used = 0;          // footprint of admitted (running) requests
  size_t pooled = 0;        // footprint of idle plans kept for reuse
  size_t eig_alloc = 0;     // engine buffers allocated (scheduler's last report)
  size_t eig_need = 0;      // engine shares of the running requests
  std::map<int, int> running_by_s;  // running requests per Gram size
  double queue_timeout = 0; // seconds a request may wait for admission (0: no limit)
  int waiters = 0;          // threads inside slrx_wait / slrx_wait_for
  std::condition_variable cv_idle;
  std::unordered_set<slrx_plan*> busy;  // caller plans queued or running
  std::multimap<ShapeKey, std::pair<slrx_plan*, size_t>> pool;  // idle server-owned plans
  uint64_t next_id = 1;
  bool stop = false;
  std::thread scheduler;
  BatchEig eig;  // used by the scheduler thread only
};

static void release_budget(slrx_server* s, Req* r) {
  if (r->holds_budget) {
    s->used -= r->bytes;
    s->eig_need -= r->eig;
    if (--s->running_by_s[r->s] == 0) s->running_by_s.erase(r->s);
    r->holds_budget = false;
  }
}

// Engine bytes allocated beyond what the running requests are charged for.
static size_t eig_excess(const slrx_server* s) { return s->eig_alloc > s->eig_need ? s->eig_alloc - s->eig_need : 0; }

// Device bytes the server holds (caller holds mu).
static size_t held(const slrx_server* s) { return s->used + s->pooled + eig_excess(s); }

// Pick the first queued request that can run (caller holds mu; called by the
// scheduler thread, which owns the engine).  A server-owned request takes an
// idle plan of its shape from the pool if there is one (then only its engine
// share is new); otherwise its whole footprint must fit the budget next to
// what the server holds, evicting idle plans of other shapes and trimming the
// engine's buffers to the running requests' needs if that is what it takes.
// Evicted plans are returned through `evict` and destroyed by the caller
// outside the lock.
static Req* take_admissible(slrx_server* s, BatchEig& eig, std::vector<slrx_plan*>& evict) {
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    Req* r = *it;
    auto pit = s->pool.end();
    if (r->owned) pit = s->pool.find(key_of(r->dims));
    const size_t plan_new = pit != s->pool.end() ? 0 : r->bytes - r->eig;
    const size_t plan_reused = pit != s->pool.end() ? pit->second.second : 0;
    auto fits = [&]() { return held(s) + plan_new + r->eig <= s->budget; };
    if (s->used + r->bytes > s->budget) continue;  // cannot fit next to the running requests
    if (!fits() && eig_excess(s) > 0) {
      (void)engine_trim(eig, s->running_by_s);
      s->eig_alloc = eig.allocated();
    }
    while (!fits() && !s->pool.empty()) {
      auto victim = s->pool.begin();
      if (victim == pit) {
        if (++victim == s->pool.end()) break;
      }
      evict.push_back(victim->second.first);
      s->pooled -= victim->second.second;
      s->pool.erase(victim);
    }
    if (!fits()) continue;
    if (pit != s->pool.end()) {
      r->plan = pit->second.first;
      s->pooled -= plan_reused;
      s->pool.erase(pit);
    }
    s->queue.erase(it);
    return r;
  }
  return nullptr;
}

// Complete queued requests whose wait for admission exceeded the queue timeout
// (caller holds mu).
static void expire_queued(slrx_server* s) {
  if (!(s->queue_timeout > 0)) return;
  const double now = now_s();
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    Req* r = *it;
    if (now - r->t_submit > s->queue_timeout) {
      r->state = 2;
      r->status = SLRX_ETIMEDOUT;
      r->err = "request waited longer than the queue timeout";
      r->t_done = now;
      if (!r->owned) s->busy.erase(r->plan);
      it = s->queue.erase(it);
      s->cv_done.notify_all();
    } else {
      ++it;
    }
  }
}

// Bind a newly admitted request to its plan and start it on the engine.
static slrx_status start_request(Req* r) {
  slrx_status st = SLRX_OK;
  if (r->owned) {
    if (r->plan) {  // reused idle plan of the same shape
      st = slrx_set_params(r->plan, &r->prm);
      if (st == SLRX_OK) st = slrx_clear_init(r->plan);
    } else {
      st = slrx_plan_create(&r->dims, &r->prm, nullptr, &r->plan);
    }
    if (st == SLRX_OK) st = slrx_set_kspace(r->plan, r->b.data(), SLRX_MEM_HOST);
    if (st == SLRX_OK) st = slrx_set_mask(r->plan, r->S.data(), SLRX_MEM_HOST);
    std::vector<float2>().swap(r->b);
    std::vector<uint8_t>().swap(r->S);
  } else if (r->plan->running && hipEventQuery(r->plan->ev_run[1]) == hipErrorNotReady) {
    st = fail(SLRX_EBUSY, "plan is running");
  } else if (r->plan->running) {
    st = finish(r->plan);
  }
  if (st == SLRX_OK) st = engine_begin(r->plan);
  return st;
}

// Results of a request whose last step has run on the device.
static slrx_status collect_request(Req* r) {
  slrx_status st = finish(r->plan);
  if (st == SLRX_OK && r->owned) {
    r->result.resize((size_t)r->dims.T * r->dims.P * r->dims.Q);
    st = slrx_get_images(r->plan, r->result.data(), SLRX_MEM_HOST);
  }
  return st;
}

// Mark a request done, release its budget, keep its plan idle for reuse.
static void complete_request(slrx_server* s, Req* r, slrx_status st) {
  std::string err = st != SLRX_OK ? std::string(slrx_last_error(nullptr)) : std::string();
  if (r->owned && r->plan && st != SLRX_OK) {
    slrx_plan_destroy(r->plan);
    r->plan = nullptr;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = st;
  r->err = err;
  r->t_done = now_s();
  r->state = 2;
  release_budget(s, r);
  if (!r->owned) s->busy.erase(r->plan);
  if (r->owned && r->plan) {  // the plan alone: its engine share stays with the engine's buffers
    const size_t plan_bytes = r->bytes - r->eig;
    s->pool.emplace(key_of(r->dims), std::make_pair(r->plan, plan_bytes));
    s->pooled += plan_bytes;
    r->plan = nullptr;
  }
  s->cv_done.notify_all();
}

static void scheduler_main(slrx_server* s) {
  (void)hipSetDevice(s->device);
  std::vector<Req*> active;     // requests with steps left
  std::vector<Req*> finishing;  // last step enqueued, results not yet collected
  for (;;) {
    // 1. admission (blocks only when nothing is in flight)
    std::vector<Req*> admitted;
    std::vector<slrx_plan*> evict;
    bool stopping = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        expire_queued(s);
        s->eig_alloc = s->eig.allocated();
        while (!s->stop && (int)(active.size() + admitted.size()) < s->max_slots) {
          Req* r = take_admissible(s, s->eig, evict);
          if (!r) break;
          s->used += r->bytes;
          s->eig_need += r->eig;
          ++s->running_by_s[r->s];
          r->holds_budget = true;
          r->state = 1;
          r->t_admit = now_s();
          admitted.push_back(r);
        }
        stopping = s->stop;
        if (!admitted.empty() || !active.empty() || !finishing.empty() || stopping) break;
        if (s->queue_timeout > 0 && !s->queue.empty())
          s->cv_work.wait_for(lk, std::chrono::duration<double>(s->queue_timeout / 4));
        else
          s->cv_work.wait(lk);
      }
    }
    for (slrx_plan* p : evict) slrx_plan_destroy(p);
    if (stopping && active.empty() && finishing.empty() && admitted.empty()) return;
    for (Req* r : admitted) {
      const slrx_status st = start_request(r);
      if (st == SLRX_OK) active.push_back(r);
      else complete_request(s, r, st);
    }

    // 2. one engine step over every active request
    if (!active.empty()) {
      std::vector<slrx_plan*> plans;
      for (Req* r : active) plans.push_back(r->plan);
      slrx_status st = engine_step(plans, s->eig);
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->eig_alloc = s->eig.allocated();
      }
      for (Req* r : active) {
        slrx_plan* pl = r->plan;
        if (st == SLRX_OK && hipEventRecord(pl->ev_iter[(pl->it_next - 1) & 1], pl->stream) != hipSuccess)
          st = fail(SLRX_EDEVICE, "hipEventRecord failed");
      }
      if (st != SLRX_OK) {  // device-side state of the step is unknown: fail every active request
        for (Req* r : active) {
          (void)hipStreamSynchronize(r->plan->stream);
          r->plan->running = false;
          complete_request(s, r, st);
        }
        active.clear();
      }
      // pacing: wait for the previous step of each request (one step stays queued)
      for (Req* r : active) {
        slrx_plan* pl = r->plan;
        if (pl->it_next >= 2) (void)hipEventSynchronize(pl->ev_iter[(pl->it_next - 2) & 1]);
      }
      for (size_t i = 0; i < active.size();) {
        Req* r = active[i];
        if (r->plan->it_next >= r->plan->prm.n_irls) {
          const slrx_status se = engine_end(r->plan);
          if (se != SLRX_OK) complete_request(s, r, se);
          else finishing.push_back(r);
          active.erase(active.begin() + i);
        } else {
          ++i;
        }
      }
    }

    // 3. collect finished requests (wait for one only when nothing else is in flight)
    for (size_t i = 0; i < finishing.size();) {
      Req* r = finishing[i];
      const bool must_wait = active.empty() && i == 0;
      if (must_wait || hipEventQuery(r->plan->ev_run[1]) != hipErrorNotReady) {
        complete_request(s, r, collect_request(r));
        finishing.erase(finishing.begin() + i);
      } else {
        ++i;
      }
    }
  }
}

extern "C" slrx_status slrx_server_create(size_t budget_bytes, int32_t max_slots, void* hip_stream,
                                          slrx_server** out) {
  (void)hip_stream;  // every request runs on a stream of its own
  if (!out) return fail(SLRX_EINVAL, "out is NULL");
  *out = nullptr;
  if (budget_bytes == 0) return fail(SLRX_EINVAL, "budget must be > 0");
  if (max_slots < 1 || max_slots > 64) return fail(SLRX_EINVAL, "max_slots must be in [1,64]");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SLRX_EDEVICE, "no HIP device");
  slrx_server* s = new slrx_server();
  s->budget = budget_bytes;
  s->max_slots = max_slots;
  s->device = dev;
  s->scheduler = std::thread(scheduler_main, s);
  *out = s;
  return SLRX_OK;
}

extern "C" void slrx_server_destroy(slrx_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // queued requests are cancelled
    for (Req* r : s->queue) {
      r->state = 2;
      r->status = SLRX_ECANCELED;
      r->err = "server destroyed before admission";
      r->t_done = now_s();
    }
    s->queue.clear();
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
  if (s->scheduler.joinable()) s->scheduler.join();  // running requests complete
  {
    // threads still inside slrx_wait leave before the server goes away
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.notify_all();
    s->cv_idle.wait(lk, [&] { return s->waiters == 0; });
  }
  for (auto& kv : s->pool) slrx_plan_destroy(kv.second.first);
  for (auto& kv : s->reqs) {
    Req* r = kv.second;
    if (r->owned && r->plan) slrx_plan_destroy(r->plan);
    delete r;
  }
  delete s;
}

static slrx_status enqueue(slrx_server* s, Req* r, uint64_t* ticket) {
  if (r->bytes > s->budget) {
    const size_t need = r->bytes, have = s->budget;
    delete r;
    return fail(SLRX_ENOMEM, "request needs %zu bytes, server budget is %zu", need, have);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    delete r;
    return fail(SLRX_ESTATE, "server is stopping");
  }
  r->id = s->next_id++;
  r->t_submit = now_s();
  s->reqs[r->id] = r;
  s->queue.push_back(r);
  *ticket = r->id;
  s->cv_work.notify_one();
  return SLRX_OK;
}

extern "C" slrx_status slrx_submit(slrx_server* s, slrx_plan* plan, uint64_t* ticket) {
  if (!s || !plan || !ticket) return fail(SLRX_EINVAL, "NULL argument");
  if (!(plan->has_b || plan->ncoils > 0) || !plan->has_S) return fail(SLRX_ESTATE, "plan has no k-space or mask");
  if (plan->lib_eigh()) return fail(SLRX_EINVAL, "the library eigensolver is a test reference and is not served");
  if (plan->direct()) return fail(SLRX_EINVAL, "IRLS-direct is a comparison method and is not served");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->busy.count(plan)) return fail(SLRX_EBUSY, "plan is already queued or running on this server");
    s->busy.insert(plan);
  }
  Req* r = new Req();
  r->plan = plan;
  r->owned = false;
  r->s = plan->s();
  r->eig = plan->voxel() ? 0 : engine_problem_bytes(r->s);  // voxel plans need no shared eigensolver
  r->bytes = slrx_footprint(&plan->cap) + r->eig;
  const slrx_status st = enqueue(s, r, ticket);
  if (st != SLRX_OK) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->busy.erase(plan);
  }
  return st;
}

extern "C" slrx_status slrx_submit_data(slrx_server* s, const slrx_dims* dims, const slrx_params* params,
                                        const void* b, const uint8_t* S, uint64_t* ticket) {
  if (!s || !dims || !b || !S || !ticket) return fail(SLRX_EINVAL, "NULL argument");
  slrx_status st = slrx_validate(dims, params);
  if (st != SLRX_OK) return st;
  Req* r = new Req();
  r->owned = true;
  r->dims = *dims;
  if (params) r->prm = *params;
  else slrx_default_params(&r->prm);
  const size_t V = (size_t)dims->T * dims->P * dims->Q;
  if (r->prm.flags & SLRX_FLAG_LIBEIGH) {
    delete r;
    return fail(SLRX_EINVAL, "the library eigensolver is a test reference and is not served");
  }
  if (r->prm.flags & SLRX_FLAG_DIRECT) {
    delete r;
    return fail(SLRX_EINVAL, "IRLS-direct is a comparison method and is not served");
  }
  r->b.assign((const float2*)b, (const float2*)b + V);
  r->S.assign(S, S + V);
  r->s = dims->N1 * dims->N2 * dims->M;
  r->eig = (r->prm.flags & SLRX_FLAG_HLR_VOXEL) ? 0 : engine_problem_bytes(r->s);
  r->bytes = slrx_footprint(dims) + r->eig;
  return enqueue(s, r, ticket);
}

static Req* find(slrx_server* s, uint64_t ticket) {
  auto it = s->reqs.find(ticket);
  return it == s->reqs.end() ? nullptr : it->second;
}

extern "C" slrx_status slrx_poll(slrx_server* s, uint64_t ticket, int32_t* done) {
  if (!s || !done) return fail(SLRX_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(SLRX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  *done = r->state == 2;
  return SLRX_OK;
}

// Block until the request is done or `timeout_s` seconds have passed (< 0: no limit).
static slrx_status wait_request(slrx_server* s, uint64_t ticket, double timeout_s) {
  if (!s) return fail(SLRX_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(SLRX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  ++s->waiters;
  auto done = [&] { return r->state == 2 || s->stop; };
  bool ok = true;
  if (timeout_s < 0) s->cv_done.wait(lk, done);
  else ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
  const int state = r->state;
  const slrx_status rst = r->status;
  const std::string err = r->err;
  if (--s->waiters == 0) s->cv_idle.notify_all();
  if (!ok || state != 2) return fail(SLRX_ENOTREADY, "request %llu not finished", (unsigned long long)ticket);
  if (rst != SLRX_OK) return fail(rst, "%s", err.c_str());
  return SLRX_OK;
}

extern "C" slrx_status slrx_wait(slrx_server* s, uint64_t ticket) { return wait_request(s, ticket, -1.0); }

extern "C" slrx_status slrx_wait_for(slrx_server* s, uint64_t ticket, double timeout_s) {
  if (!(timeout_s >= 0.0)) return fail(SLRX_EINVAL, "timeout must be >= 0");
  return wait_request(s, ticket, timeout_s);
}

extern "C" slrx_status slrx_cancel(slrx_server* s, uint64_t ticket) {
  if (!s) return fail(SLRX_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(SLRX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (r->state == 2) return fail(SLRX_ESTATE, "request %llu already finished", (unsigned long long)ticket);
  if (r->state == 1) return fail(SLRX_EBUSY, "request %llu is running", (unsigned long long)ticket);
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
    if (*it == r) {
      s->queue.erase(it);
      break;
    }
  r->state = 2;
  r->status = SLRX_ECANCELED;
  r->err = "request canceled before admission";
  r->t_done = now_s();
  if (!r->owned) s->busy.erase(r->plan);
  s->cv_done.notify_all();
  return SLRX_OK;
}

extern "C" slrx_status slrx_server_set_queue_timeout(slrx_server* s, double seconds) {
  if (!s) return fail(SLRX_EINVAL, "NULL argument");
  if (!(seconds >= 0.0) || !std::isfinite(seconds)) return fail(SLRX_EINVAL, "timeout must be finite and >= 0");
  std::lock_guard<std::mutex> lk(s->mu);
  s->queue_timeout = seconds;
  s->cv_work.notify_all();
  return SLRX_OK;
}

extern "C" slrx_status slrx_get_request_info(slrx_server* s, uint64_t ticket, slrx_request_info* out) {
  if (!s || !out) return fail(SLRX_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(SLRX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  out->t_submit = r->t_submit;
  out->t_admit = r->t_admit;
  out->t_done = r->t_done;
  out->state = r->state;
  out->status = (int32_t)r->status;
  out->bytes = r->bytes;
  return SLRX_OK;
}

extern "C" slrx_status slrx_server_usage(slrx_server* s, size_t* used, int32_t* queued) {
  if (!s) return fail(SLRX_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (used) *used = held(s);
  if (queued) *queued = (int32_t)s->queue.size();
  return SLRX_OK;
}

// Copy a finished server-owned request's images to host memory.
extern "C" slrx_status slrx_fetch_images(slrx_server* s, uint64_t ticket, void* out_host) {
  if (!s || !out_host) return fail(SLRX_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(SLRX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (r->state != 2) return fail(SLRX_ENOTREADY, "request %llu not finished", (unsigned long long)ticket);
  if (r->status != SLRX_OK) return fail(r->status, "%s", r->err.c_str());
  if (!r->owned || r->result.empty()) return fail(SLRX_ESTATE, "request has no server-owned result");
  std::memcpy(out_host, r->result.data(), r->result.size() * sizeof(float2));
  return SLRX_OK;
}

// Forget a finished request (frees any state it still holds).
extern "C" slrx_status slrx_release(slrx_server* s, uint64_t ticket) {
  if (!s) return fail(SLRX_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(SLRX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (r->state != 2) return fail(SLRX_EBUSY, "request %llu not finished", (unsigned long long)ticket);
  if (r->owned && r->plan) slrx_plan_destroy(r->plan);
  release_budget(s, r);
  s->reqs.erase(ticket);
  delete r;
  s->cv_work.notify_all();
  return SLRX_OK;
}
