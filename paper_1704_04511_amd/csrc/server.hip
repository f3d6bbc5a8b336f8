// Continuous-batching reconstruction server.
//
// Requests wait in a FIFO queue and are admitted, first fit, as soon as a slot
// is free and their device footprint fits the remaining HBM budget.  Each
// admitted request runs its whole IRLS loop on its own stream in a slot worker
// thread, so the device interleaves the kernels of all admitted requests;
// requests that arrive while others run join at the next free slot.  A
// request's IRLS state stays resident on the device while it runs; when a
// server-owned request finishes, its images are copied to host memory and its
// device state and budget share are released at once, so finished results never
// block admission.  Every request computes on its own buffers with fixed-order
// reductions, so a result does not depend on what runs beside it.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

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
  size_t bytes = 0;
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

struct slrx_server {
  size_t budget = 0;
  int max_slots = 1;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  size_t used = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::vector<std::thread> workers;
};

static void release_budget(slrx_server* s, Req* r) {
  if (r->holds_budget) {
    s->used -= r->bytes;
    r->holds_budget = false;
  }
}

// Pick the first queued request that fits the remaining budget (caller holds mu).
static Req* take_admissible(slrx_server* s) {
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    Req* r = *it;
    if (s->used + r->bytes <= s->budget) {
      s->queue.erase(it);
      return r;
    }
  }
  return nullptr;
}

static void run_request(slrx_server* s, Req* r) {
  slrx_status st = SLRX_OK;
  if (r->owned) {
    st = slrx_plan_create(&r->dims, &r->prm, nullptr, &r->plan);
    if (st == SLRX_OK) st = slrx_set_kspace(r->plan, r->b.data(), SLRX_MEM_HOST);
    if (st == SLRX_OK) st = slrx_set_mask(r->plan, r->S.data(), SLRX_MEM_HOST);
    std::vector<float2>().swap(r->b);
    std::vector<uint8_t>().swap(r->S);
  }
  if (st == SLRX_OK) st = slrx_run(r->plan);
  if (st == SLRX_OK) st = slrx_sync(r->plan);
  if (st == SLRX_OK && r->owned) {
    r->result.resize((size_t)r->dims.T * r->dims.P * r->dims.Q);
    st = slrx_get_images(r->plan, r->result.data(), SLRX_MEM_HOST);
  }
  std::string err = st != SLRX_OK ? std::string(slrx_last_error()) : std::string();
  if (r->owned && r->plan) {
    slrx_plan_destroy(r->plan);
    r->plan = nullptr;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = st;
  r->err = err;
  r->t_done = now_s();
  r->state = 2;
  release_budget(s, r);
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

static void worker_main(slrx_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    Req* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || (r = take_admissible(s)) != nullptr; });
      if (!r) return;  // stopping
      s->used += r->bytes;
      r->holds_budget = true;
      r->state = 1;
      r->t_admit = now_s();
    }
    run_request(s, r);
  }
}

extern "C" slrx_status slrx_server_create(size_t budget_bytes, int32_t max_slots, void* hip_stream,
                                          slrx_server** out) {
  (void)hip_stream;  // every slot runs on a stream of its own
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
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker_main, s);
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
      r->status = SLRX_ESTATE;
      r->err = "server destroyed before admission";
    }
    s->queue.clear();
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
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
  if (!plan->has_b || !plan->has_S) return fail(SLRX_ESTATE, "plan has no k-space or mask");
  Req* r = new Req();
  r->plan = plan;
  r->owned = false;
  r->bytes = slrx_footprint(&plan->cap);
  return enqueue(s, r, ticket);
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
  r->b.assign((const float2*)b, (const float2*)b + V);
  r->S.assign(S, S + V);
  r->bytes = slrx_footprint(dims);
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

extern "C" slrx_status slrx_wait(slrx_server* s, uint64_t ticket) {
  if (!s) return fail(SLRX_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(SLRX_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  s->cv_done.wait(lk, [&] { return r->state == 2; });
  if (r->status != SLRX_OK) return fail(r->status, "%s", r->err.c_str());
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
  if (used) *used = s->used;
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
