// Online autotuner of launch configurations.
//
// For a kernel class and shape (a key), the first calls try each candidate
// configuration in turn on the real work, timed by an event pair on the
// caller's stream; the times are read back later without blocking (an event
// pair is collected once its end event has completed).  When every candidate
// has kTuneSamples times, the fastest (by its best time) is kept for the key
// for the rest of the process and appended to the file named by the
// SLRX_TUNE_CACHE environment variable, if set, which later processes read
// back instead of tuning again.  Only choices that leave results unchanged bit
// for bit are tuned this way (how rows are split among workgroups, cache
// policies, how launches are grouped), so the calls made while tuning are
// ordinary calls.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "tune.h"
#include "../../include/slrx.h"

namespace slrx {
namespace {

constexpr int kTuneSamples = 2;

typedef std::tuple<int, int, int, int, int> Key;  // device, kind, a, b, c

struct Pending {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int cand = 0;
  bool ended = false;
};

struct Entry {
  int ncand = 0;
  int chosen = -1;
  std::vector<float> best;
  std::vector<int> samples;   // completed
  std::vector<int> inflight;  // recorded, not yet read
  std::vector<Pending> pending;
};

std::mutex g_mu;
std::map<Key, Entry> g_entries;
std::vector<hipEvent_t> g_pool;
bool g_loaded = false;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void load_cache() {
  g_loaded = true;
  const char* path = std::getenv("SLRX_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int dev, kind, a, b, c, ncand, chosen;
  while (std::fscanf(f, "%d %d %d %d %d %d %d", &dev, &kind, &a, &b, &c, &ncand, &chosen) == 7) {
    if (chosen < 0 || chosen >= ncand) continue;
    Entry& en = g_entries[Key(dev, kind, a, b, c)];
    en.ncand = ncand;
    en.chosen = chosen;
  }
  std::fclose(f);
}

void save_choice(const Key& k, const Entry& en) {
  const char* path = std::getenv("SLRX_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
               std::get<4>(k), en.ncand, en.chosen);
  std::fclose(f);
}

// Read back every completed event pair of an entry (caller holds g_mu).
void collect(Entry& en) {
  for (size_t i = 0; i < en.pending.size();) {
    Pending& p = en.pending[i];
    if (p.ended && hipEventQuery(p.e1) == hipSuccess) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
        if (ms < en.best[p.cand]) en.best[p.cand] = ms;
        ++en.samples[p.cand];
      }
      --en.inflight[p.cand];
      g_pool.push_back(p.e0);
      g_pool.push_back(p.e1);
      en.pending.erase(en.pending.begin() + (long)i);
    } else {
      ++i;
    }
  }
}

}  // namespace

int tune_begin(int kind, int a, int b, int c, int ncand, hipStream_t s, TuneTicket& t) {
  t = TuneTicket{};
  if (ncand <= 1) return 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_loaded) load_cache();
  const Key key(dev, kind, a, b, c);
  Entry& en = g_entries[key];
  if (en.ncand != ncand) {  // new key (or a cached entry for another candidate list)
    en = Entry{};
    en.ncand = ncand;
  }
  if (en.chosen >= 0) return en.chosen;
  if (en.best.empty()) {
    en.best.assign(ncand, 3.4e38f);
    en.samples.assign(ncand, 0);
    en.inflight.assign(ncand, 0);
  }
  collect(en);
  int cand = -1, least = kTuneSamples;
  for (int i = 0; i < ncand; ++i) {
    const int n = en.samples[i] + en.inflight[i];
    if (n < least) {
      least = n;
      cand = i;
    }
  }
  if (cand < 0) {  // every candidate timed (or in flight)
    bool done = true;
    for (int i = 0; i < ncand; ++i) done = done && en.samples[i] >= kTuneSamples;
    if (!done) return 0;  // results still in flight: the first candidate meanwhile
    int bi = 0;
    for (int i = 1; i < ncand; ++i)
      if (en.best[i] < en.best[bi]) bi = i;
    en.chosen = bi;
    save_choice(key, en);
    return bi;
  }
  Pending p;
  p.e0 = take_event();
  p.e1 = take_event();
  p.cand = cand;
  if (!p.e0 || !p.e1 || hipEventRecord(p.e0, s) != hipSuccess) {
    if (p.e0) g_pool.push_back(p.e0);
    if (p.e1) g_pool.push_back(p.e1);
    return cand;  // untimed call; the candidate is tried again later
  }
  ++en.inflight[cand];
  en.pending.push_back(p);
  t.key_kind = kind;
  t.a = a;
  t.b = b;
  t.c = c;
  t.dev = dev;
  t.slot = (int)en.pending.size() - 1;
  t.e1 = p.e1;
  return cand;
}

void tune_end(const TuneTicket& t, hipStream_t s) {
  if (!t.e1) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_entries.find(Key(t.dev, t.key_kind, t.a, t.b, t.c));
  if (it == g_entries.end()) return;
  for (Pending& p : it->second.pending)
    if (p.e1 == t.e1 && !p.ended) {
      if (hipEventRecord(p.e1, s) == hipSuccess) p.ended = true;
      break;
    }
}

int tune_choice(int kind, int a, int b, int c) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_entries.find(Key(dev, kind, a, b, c));
  return it == g_entries.end() ? -1 : it->second.chosen;
}

}  // namespace slrx

extern "C" int32_t slrx_tri_workgroup_budget(int32_t n, int32_t nbatch) {
  if (n < 1 || nbatch < 1) return 0;
  const int c = slrx::tune_choice(slrx::TUNE_TRI, n, nbatch, 0);
  return c < 0 ? 0 : slrx::tri_budget(nbatch, c);
}
