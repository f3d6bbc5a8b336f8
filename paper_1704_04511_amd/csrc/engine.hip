// Lock-step execution of many reconstructions (batch and continuous serving).
//
// Every active problem advances by one outer IRLS iteration per engine step.
// Problems whose Gram matrices have the same size s share one launch sequence
// of the eigen-decomposition chain (tridiagonalisation, divide and conquer,
// back-transformation), each kernel covering all of them at once; the kernels
// treat every problem independently with the same arithmetic as for a single
// problem, so a result is bit-identical alone, in a batch and in the server.
// The Gram matrix, weights, masks and CG of each problem run on the problem's
// own stream, ordered against the shared eigen-decomposition by events.
// Problems may join between steps (each keeps its own iteration index and
// epsilon schedule), which is what the server does.  Problems that use the
// library eigensolver take the single-problem path.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <vector>

#include "engine.h"
#include "kernels.h"
#include "plan.h"
#include "tune.h"

using namespace slrx;


#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(SLRX_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                  __LINE__);                                                                 \
  } while (0)

#define STCHK(expr)               \
  do {                            \
    slrx_status _s = (expr);      \
    if (_s != SLRX_OK) return _s; \
  } while (0)

slrx::EigGroup::~EigGroup() {
  if (mem) (void)hipFree(mem);
  if (tree) (void)hipFree(tree);
}

slrx::CgTable::~CgTable() {
  if (dev) (void)hipFree(dev);
  if (pinned) (void)hipHostFree(pinned);
  if (copied) (void)hipEventDestroy(copied);
}

slrx::BatchEig::~BatchEig() {
  if (stream) (void)hipStreamSynchronize(stream);
  if (cg_stream) (void)hipStreamSynchronize(cg_stream);
  groups.clear();
  cg_tables.clear();
  if (ev) (void)hipEventDestroy(ev);
  if (ev_free) (void)hipEventDestroy(ev_free);
  if (ev_cg) (void)hipEventDestroy(ev_cg);
  if (stream) (void)hipStreamDestroy(stream);
  if (cg_stream) (void)hipStreamDestroy(cg_stream);
}

static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// Layout of the buffers for nb problems of size n: every matrix-sized buffer
// per problem, the vectors for all of them.
struct GroupLayout {
  size_t sA, sQ, sWi, sWd, sB, sv, sd, total;
};
static GroupLayout group_layout(int n, int nb) {
  GroupLayout L;
  const size_t nn = (size_t)n * n;
  L.sA = al(nn * sizeof(double2));
  L.sQ = al(3 * nn * sizeof(double));
  L.sWi = al(dc_ws_ints(n) * sizeof(int));
  L.sWd = al(dc_ws_doubles(n) * sizeof(double));
  L.sB = al(bt_scratch_elems(n) * sizeof(double2));
  L.sv = al((size_t)nb * n * sizeof(double2));
  L.sd = al((size_t)nb * n * sizeof(double));
  L.total = (size_t)nb * (3 * L.sA + L.sQ + L.sWi + L.sWd + L.sB) + 5 * L.sv + 2 * L.sd;
  return L;
}
static size_t tree_bytes(int n) { return std::max<size_t>((size_t)4 * n, 4) * sizeof(int); }

size_t slrx::engine_problem_bytes(int n) { return group_layout(n, 1).total + tree_bytes(n); }

size_t slrx::BatchEig::allocated() const {
  size_t b = 0;
  for (const auto& kv : groups) {
    if (kv.second.mem) b += group_layout(kv.first, kv.second.cap).total;
    if (kv.second.tree) b += tree_bytes(kv.first);
  }
  for (const auto& kv : cg_tables) b += kv.second.cap * sizeof(CgSlice);
  return b;
}

slrx_status slrx::engine_trim(BatchEig& be, const std::map<int, int>& keep) {
  bool synced = false;
  for (auto it = be.groups.begin(); it != be.groups.end();) {
    const auto k = keep.find(it->first);
    const int want = k == keep.end() ? 0 : k->second;
    if (it->second.cap <= want) {
      ++it;
      continue;
    }
    if (!synced) {
      if (be.stream) HIPCHK(hipStreamSynchronize(be.stream));  // no reader of the buffers is left
      synced = true;
    }
    if (want == 0) {
      it = be.groups.erase(it);  // frees the buffers and the tree
      continue;
    }
    if (it->second.mem) HIPCHK(hipFree(it->second.mem));
    it->second.mem = nullptr;
    it->second.cap = 0;  // reserved again at the next step, for the problems present then
    ++it;
  }
  return SLRX_OK;
}

// Buffers for nb problems of size n (grown on demand; engine_trim shrinks them).
static slrx_status group_reserve(BatchEig& be, int n, int nb, EigGroup*& out) {
  if (!be.stream) {
    HIPCHK(hipStreamCreateWithFlags(&be.stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&be.ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&be.ev_free, hipEventDisableTiming));
  }
  EigGroup& G = be.groups[n];
  if (G.n != n) {  // first use of this size: the divide-and-conquer tree
    std::vector<int> nodes;
    dc_build_tree(n, nodes, G.level_start);
    G.node_sizes.resize(nodes.size() / 4);
    for (size_t q = 0; q < nodes.size() / 4; ++q) G.node_sizes[q] = nodes[4 * q + 1];
    if (!G.tree && dev_malloc((void**)&G.tree, tree_bytes(n)) != hipSuccess) {
      (void)hipGetLastError();
      G.tree = nullptr;
      return fail(SLRX_ENOMEM, "divide-and-conquer tree");
    }
    if (!nodes.empty())
      HIPCHK(hipMemcpy(G.tree, nodes.data(), nodes.size() * sizeof(int), hipMemcpyHostToDevice));
    G.n = n;  // only once the tree is on the device
  }
  if (nb > G.cap) {
    HIPCHK(hipStreamSynchronize(be.stream));  // every reader of the old buffers has finished
    if (G.mem) (void)hipFree(G.mem);
    G.mem = nullptr;
    G.cap = 0;
    const size_t nn = (size_t)n * n;
    const GroupLayout L = group_layout(n, nb);
    const size_t sA = L.sA, sQ = L.sQ, sWi = L.sWi, sWd = L.sWd, sB = L.sB, sv = L.sv, sd = L.sd;
    const size_t total = L.total;
    if (dev_malloc(&G.mem, total) != hipSuccess) {
      (void)hipGetLastError();
      G.mem = nullptr;
      return fail(SLRX_ENOMEM, "eigen-decomposition buffers (%zu bytes)", total);
    }
    char* p = (char*)G.mem;
    auto take = [&](size_t b) {
      char* q = p;
      p += b;
      return q;
    };
    EighBufs& e = G.bufs;
    e.n = n;
    e.A = (double2*)take(nb * sA);
    e.V = (double2*)take(nb * sA);
    e.Z = (double2*)take(nb * sA);
    e.Q = (double*)take(nb * sQ);
    e.Qs = e.Q + nn;
    e.U = e.Q + 2 * nn;
    e.wsi = (int*)take(nb * sWi);
    e.wsd = (double*)take(nb * sWd);
    e.bts = (double2*)take(nb * sB);
    e.tau = (double2*)take(sv);
    e.triv[0] = (double2*)take(sv);
    e.triv[1] = (double2*)take(sv);
    e.trip[0] = (double2*)take(sv);
    e.trip[1] = (double2*)take(sv);
    e.D = (double*)take(sd);
    e.E = (double*)take(sd);
    e.sA = (long)(sA / sizeof(double2));
    e.sZ = e.sA;
    e.sQ = (long)(sQ / sizeof(double));
    e.s_wsi = (long)(sWi / sizeof(int));
    e.s_wsd = (long)(sWd / sizeof(double));
    e.s_bts = (long)(sB / sizeof(double2));
    G.cap = nb;
  }
  G.bufs.tree = G.tree;
  G.bufs.level_start = &G.level_start;
  G.bufs.node_sizes = &G.node_sizes;
  out = &G;
  return SLRX_OK;
}

slrx_status slrx::engine_begin(slrx_plan* pl) {
  if (pl->direct() && pl->ncoils > 0) return fail(SLRX_EINVAL, "SLRX_FLAG_DIRECT is single-channel only");
  STCHK(prepare(pl));
  if (pl->direct()) STCHK(direct_setup(pl));
  pl->ktime = false;
  for (int c = 0; c < SLRX_K_NCLASS; ++c) pl->kused[c] = 0;
  HIPCHK(hipMemsetAsync(pl->info, 0, kInfoEntries * sizeof(rocblas_int), pl->stream));
  HIPCHK(hipEventRecord(pl->ev_run[0], pl->stream));
  pl->it_next = 0;
  pl->running = true;
  pl->ran = false;
  pl->run_irls = pl->prm.n_irls;
  pl->run_timing = false;
  return SLRX_OK;
}

slrx_status slrx::engine_end(slrx_plan* pl) {
  HIPCHK(hipEventRecord(pl->ev_run[1], pl->stream));
  return SLRX_OK;
}

// CG strategy of the engine steps: -1 tuned online, 0 every problem on its own
// stream, 1 grouped launches (slrx_set_cg_grouping).
static std::atomic<int> g_cg_grouping{-1};

extern "C" void slrx_set_cg_grouping(int32_t mode) { g_cg_grouping.store(mode < 0 ? -1 : (mode > 0 ? 1 : 0)); }

// Plans whose CG joins a grouped launch (single-channel, FFT-based operator).
static bool cg_groupable(const slrx_plan* pl) { return pl->ncoils == 0 && !pl->direct(); }

// One outer iteration of one problem on its own stream (the path of a plan run
// alone); with `deferred` the CG of a groupable plan is left to the grouped launch
// (its weights-done event recorded).
static slrx_status step_single(slrx_plan* pl, std::vector<slrx_plan*>* deferred = nullptr) {
  const int it = pl->it_next;
  if (pl->direct()) {
    STCHK(step_direct_gram(pl));
    STCHK(step_eigh(pl, it));
    STCHK(step_direct_weights(pl, it, it == 0, pl->prm.gamma));
    STCHK(run_cg_direct(pl, pl->prm.n_cg, it));
    pl->it_next = it + 1;
    return SLRX_OK;
  }
  if (pl->voxel()) {
    STCHK(step_voxel(pl, it, it == 0, pl->prm.gamma));
  } else {
    STCHK(step_gram(pl));
    STCHK(step_eigh(pl, it));
    STCHK(step_weights(pl, it, it == 0, pl->prm.gamma));
  }
  if (deferred && cg_groupable(pl)) {  // deferred: the step runs its CG in grouped launches
    HIPCHK(hipEventRecord(pl->ev_step, pl->stream));
    deferred->push_back(pl);
    return SLRX_OK;
  }
  STCHK(run_cg(pl, pl->prm.n_cg, it, false));
  pl->it_next = it + 1;
  return SLRX_OK;
}

// The table entry of a plan (its buffers and its own grids).
static CgSlice cg_slice_of(const slrx_plan* pl) {
  const slrx_dims& d = pl->d;
  CgSlice c{};
  c.P = d.P; c.Q = d.Q; c.T = d.T;
  c.circ = (pl->prm.flags & SLRX_FLAG_GIRAF) ? 1 : 0;
  c.pen_scale = (float)(pl->prm.lambda / ((double)d.P * d.Q));
  c.x = pl->x; c.r = pl->r; c.p = pl->p; c.q = pl->q; c.t = pl->t;
  c.bm = pl->bm;
  c.S = pl->S;
  c.Et = pl->Et;
  c.twQ = pl->twQf;
  c.twP = pl->twPf;
  c.partA = pl->partA; c.partB = pl->partB; c.rr_hist = pl->rr_hist;
  c.flag = pl->flag;
  cg_slice_grids(c);
  return c;
}

// The CG of one outer iteration for every plan of `g` (same M and n_cg) in grouped
// launches on the engine's CG stream, after each plan's weights (ev_step) and
// before its next work (the plans' streams wait for the CG).
static slrx_status run_cg_group(BatchEig& be, const std::vector<slrx_plan*>& g, int M, int n_cg) {
  if (!be.cg_stream) {
    HIPCHK(hipStreamCreateWithFlags(&be.cg_stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&be.ev_cg, hipEventDisableTiming));
  }
  CgTable& tb = be.cg_tables[std::make_pair(M, n_cg)];
  std::vector<CgSlice> host(g.size());
  int rows = 0, cols = 0, upd = 0;
  size_t pen_lds = 0;
  auto up8 = [](int n) { return (n + 7) & ~7; };
  for (size_t i = 0; i < g.size(); ++i) {
    CgSlice& c = host[i];
    c = cg_slice_of(g[i]);
    c.rows0 = rows;
    c.cols0 = cols;
    c.upd0 = upd;
    rows += up8(c.rows_gx * c.rows_gy);
    cols += up8(c.cols_gx);
    upd += up8(c.upd_gx);
    pen_lds = std::max(pen_lds, group_pen_lds(c.P, c.Q, c.T));
  }
  for (slrx_plan* pl : g) HIPCHK(hipStreamWaitEvent(be.cg_stream, pl->ev_step, 0));
  const bool same = tb.host.size() == host.size() &&
                    std::memcmp(tb.host.data(), host.data(), host.size() * sizeof(CgSlice)) == 0;
  if (!same) {  // upload the new table (stream-ordered after the launches that read the old one)
    if (host.size() > tb.cap) {
      HIPCHK(hipStreamSynchronize(be.cg_stream));
      if (tb.dev) HIPCHK(hipFree(tb.dev));
      if (tb.pinned) HIPCHK(hipHostFree(tb.pinned));
      tb.dev = nullptr;
      tb.pinned = nullptr;
      tb.cap = 0;
      tb.pending = false;
      const size_t cap = std::max<size_t>(host.size(), 32);
      if (dev_malloc((void**)&tb.dev, cap * sizeof(CgSlice)) != hipSuccess) {
        (void)hipGetLastError();
        tb.dev = nullptr;
        return fail(SLRX_ENOMEM, "grouped CG table (%zu entries)", cap);
      }
      HIPCHK(hipHostMalloc((void**)&tb.pinned, cap * sizeof(CgSlice), hipHostMallocDefault));
      if (!tb.copied) HIPCHK(hipEventCreateWithFlags(&tb.copied, hipEventDisableTiming));
      tb.cap = cap;
    }
    if (tb.pending) HIPCHK(hipEventSynchronize(tb.copied));  // the staging copy is free again
    std::memcpy(tb.pinned, host.data(), host.size() * sizeof(CgSlice));
    HIPCHK(hipMemcpyAsync(tb.dev, tb.pinned, host.size() * sizeof(CgSlice), hipMemcpyHostToDevice, be.cg_stream));
    HIPCHK(hipEventRecord(tb.copied, be.cg_stream));
    tb.pending = true;
    tb.host = host;
  }
  CgGroup G{};
  G.tab = tb.dev;
  G.ns = (int)host.size();
  G.M = M;
  G.rows_blocks = rows;
  G.cols_blocks = cols;
  G.upd_blocks = upd;
  G.pen_lds = pen_lds;
  hipStream_t s = be.cg_stream;
  // initial residual r = bm - A x, then n_cg iterations
  HIPCHK(launch_group_rows(G, ROW_PLAIN, 0, s));
  HIPCHK(launch_group_pen(G, s));
  HIPCHK(launch_group_fin(G, 1, s));
  for (int k = 0; k < n_cg; ++k) {
    HIPCHK(launch_group_rows(G, ROW_PUPDATE, k, s));
    HIPCHK(launch_group_pen(G, s));
    HIPCHK(launch_group_fin(G, 0, s));
    HIPCHK(launch_group_update(G, k, s));
  }
  HIPCHK(hipEventRecord(be.ev_cg, s));
  for (size_t i = 0; i < g.size(); ++i) {
    slrx_plan* pl = g[i];
    const int it = pl->it_next;
    HIPCHK(hipStreamWaitEvent(pl->stream, be.ev_cg, 0));
    HIPCHK(launch_store_sum(n_cg == 0 ? pl->partA : pl->partB, n_cg == 0 ? host[i].nfin : host[i].nupd,
                            pl->stats + 2 * SLRX_MAX_IRLS + it, pl->stream));
    pl->it_next = it + 1;
  }
  return SLRX_OK;
}

slrx_status slrx::engine_step(const std::vector<slrx_plan*>& plans, BatchEig& be) {
  roctxRangePushA("slrx engine step");  // host side: the enqueueing of one lock-step outer iteration
  struct PopRange {
    ~PopRange() { roctxRangePop(); }
  } pop;
  std::map<int, std::vector<slrx_plan*>> groups;
  std::vector<slrx_plan*> live;
  for (slrx_plan* pl : plans)
    if (pl->it_next < pl->prm.n_irls) live.push_back(pl);
  for (slrx_plan* pl : live)
    if (!(pl->lib_eigh() || pl->voxel() || pl->direct())) groups[pl->s()].push_back(pl);
  // The CG strategy of this step: each problem's CG on its own stream, or one
  // grouped launch per pass (bit-identical results).  Chosen per step shape by the
  // online tuner on whole-step times, once the tridiagonalisation's launch shape
  // for the step's groups is settled (so that one tuning does not time the other).
  int ng = 0, maxm = 0, maxcg = 0;
  long vsum = 0;
  for (slrx_plan* pl : live)
    if (cg_groupable(pl)) {
      ++ng;
      vsum += (long)pl->vol();
      maxm = std::max(maxm, pl->d.M);
      maxcg = std::max(maxcg, std::min(pl->prm.n_cg, 65535));
    }
  bool grouped = false;
  TuneTicket tk;
  const int forced = g_cg_grouping.load();
  if (forced >= 0) {
    grouped = forced == 1 && ng >= 1;
  } else if (ng >= 2) {
    bool settled = true;
    for (auto& kv : groups) {
      const int nb = (int)kv.second.size();
      const int c = tune_choice(TUNE_TRI, kv.first, nb, 0);
      settled = settled && c >= 0 && tune_choice(TUNE_TRI_ACCESS, kv.first, nb, c) >= 0;
    }
    if (settled) {
      if (!be.cg_stream) {
        HIPCHK(hipStreamCreateWithFlags(&be.cg_stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&be.ev_cg, hipEventDisableTiming));
      }
      for (slrx_plan* pl : live) {
        HIPCHK(hipEventRecord(pl->ev_begin, pl->stream));
        HIPCHK(hipStreamWaitEvent(be.cg_stream, pl->ev_begin, 0));
      }
      const int b = (int)std::min<long>(vsum >> 12, 1 << 30);
      grouped = tune_begin(TUNE_CG_GROUP, ng, b, (maxm << 16) | maxcg, 2, be.cg_stream, tk) == 1;
    }
  }
  std::vector<slrx_plan*> deferred;  // CG left to the grouped launches
  std::vector<slrx_plan*>* defer = grouped ? &deferred : nullptr;
  for (slrx_plan* pl : live)
    if (pl->lib_eigh() || pl->voxel() || pl->direct()) STCHK(step_single(pl, defer));
  bool used = false;
  for (auto& kv : groups) {
    const int n = kv.first;
    std::vector<slrx_plan*>& g = kv.second;
    const int nb = (int)g.size();
    EigGroup* G = nullptr;
    STCHK(group_reserve(be, n, nb, G));
    EighBufs e = G->bufs;
    e.nb = nb;
    // Gram matrices (row-major) into the group buffer once the previous step's readers are done
    for (int i = 0; i < nb; ++i) {
      slrx_plan* pl = g[i];
      if (be.have_free) HIPCHK(hipStreamWaitEvent(pl->stream, be.ev_free, 0));
      STCHK(step_gram(pl, false, e.A + (size_t)i * e.sA));
      HIPCHK(hipEventRecord(pl->ev_step, pl->stream));
      HIPCHK(hipStreamWaitEvent(be.stream, pl->ev_step, 0));
    }
    HIPCHK(eigh_tri(e, be.stream));
    HIPCHK(eigh_tdeig(e, be.stream));
    HIPCHK(eigh_backtr(e, be.stream));
    HIPCHK(hipEventRecord(be.ev, be.stream));
    for (int i = 0; i < nb; ++i) {
      slrx_plan* pl = g[i];
      const int it = pl->it_next;
      HIPCHK(hipStreamWaitEvent(pl->stream, be.ev, 0));
      STCHK(step_weights(pl, it, it == 0, pl->prm.gamma, e.Z + (size_t)i * e.sZ, e.D + (size_t)i * n));
      HIPCHK(hipEventRecord(pl->ev_step, pl->stream));
      HIPCHK(hipStreamWaitEvent(be.stream, pl->ev_step, 0));
      if (grouped && cg_groupable(pl)) {
        deferred.push_back(pl);
      } else {
        STCHK(run_cg(pl, pl->prm.n_cg, it, false));
        pl->it_next = it + 1;
      }
    }
    used = true;
  }
  if (used) {
    HIPCHK(hipEventRecord(be.ev_free, be.stream));
    be.have_free = true;
  }
  // the CG of every deferred plan: one grouped launch per pass for each (M, n_cg)
  std::map<std::pair<int, int>, std::vector<slrx_plan*>> cg;
  for (slrx_plan* pl : deferred) cg[std::make_pair(pl->d.M, pl->prm.n_cg)].push_back(pl);
  for (auto& kv : cg) STCHK(run_cg_group(be, kv.second, kv.first.first, kv.first.second));
  if (tk.e1) {  // a timed step ends when every problem's CG has run
    for (slrx_plan* pl : live) {
      HIPCHK(hipEventRecord(pl->ev_step, pl->stream));
      HIPCHK(hipStreamWaitEvent(be.cg_stream, pl->ev_step, 0));
    }
    tune_end(tk, be.cg_stream);
  }
  return SLRX_OK;
}
