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
#include <map>
#include <vector>

#include "engine.h"
#include "kernels.h"
#include "plan.h"

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

slrx::BatchEig::~BatchEig() {
  if (stream) (void)hipStreamSynchronize(stream);
  groups.clear();
  if (ev) (void)hipEventDestroy(ev);
  if (ev_free) (void)hipEventDestroy(ev_free);
  if (stream) (void)hipStreamDestroy(stream);
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

// One outer iteration of one problem on its own stream (the path of a plan run alone).
static slrx_status step_single(slrx_plan* pl) {
  const int it = pl->it_next;
  if (pl->voxel()) {
    STCHK(step_voxel(pl, it, it == 0, pl->prm.gamma));
  } else if (pl->direct()) {
    STCHK(step_direct_gram(pl));
    STCHK(step_eigh(pl, it));
    STCHK(step_direct_weights(pl, it, it == 0, pl->prm.gamma));
    STCHK(run_cg_direct(pl, pl->prm.n_cg, it));
    pl->it_next = it + 1;
    return SLRX_OK;
  } else {
    STCHK(step_gram(pl));
    STCHK(step_eigh(pl, it));
    STCHK(step_weights(pl, it, it == 0, pl->prm.gamma));
  }
  STCHK(run_cg(pl, pl->prm.n_cg, it, false));
  pl->it_next = it + 1;
  return SLRX_OK;
}

slrx_status slrx::engine_step(const std::vector<slrx_plan*>& plans, BatchEig& be) {
  roctxRangePushA("slrx engine step");  // host side: the enqueueing of one lock-step outer iteration
  struct PopRange {
    ~PopRange() { roctxRangePop(); }
  } pop;
  std::map<int, std::vector<slrx_plan*>> groups;
  for (slrx_plan* pl : plans) {
    if (pl->it_next >= pl->prm.n_irls) continue;
    if (pl->lib_eigh() || pl->voxel() || pl->direct()) STCHK(step_single(pl));
    else groups[pl->s()].push_back(pl);
  }
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
      STCHK(run_cg(pl, pl->prm.n_cg, it, false));
      pl->it_next = it + 1;
    }
    used = true;
  }
  if (used) {
    HIPCHK(hipEventRecord(be.ev_free, be.stream));
    be.have_free = true;
  }
  return SLRX_OK;
}
