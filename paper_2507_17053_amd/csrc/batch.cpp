// Batched applies across operators (the serving layer's launches): a batch plan groups its
// operators by kernel instantiation (discretisation, dimension, degree) and runs every group as
// one launch per stage (kernels_apply.hip: batch_group_build / launch_batch_group).  The
// plan's tables live in one device allocation uploaded at creation; with graph != 0 the first
// run captures the whole batch (truncated-extension face launches, then the group launches)
// into a HIP graph that later runs replay.
#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

#include "sbm_internal.h"

using namespace sbm;

struct sbm_batch_s {
  int prec = SBM_F64;
  int device = 0;
  std::vector<sbm_ctx *> hs;         // operators with DoFs, in the caller's order
  std::vector<const void *> u;
  std::vector<void *> v;
  std::vector<int> taylor;           // indices (into hs) whose surrogate faces launch one by one
  std::vector<BatchGroup> groups;
  std::vector<double> work;          // per group: DoFs (the balance estimate)
  void *d_tables = nullptr;
  bool use_graph = false, graph_off = false;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;         // completion of the last run
  // groups spread over the batch's own streams (forked from and joined to the run's stream)
  std::vector<hipStream_t> streams;
  std::vector<std::vector<int>> lanes;  // per stream: its groups
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
};

namespace {

// Tables of one-shot batches (sbm_apply_batch), released once their run has completed, and the
// prepared batches alive: sbm_destroy waits for the runs of both (a batch records one event per
// run instead of one per handle, which would cost a host call per operator).
std::mutex g_deferred_mu;
struct Deferred {
  int device;
  hipEvent_t done;
  void *mem;
};
std::vector<Deferred> g_deferred;
std::set<sbm_batch> g_live;

void reap_deferred() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_deferred_mu);
  for (size_t i = 0; i < g_deferred.size();) {
    Deferred &d = g_deferred[i];
    if (d.device == dev && hipEventQuery(d.done) == hipSuccess) {
      dev_free(d.mem);
      (void)hipEventDestroy(d.done);
      d = g_deferred.back();
      g_deferred.pop_back();
    } else {
      ++i;
    }
  }
}

void release(sbm_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->d_tables) dev_free(b->d_tables);
  if (b->done) (void)hipEventDestroy(b->done);
  delete b;
}

sbm_status build(int n, const sbm_handle *hs, const void *const *u, void *const *v, int prec, int graph,
                 int max_streams, sbm_batch *out) {
  if (n < 0 || !out || (n > 0 && (!hs || !u || !v)) || (prec != SBM_F64 && prec != SBM_F32)) {
    set_error("sbm_batch_create: invalid argument");
    return SBM_EINVAL;
  }
  *out = nullptr;
  std::set<const sbm_ctx *> seen;
  std::set<const void *> outs;
  for (int i = 0; i < n; ++i) {
    const sbm_ctx *c = hs[i];
    if (!c || c->host_only) {
      set_error("sbm_batch_create: NULL or host-only handle");
      return SBM_EINVAL;
    }
    if (!seen.insert(c).second) {
      set_error("sbm_batch_create: a handle appears more than once");
      return SBM_EINVAL;
    }
    if (c->n_dofs == 0) continue;
    if (!u[i] || !v[i] || u[i] == v[i]) {
      set_error("sbm_batch_create: NULL or aliased vectors");
      return SBM_EINVAL;
    }
    if (!outs.insert(v[i]).second) {
      set_error("sbm_batch_create: two outputs share a vector");
      return SBM_EINVAL;
    }
  }
  for (int i = 0; i < n; ++i)
    if (hs[i]->n_dofs > 0 && outs.count(u[i])) {
      set_error("sbm_batch_create: an input is another apply's output");
      return SBM_EINVAL;
    }
  sbm_batch b = new sbm_batch_s;
  b->prec = prec;
  b->use_graph = graph != 0;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    set_error("sbm_batch_create: no device");
    return SBM_EHIP;
  }
  // groups by (discretisation, dimension, degree), in order of first appearance
  std::map<std::tuple<int, int, int>, int> gid;
  std::vector<std::vector<int>> members;
  for (int i = 0; i < n; ++i) {
    sbm_ctx *c = hs[i];
    if (c->n_dofs == 0) continue;
    const int k = (int)b->hs.size();
    b->hs.push_back(c);
    b->u.push_back(u[i]);
    b->v.push_back(v[i]);
    if (c->taylor_m >= 0) b->taylor.push_back(k);
    auto key = std::make_tuple(c->disc, c->dim, c->p);
    auto it = gid.find(key);
    if (it == gid.end()) {
      it = gid.emplace(key, (int)members.size()).first;
      members.emplace_back();
    }
    members[it->second].push_back(k);
  }
  std::vector<unsigned char> image;
  for (const auto &m : members) {
    BatchGroup g;
    g.prec = prec;
    std::vector<const sbm_ctx *> cs;
    std::vector<const void *> us;
    std::vector<void *> vs;
    std::vector<int> own;
    for (int k : m) {
      cs.push_back(b->hs[k]);
      us.push_back(b->u[k]);
      vs.push_back(b->v[k]);
      own.push_back(b->hs[k]->taylor_m < 0 ? 1 : 0);
    }
    if (batch_group_build(g, cs, us, vs, own, image) != hipSuccess) {
      delete b;
      set_error("sbm_batch_create: batch too large");
      return SBM_EINVAL;
    }
    b->groups.push_back(g);
    double w = 0.0;
    for (const sbm_ctx *c : cs) w += (double)c->n_dofs;
    b->work.push_back(w);
  }
  if (!image.empty()) {
    hipError_t e = dev_alloc(&b->d_tables, image.size());
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_tables, image.data(), image.size(), hipMemcpyHostToDevice, lib_stream());
    if (e == hipSuccess) e = hipStreamSynchronize(lib_stream());
    if (e != hipSuccess) {
      release(b);
      set_error(std::string("sbm_batch_create: upload: ") + hipGetErrorString(e));
      return SBM_EHIP;
    }
  }
  if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
    b->done = nullptr;
    release(b);
    set_error("sbm_batch_create: event");
    return SBM_EHIP;
  }
  // the groups' launch chains are independent: with more than one group, spread them over up
  // to max_streams streams of the batch (largest first, each to the least loaded stream)
  const int k = std::min<int>(std::max(1, max_streams), (int)b->groups.size());
  if (k > 1) {
    std::vector<int> order(b->groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->work[x] > b->work[y]; });
    std::vector<double> load(k, 0.0);
    b->lanes.assign(k, {});
    for (int gi : order) {
      const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      b->lanes[j].push_back(gi);
      load[j] += b->work[gi];
    }
    bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    if (!ok) b->fork = nullptr;
    for (int j = 0; ok && j < k; ++j) {
      hipStream_t st = nullptr;
      hipEvent_t e = nullptr;
      ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
      if (ok) b->streams.push_back(st);
      ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
      if (ok) b->join.push_back(e);
    }
    if (!ok) {
      release(b);
      set_error("sbm_batch_create: streams");
      return SBM_EHIP;
    }
  }
  *out = b;
  return SBM_OK;
}

// One group's launches: its truncated-extension faces, then its stages.
hipError_t enqueue_group(sbm_batch b, int gi, hipStream_t s) {
  const BatchGroup &g = b->groups[gi];
  for (int k : b->taylor) {
    const sbm_ctx *c = b->hs[k];
    if (c->disc != g.first->disc || c->dim != g.first->dim || c->p != g.first->p) continue;
    hipError_t e = launch_taylor_faces(c, b->u[k], c->d_fbuf, b->prec, s);
    if (e != hipSuccess) return e;
  }
  return launch_batch_group(g, b->d_tables, s);
}

// Every launch of the batch: on s, or forked over the batch's streams and joined back to s.
hipError_t enqueue(sbm_batch b, hipStream_t s) {
  if (b->streams.empty()) {
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      hipError_t e = enqueue_group(b, (int)gi, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t e = hipEventRecord(b->fork, s);
  if (e != hipSuccess) return e;
  // every stream that took the fork is joined back, also after a failed launch, so that the
  // run's completion event on s covers all of the batch's work
  for (size_t j = 0; j < b->streams.size(); ++j) {
    hipError_t ej = hipStreamWaitEvent(b->streams[j], b->fork, 0);
    if (ej != hipSuccess) {
      if (e == hipSuccess) e = ej;
      continue;
    }
    for (size_t q = 0; e == hipSuccess && q < b->lanes[j].size(); ++q) e = enqueue_group(b, b->lanes[j][q], b->streams[j]);
    ej = hipEventRecord(b->join[j], b->streams[j]);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(s, b->join[j], 0);
    if (ej != hipSuccess && e == hipSuccess) e = ej;
  }
  return e;
}

sbm_status run(sbm_batch b, hipStream_t s) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device) {
    set_error("sbm_batch_run: the batch was created on another device");
    return SBM_EINVAL;
  }
  if (b->hs.empty()) return SBM_OK;
  if (b->use_graph && !b->graph_off && !b->exec) {
    hipGraph_t g = nullptr;
    bool ok = s != nullptr && hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      const hipError_t e = enqueue(b, s);
      ok = hipStreamEndCapture(s, &g) == hipSuccess && e == hipSuccess && g;
      if (ok) ok = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
    }
    if (!ok) {
      (void)hipGetLastError();
      b->exec = nullptr;
      b->graph_off = true;  // launches are issued directly from now on
    }
  }
  const hipError_t e = b->exec ? hipGraphLaunch(b->exec, s) : enqueue(b, s);
  // recorded also after a failed launch: destroy then waits for whatever was enqueued
  const hipError_t er = hipEventRecord(b->done, s);
  SBM_HIP_CHECK(e);
  SBM_HIP_CHECK(er);
  return SBM_OK;
}

}  // namespace

namespace sbm {
void wait_batches() {
  std::lock_guard<std::mutex> lk(g_deferred_mu);
  for (const Deferred &d : g_deferred) (void)hipEventSynchronize(d.done);
  for (sbm_batch b : g_live)
    if (b->done) (void)hipEventSynchronize(b->done);
}
}  // namespace sbm

extern "C" {

sbm_status sbm_batch_create(int n, const sbm_handle *hs, const void *const *u, void *const *v, int prec, int graph,
                            int max_streams, sbm_batch *out) {
  reap_deferred();
  const sbm_status st = build(n, hs, u, v, prec, graph, max_streams, out);
  if (st == SBM_OK) {
    std::lock_guard<std::mutex> lk(g_deferred_mu);
    g_live.insert(*out);
  }
  return st;
}

sbm_status sbm_batch_run(sbm_batch b, void *stream) {
  if (!b) {
    set_error("sbm_batch_run: NULL batch");
    return SBM_EINVAL;
  }
  return run(b, (hipStream_t)stream);
}

sbm_status sbm_batch_destroy(sbm_batch b) {
  if (!b) return SBM_OK;
  {
    std::lock_guard<std::mutex> lk(g_deferred_mu);
    g_live.erase(b);
  }
  const hipError_t e = b->done ? hipEventSynchronize(b->done) : hipSuccess;
  release(b);
  if (e != hipSuccess) {
    set_error(std::string("sbm_batch_destroy: ") + hipGetErrorString(e));
    return SBM_EHIP;
  }
  return SBM_OK;
}

sbm_status sbm_apply_batch(int n, const sbm_handle *hs, const void *const *u, void *const *v, int prec,
                           void *stream) {
  if (n == 0) return SBM_OK;
  reap_deferred();
  sbm_batch b = nullptr;
  sbm_status st = build(n, hs, u, v, prec, 0, 1, &b);
  if (st != SBM_OK) return st;
  st = run(b, (hipStream_t)stream);
  if (st != SBM_OK) {
    (void)hipStreamSynchronize((hipStream_t)stream);  // launches already issued may read the tables
    release(b);
    return st;
  }
  if (!b->d_tables) {
    release(b);
    return st;
  }
  // the tables are released by a later batch call once this run has completed
  {
    std::lock_guard<std::mutex> lk(g_deferred_mu);
    g_deferred.push_back(Deferred{b->device, b->done, b->d_tables});
  }
  b->done = nullptr;
  b->d_tables = nullptr;
  release(b);
  return SBM_OK;
}

}  // extern "C"
