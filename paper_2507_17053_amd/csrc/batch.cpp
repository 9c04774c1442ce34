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
  void *d_tables = nullptr;
  bool use_graph = false, graph_off = false;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;         // completion of the last run
};

namespace {

// Tables of one-shot batches (sbm_apply_batch), released once their run has completed.
std::mutex g_deferred_mu;
struct Deferred {
  int device;
  hipEvent_t done;
  void *mem;
};
std::vector<Deferred> g_deferred;

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
  if (b->d_tables) dev_free(b->d_tables);
  if (b->done) (void)hipEventDestroy(b->done);
  delete b;
}

sbm_status build(int n, const sbm_handle *hs, const void *const *u, void *const *v, int prec, int graph,
                 sbm_batch *out) {
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
  *out = b;
  return SBM_OK;
}

// Every launch of the batch, in order: the truncated-extension faces, then each group's stages.
hipError_t enqueue(sbm_batch b, hipStream_t s) {
  for (int k : b->taylor) {
    const sbm_ctx *c = b->hs[k];
    hipError_t e = launch_taylor_faces(c, b->u[k], c->d_fbuf, b->prec, s);
    if (e != hipSuccess) return e;
  }
  for (const BatchGroup &g : b->groups) {
    hipError_t e = launch_batch_group(g, b->d_tables, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
  if (b->exec) {
    SBM_HIP_CHECK(hipGraphLaunch(b->exec, s));
  } else {
    SBM_HIP_CHECK(enqueue(b, s));
  }
  SBM_HIP_CHECK(hipEventRecord(b->done, s));
  for (sbm_ctx *c : b->hs) note_work(c, s);
  return SBM_OK;
}

}  // namespace

extern "C" {

sbm_status sbm_batch_create(int n, const sbm_handle *hs, const void *const *u, void *const *v, int prec, int graph,
                            sbm_batch *out) {
  reap_deferred();
  return build(n, hs, u, v, prec, graph, out);
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
  sbm_status st = build(n, hs, u, v, prec, 0, &b);
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
