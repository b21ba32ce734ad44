// Batches of independent geometries: one plan per geometry, applied together.
//
// hfmm_apply_batch forks the caller's stream into a few internal streams (all
// at the default priority), runs the plans' pipelines on them largest first,
// and joins them back, so that small geometries fill the GPU alongside large
// ones. With graph mode on, the first call for a set of buffers is captured
// into a HIP graph (the workspaces are reserved before the capture; the
// pipeline contains no memsets or host synchronisation) and later calls with
// the same buffers replay it.
#include "plan_internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

namespace {

constexpr int kBatchStreams = 4;  // the hardware queues a process gets by default

}  // namespace

struct hfmm_batch_s {
  std::vector<hfmm_plan_t> plans;
  std::vector<int> order;  // plans by decreasing size
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  hipEvent_t done = nullptr;  // recorded on the caller's stream after every batch apply
  bool graph_on = false;
  hipGraphExec_t exec = nullptr;
  std::vector<const double*> gq;
  std::vector<double*> gu;
  std::vector<int64_t> ggen;  // the plans' workspace generations the graph was captured with
  int gnrhs = 0;
  hipStream_t gstream = nullptr;

  void release_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    gq.clear();
    gu.clear();
    ggen.clear();
    gnrhs = 0;
  }
  ~hfmm_batch_s() {
    // the last apply (eager or a graph replay) has ended before anything is freed
    if (done) (void)hipEventSynchronize(done);
    for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
    release_graph();
    if (done) (void)hipEventDestroy(done);
    for (hipEvent_t e : joins) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    for (hfmm_plan_t p : plans) hfmm_destroy(p);
  }
};

namespace {

hfmm_status_t batch_fail(hfmm_status_t st, const std::string& where, hipError_t e) {
  return hfmm::report(st, "batch " + where + ": " + hipGetErrorString(e));
}

// Enqueue every plan's apply on the internal streams between a fork and a
// join on s.
hfmm_status_t enqueue(hfmm_batch_t b, const double* const* q, double* const* u, int nrhs, hipStream_t s) {
  hipError_t e = hipEventRecord(b->fork, s);
  if (e != hipSuccess) return batch_fail(HFMM_ERR_DEVICE, "fork", e);
  for (hipStream_t st : b->streams)
    if ((e = hipStreamWaitEvent(st, b->fork, 0)) != hipSuccess) return batch_fail(HFMM_ERR_DEVICE, "fork", e);
  for (size_t i = 0; i < b->order.size(); ++i) {
    const int g = b->order[i];
    hfmm_status_t st = hfmm_apply(b->plans[g], q[g], u[g], nrhs, (hfmm_stream_t)b->streams[i % b->streams.size()]);
    if (st != HFMM_OK) return st;
  }
  for (size_t k = 0; k < b->streams.size(); ++k) {
    if ((e = hipEventRecord(b->joins[k], b->streams[k])) != hipSuccess) return batch_fail(HFMM_ERR_DEVICE, "join", e);
    if ((e = hipStreamWaitEvent(s, b->joins[k], 0)) != hipSuccess) return batch_fail(HFMM_ERR_DEVICE, "join", e);
  }
  return HFMM_OK;
}

}  // namespace

extern "C" {

hfmm_status_t hfmm_plan_batch(hfmm_batch_t* out, int32_t nplans, int32_t layers, const double* wavenumbers,
                              const double* interfaces, const int64_t* n, const double* const* points, double tol,
                              const hfmm_options_t* opts, hfmm_stream_t stream) {
  if (!out || !n || !points || nplans < 1)
    return hfmm::report(HFMM_ERR_INVALID_ARG, "NULL out, n or points, or nplans < 1");
  *out = nullptr;
  hfmm_batch_t b = new hfmm_batch_s();
  for (int g = 0; g < nplans; ++g) {
    hfmm_plan_t p = nullptr;
    hfmm_status_t st = hfmm_plan(&p, layers, wavenumbers, interfaces, n[g], points[g], tol, opts, stream);
    if (st != HFMM_OK) {
      delete b;
      return st;
    }
    b->plans.push_back(p);
  }
  b->order.resize(nplans);
  for (int g = 0; g < nplans; ++g) b->order[g] = g;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
    return hfmm::plan_points(b->plans[a]) > hfmm::plan_points(b->plans[c]);
  });
  const int ns = std::min(nplans, kBatchStreams);
  for (int k = 0; k < ns; ++k) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    hipError_t he = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&e, hipEventDisableTiming);
    if (he != hipSuccess) {
      if (s) (void)hipStreamDestroy(s);
      delete b;
      return batch_fail(HFMM_ERR_DEVICE, "streams", he);
    }
    b->streams.push_back(s);
    b->joins.push_back(e);
  }
  hipError_t fe = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (fe == hipSuccess) fe = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (fe != hipSuccess) {
    delete b;
    return batch_fail(HFMM_ERR_DEVICE, "events", fe);
  }
  *out = b;
  return HFMM_OK;
}

hfmm_status_t hfmm_batch_plan(hfmm_batch_t b, int32_t g, hfmm_plan_t* out) {
  if (!b || !out || g < 0 || g >= (int)b->plans.size())
    return hfmm::report(HFMM_ERR_INVALID_ARG, "NULL batch or out, or plan index out of range");
  *out = b->plans[g];
  return HFMM_OK;
}

hfmm_status_t hfmm_batch_graph(hfmm_batch_t b, int32_t enable) {
  if (!b) return hfmm::report(HFMM_ERR_INVALID_ARG, "NULL batch");
  b->graph_on = enable != 0;
  if (!b->graph_on) b->release_graph();
  for (hfmm_plan_t p : b->plans)
    if (b->graph_on) (void)hfmm_profile_enable(p, 0);  // no stage events inside a graph
  return HFMM_OK;
}

hfmm_status_t hfmm_apply_batch(hfmm_batch_t b, const double* const* q, double* const* u, int32_t nrhs,
                               hfmm_stream_t stream_) {
  if (!b || !q || !u) return hfmm::report(HFMM_ERR_INVALID_ARG, "NULL batch, q or u");
  if (nrhs < 1) return hfmm::report(HFMM_ERR_INVALID_ARG, "nrhs must be >= 1");
  const int G = (int)b->plans.size();
  for (int g = 0; g < G; ++g)
    if (!q[g] || !u[g]) return hfmm::report(HFMM_ERR_INVALID_ARG, "NULL q[g] or u[g]");
  hipStream_t s = (hipStream_t)stream_;
  for (hfmm_plan_t p : b->plans) {
    hfmm_status_t st = hfmm::plan_reserve(p, nrhs, s);
    if (st != HFMM_OK) return st;
  }
  if (!b->graph_on) {
    const hfmm_status_t st = enqueue(b, q, u, nrhs, s);
    if (st != HFMM_OK) return st;
    const hipError_t e = hipEventRecord(b->done, s);
    return e == hipSuccess ? HFMM_OK : batch_fail(HFMM_ERR_DEVICE, "record", e);
  }
  // A captured graph holds the plans' workspace pointers: a plan whose
  // workspace was reallocated since (a direct apply with more right-hand
  // sides) makes the graph stale.
  std::vector<int64_t> gen(G);
  for (int g = 0; g < G; ++g) gen[g] = hfmm::plan_workspace_generation(b->plans[g]);
  const bool same = b->exec && b->gnrhs == nrhs && b->gstream == s && b->ggen == gen &&
                    std::equal(b->gq.begin(), b->gq.end(), q) && std::equal(b->gu.begin(), b->gu.end(), u);
  if (!same) {
    b->release_graph();
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return batch_fail(HFMM_ERR_DEVICE, "begin capture", e);
    hfmm_status_t st = enqueue(b, q, u, nrhs, s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (st != HFMM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return batch_fail(HFMM_ERR_DEVICE, "end capture", e);
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return batch_fail(HFMM_ERR_DEVICE, "instantiate", e);
    }
    b->gq.assign(q, q + G);
    b->gu.assign(u, u + G);
    b->ggen = gen;
    b->gnrhs = nrhs;
    b->gstream = s;
  }
  hipError_t le = hipGraphLaunch(b->exec, s);
  if (le == hipSuccess) le = hipEventRecord(b->done, s);
  return le == hipSuccess ? HFMM_OK : batch_fail(HFMM_ERR_DEVICE, "graph launch", le);
}

void hfmm_batch_destroy(hfmm_batch_t b) { delete b; }

}  // extern "C"
