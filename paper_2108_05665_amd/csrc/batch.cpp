// Batched form: the full contraction of several plans captured as one hipGraph
// (one launch per batch), each plan on its own forked capture stream.

#include <cmath>
#include <cstring>
#include <limits>
#include <set>
#include <string>

#include "plan.h"

namespace xeb {

struct Batch {
  std::vector<Plan*> plans;
  std::vector<void*> amps;
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t nodes = 0;
  ~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

struct StreamSet {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  ~StreamSet() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
  }
  hipStream_t stream() {
    hipStream_t s;
    hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    streams.push_back(s);
    return s;
  }
  hipEvent_t event() {
    hipEvent_t e;
    hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
    events.push_back(e);
    return e;
  }
};

constexpr int kMaxSideStreams = 4;

}  // namespace

Batch* create_batch(Plan* const* plans, void* const* amps, int n) {
  if (n < 1) fail(XEB_EINVAL, "a batch needs at least one plan");
  if (!plans || !amps) fail(XEB_EINVAL, "plans or amps is NULL");
  std::set<Plan*> seen;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) fail(XEB_EINVAL, "plan handle is NULL");
    if (!seen.insert(plans[i]).second) fail(XEB_EINVAL, "a plan is listed twice");
    if (!plans[i]->ws) fail(XEB_ESTATE, "a plan has no workspace bound");
    if (plans[i]->k > 0 && !amps[i]) fail(XEB_EINVAL, "amps buffer is NULL");
    if (plans[i]->opt.device != plans[0]->opt.device)
      fail(XEB_EINVAL, "plans of one batch must share a device");
  }
  auto b = std::make_unique<Batch>();
  b->plans.assign(plans, plans + n);
  b->amps.assign(amps, amps + n);
  b->device = plans[0]->opt.device;

  int prev = -1;
  hip_check(hipGetDevice(&prev), "hipGetDevice");
  if (prev != b->device) hip_check(hipSetDevice(b->device), "hipSetDevice");
  struct Restore {
    int dev;
    ~Restore() {
      int cur = -1;
      if (hipGetDevice(&cur) == hipSuccess && cur != dev && dev >= 0) (void)hipSetDevice(dev);
    }
  } restore{prev};

  std::set<int> precs;
  for (Plan* p : b->plans) precs.insert(p->opt.precision);
  for (int pr : precs) prepare_mfma_launch(pr);

  StreamSet ss;
  hipStream_t cs = ss.stream();
  const int nside = n < kMaxSideStreams ? n : kMaxSideStreams;
  std::vector<hipStream_t> side(nside);
  for (int j = 0; j < nside; ++j) side[j] = ss.stream();
  hipEvent_t fork = ss.event();
  std::vector<hipEvent_t> join(nside);
  for (int j = 0; j < nside; ++j) join[j] = ss.event();

  hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  try {
    hip_check(hipEventRecord(fork, cs), "hipEventRecord");
    for (int j = 0; j < nside; ++j) hip_check(hipStreamWaitEvent(side[j], fork, 0), "hipStreamWaitEvent");
    for (int i = 0; i < n; ++i) {
      Plan* p = b->plans[i];
      if (p->k == 0) continue;
      hipStream_t st = side[i % nside];
      p->capturing = true;
      launch_zero(b->amps[i], (uint64_t(p->k) << p->w) * 16, st);
      contract_plan(p, 0, int64_t(1) << p->s, b->amps[i], st);
      launch_plan_xeb(p, b->amps[i], st);
      p->capturing = false;
    }
    for (int j = 0; j < nside; ++j) {
      hip_check(hipEventRecord(join[j], side[j]), "hipEventRecord");
      hip_check(hipStreamWaitEvent(cs, join[j], 0), "hipStreamWaitEvent");
    }
  } catch (...) {
    for (Plan* p : b->plans) p->capturing = false;
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hip_check(hipStreamEndCapture(cs, &b->graph), "hipStreamEndCapture");
  size_t nodes = 0;
  hip_check(hipGraphGetNodes(b->graph, nullptr, &nodes), "hipGraphGetNodes");
  if (nodes > XEB_BATCH_MAX_NODES)
    fail(XEB_ELIMIT, "batch graph has " + std::to_string(nodes) + " nodes, more than " +
                         std::to_string(XEB_BATCH_MAX_NODES) + "; split the batch");
  b->nodes = int64_t(nodes);
  hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  return b.release();
}

void launch_batch(Batch* b, hipStream_t stream) {
  int prev = -1;
  hip_check(hipGetDevice(&prev), "hipGetDevice");
  if (prev != b->device) hip_check(hipSetDevice(b->device), "hipSetDevice");
  hipError_t e = hipGraphLaunch(b->exec, stream);
  if (prev != b->device) (void)hipSetDevice(prev);
  hip_check(e, "hipGraphLaunch");
}

void batch_fidelities(Batch* b, hipStream_t stream, double* F) {
  if (!F) fail(XEB_EINVAL, "F is NULL");
  int prev = -1;
  hip_check(hipGetDevice(&prev), "hipGetDevice");
  if (prev != b->device) hip_check(hipSetDevice(b->device), "hipSetDevice");
  hipError_t e = hipStreamSynchronize(stream);
  for (size_t i = 0; e == hipSuccess && i < b->plans.size(); ++i) {
    Plan* p = b->plans[i];
    if (p->k == 0) {
      F[i] = std::numeric_limits<double>::quiet_NaN();
      continue;
    }
    e = hipMemcpy(&F[i], static_cast<char*>(p->ws) + p->off_scratch, sizeof(double),
                  hipMemcpyDeviceToHost);
  }
  if (prev != b->device) (void)hipSetDevice(prev);
  hip_check(e, "batch fidelities");
}

void destroy_batch(Batch* b) { delete b; }

}  // namespace xeb
