// Captured search launches ("plans"): one batch shape, fixed buffers, the
// query count read from device memory, recorded once as a HIP graph and
// replayed on any stream.
//
// A plan owns its workspace (visited bitsets, logs, queue counter, HBM beam
// lists), so replays never share scratch memory with ann_search_ex or with
// other plans.  The graph holds two kernel nodes: the queue-counter reset
// (a kernel, not a memset node) and the persistent search kernel; the search
// kernel clamps the device-held count to the capacity the plan was made
// for.  Replays of one plan are ordered on the device by an event, whatever
// streams they use, because they share the workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>

#include "ann.h"
#include "internal.h"

using namespace ann;

struct ann_plan {
  ann_index* ix = nullptr;
  Workspace ws;
  int64_t slots = 0;
  hipStream_t cap = nullptr;        // the stream the graph was captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool used = false;
  ann_launch_cfg launch{};          // the launch shape recorded in the graph

  ~ann_plan() {
    if (done) (void)hipEventSynchronize(done);
    ws.release();
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

extern "C" {

int ann_plan_create(const ann_index* cix, const ann_batch* b, const int32_t* nq_dev,
                    ann_plan** out) {
  if (!cix || !b || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  if (!nq_dev) return fail(ANN_EINVAL, "a plan reads its batch size from device memory (nq_dev)");
  if (b->nq < 1) return fail(ANN_EINVAL, "a plan needs a capacity nq >= 1");
  ann_index* ix = const_cast<ann_index*>(cix);
  SearchParams P;
  int rc = make_params(ix, b, &P);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(ix->mu);
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  std::unique_ptr<ann_plan> pl(new ann_plan);
  pl->ix = ix;
  pl->launch = ix->cfg[b->mode];
  pl->slots = pick_slots(ix, P, ix->cfg[b->mode].slots);
  if ((rc = ensure_workspace(ix, pl->ws, pl->slots, P.glist ? P.ef_cap : 0))) return rc;
  bind_workspace(P, pl->ws);
  P.nq_dev = nq_dev;
  const size_t lds = lds_bytes(P);
  if (lds > 65536) {
    const void* fn = kernel_symbol(P);
    if (fn) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  HIP_OR_RETURN(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking), "hipStreamCreate");
  HIP_OR_RETURN(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  const hipError_t le = launch_search(P, (int)pl->slots, lds, pl->cap);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(pl->cap, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(le, "captured search launch");
  }
  HIP_OR_RETURN(ce, "hipStreamEndCapture");
  pl->graph = g;
  HIP_OR_RETURN(hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  HIP_OR_RETURN(hipEventCreateWithFlags(&pl->done, hipEventDisableTiming), "hipEventCreate");
  pl->launch.slots = (int32_t)pl->slots;
  if (!pl->launch.lanes_per_row) pl->launch.lanes_per_row = P.lanes_per_row;
  if (!pl->launch.waves_per_query) pl->launch.waves_per_query = P.waves_per_query;
  *out = pl.release();
  return ANN_OK;
}

int ann_plan_launch(ann_plan* pl, void* stream) {
  if (!pl) return fail(ANN_EINVAL, "plan is NULL");
  HIP_OR_RETURN(hipSetDevice(pl->ix->device), "hipSetDevice");
  hipStream_t st = stream ? (hipStream_t)stream : pl->ix->stream;
  if (pl->used) HIP_OR_RETURN(hipStreamWaitEvent(st, pl->done, 0), "hipStreamWaitEvent");
  HIP_OR_RETURN(hipGraphLaunch(pl->exec, st), "hipGraphLaunch");
  HIP_OR_RETURN(hipEventRecord(pl->done, st), "hipEventRecord");
  pl->used = true;
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "plan replay");
  return ANN_OK;
}

int ann_plan_info(const ann_plan* pl, ann_launch_cfg* out) {
  if (!pl || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = pl->launch;
  return ANN_OK;
}

int ann_plan_free(ann_plan* pl) {
  if (!pl) return ANN_OK;
  (void)hipSetDevice(pl->ix->device);
  delete pl;
  return ANN_OK;
}

}  // extern "C"
