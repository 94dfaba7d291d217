// Continuous-batching server over the persistent search kernel.
//
// One host thread admits queued requests into free launch lanes.  Each lane
// owns a HIP stream, a workspace (visited bitsets for its slots), pinned
// staging buffers and device buffers for one batch; a lane is free again
// once its completion event has fired.  Requests that arrive while other
// batches run are admitted into the next free lane, so batches of different
// sizes and different (k, ef) overlap on the device.  Admission is bounded by
// max_inflight (queries on the device), max_batch (queries per launch) and
// the device memory budget fixed at creation.
//
// Each lane replays one captured HIP graph (queue-counter reset + persistent
// search kernel) per batch; the kernel reads the batch size from device
// memory, so the same graph serves batches of every size.
//
// Results do not depend on how requests were batched: the kernel evaluates
// every query with the same fixed arithmetic whatever its neighbours in the
// batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "ann.h"
#include "internal.h"

using namespace ann;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t tag;
  int32_t k, ef;
  double t_submit;
  std::vector<float> q;
};

struct Done {
  uint64_t tag;
  int32_t status, k;
  std::vector<int64_t> ids;
  std::vector<float> dists;
  double t_submit, t_start, t_done;
};

struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  Workspace ws;
  float* dq = nullptr;
  int32_t* dk = nullptr;
  int32_t* def = nullptr;
  int64_t* dids = nullptr;
  float* dd = nullptr;
  int32_t* dstat = nullptr;
  int32_t* dnq = nullptr;            // query count of the batch on the device
  int32_t* hnq = nullptr;
  hipGraph_t graph = nullptr;        // [counter reset, search] captured once
  hipGraphExec_t exec = nullptr;
  float* hq = nullptr;
  int32_t* hk = nullptr;
  int32_t* hef = nullptr;
  int64_t* hids = nullptr;
  float* hd = nullptr;
  int32_t* hstat = nullptr;
  std::vector<Req> batch;
  bool busy = false;
  double t_start = 0.0;
};

}  // namespace

struct ann_server {
  ann_index* ix = nullptr;
  ann_server_cfg cfg{};
  int64_t slots = 0;
  std::vector<Lane> lanes;
  SearchParams proto{};              // kernel parameters shared by the lanes
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req> queue;
  std::deque<Done> done;
  int64_t inflight = 0;
  bool stop = false;
  int loop_error = ANN_OK;
  std::thread th;

  int launch(Lane& L, std::vector<Req>&& reqs);
  int capture(Lane& L);
  void collect(Lane& L);
  void loop();
  void free_lanes();
};

int ann_server::launch(Lane& L, std::vector<Req>&& reqs) {
  const int m = (int)reqs.size();
  const int d = ix->d;
  for (int i = 0; i < m; ++i) {
    std::memcpy(L.hq + (size_t)i * d, reqs[i].q.data(), sizeof(float) * d);
    L.hk[i] = reqs[i].k;
    L.hef[i] = reqs[i].ef;
  }
  HIP_OR_RETURN(hipMemcpyAsync(L.dq, L.hq, sizeof(float) * (size_t)m * d, hipMemcpyHostToDevice, L.st), "H2D queries");
  HIP_OR_RETURN(hipMemcpyAsync(L.dk, L.hk, sizeof(int32_t) * m, hipMemcpyHostToDevice, L.st), "H2D k");
  HIP_OR_RETURN(hipMemcpyAsync(L.def, L.hef, sizeof(int32_t) * m, hipMemcpyHostToDevice, L.st), "H2D ef");
  *L.hnq = m;
  HIP_OR_RETURN(hipMemcpyAsync(L.dnq, L.hnq, sizeof(int32_t), hipMemcpyHostToDevice, L.st), "H2D nq");
  HIP_OR_RETURN(hipGraphLaunch(L.exec, L.st), "hipGraphLaunch");
  const size_t kk = (size_t)m * cfg.k_max;
  HIP_OR_RETURN(hipMemcpyAsync(L.hids, L.dids, sizeof(int64_t) * kk, hipMemcpyDeviceToHost, L.st), "D2H ids");
  HIP_OR_RETURN(hipMemcpyAsync(L.hd, L.dd, sizeof(float) * kk, hipMemcpyDeviceToHost, L.st), "D2H dists");
  HIP_OR_RETURN(hipMemcpyAsync(L.hstat, L.dstat, sizeof(int32_t) * m, hipMemcpyDeviceToHost, L.st), "D2H status");
  HIP_OR_RETURN(hipEventRecord(L.ev, L.st), "hipEventRecord");
  L.batch = std::move(reqs);
  L.busy = true;
  L.t_start = now_s();
  return ANN_OK;
}

// Records the lane's two kernels (queue-counter reset and the persistent
// search) as a graph: the batch size is read from L.dnq on the device, so one
// graph serves every batch of the lane.
int ann_server::capture(Lane& L) {
  SearchParams P = proto;
  P.nq = cfg.max_batch;
  P.nq_dev = L.dnq;
  P.queries = L.dq;
  P.k_arr = L.dk;
  P.ef_arr = L.def;
  P.out_ids = L.dids;
  P.out_dists = L.dd;
  P.out_status = L.dstat;
  bind_workspace(P, L.ws);
  const size_t lds = lds_bytes(P);
  if (lds > 65536) {
    const void* fn = kernel_symbol(P);
    if (fn) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  HIP_OR_RETURN(hipStreamBeginCapture(L.st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  const hipError_t le = launch_search(P, (int)std::min<int64_t>(slots, cfg.max_batch), lds, L.st);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(L.st, &g);
  if (le != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(le, "captured search launch"); }
  HIP_OR_RETURN(ce, "hipStreamEndCapture");
  L.graph = g;
  HIP_OR_RETURN(hipGraphInstantiate(&L.exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  return ANN_OK;
}

void ann_server::collect(Lane& L) {
  const double t = now_s();
  std::vector<Done> out;
  out.reserve(L.batch.size());
  for (size_t i = 0; i < L.batch.size(); ++i) {
    const Req& r = L.batch[i];
    Done c;
    c.tag = r.tag;
    c.status = L.hstat[i] == 0 ? ANN_OK : ANN_EBUDGET;
    c.k = r.k;
    c.ids.assign(L.hids + i * cfg.k_max, L.hids + i * cfg.k_max + r.k);
    c.dists.assign(L.hd + i * cfg.k_max, L.hd + i * cfg.k_max + r.k);
    c.t_submit = r.t_submit;
    c.t_start = L.t_start;
    c.t_done = t;
    out.push_back(std::move(c));
  }
  std::lock_guard<std::mutex> lk(mu);
  for (auto& c : out) done.push_back(std::move(c));
  inflight -= (int64_t)L.batch.size();
  L.batch.clear();
  L.busy = false;
}

void ann_server::loop() {
  if (hipSetDevice(ix->device) != hipSuccess) { loop_error = ANN_EHIP; return; }
  while (true) {
    bool progressed = false;
    for (Lane& L : lanes) {
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.ev);
      if (q == hipSuccess) { collect(L); progressed = true; }
      else if (q != hipErrorNotReady) { loop_error = hip_fail(q, "server batch"); collect(L); }
    }
    bool any_busy = false;
    for (Lane& L : lanes) {
      if (L.busy) { any_busy = true; continue; }
      std::vector<Req> take;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (stop) break;
        const int64_t room = std::min<int64_t>(cfg.max_inflight - inflight, cfg.max_batch);
        const int64_t m = std::min<int64_t>(room, (int64_t)queue.size());
        if (m <= 0) continue;
        for (int64_t i = 0; i < m; ++i) { take.push_back(std::move(queue.front())); queue.pop_front(); }
        inflight += m;
      }
      const int rc = launch(L, std::move(take));
      if (rc) {
        // launch() keeps `take` untouched on failure: report its requests
        loop_error = rc;
        const double t = now_s();
        std::lock_guard<std::mutex> lk(mu);
        for (const Req& r : take) done.push_back(Done{r.tag, rc, 0, {}, {}, r.t_submit, t, t});
        inflight -= (int64_t)take.size();
      }
      progressed = true;
      any_busy = any_busy || L.busy;
    }
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop && !any_busy) {
        bool busy = false;
        for (Lane& L : lanes) busy = busy || L.busy;
        if (!busy) break;
      }
      if (!progressed) cv.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 500));
    }
  }
}

void ann_server::free_lanes() {
  for (Lane& L : lanes) {
    if (L.st) (void)hipStreamSynchronize(L.st);
    L.ws.release();
    if (L.exec) (void)hipGraphExecDestroy(L.exec);
    if (L.graph) (void)hipGraphDestroy(L.graph);
    void* dev[] = {L.dq, L.dk, L.def, L.dids, L.dd, L.dstat, L.dnq};
    for (void* p : dev)
      if (p) (void)hipFree(p);
    void* host[] = {L.hq, L.hk, L.hef, L.hids, L.hd, L.hstat, L.hnq};
    for (void* p : host)
      if (p) (void)hipHostFree(p);
    if (L.ev) (void)hipEventDestroy(L.ev);
    if (L.st) (void)hipStreamDestroy(L.st);
  }
  lanes.clear();
}

extern "C" {

int ann_server_create(const ann_index* cix, const ann_server_cfg* cfg, ann_server** out) {
  if (!cix || !cfg || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  const ann_server_cfg& c = *cfg;
  if (c.mode < ANN_MODE_F32 || c.mode > ANN_MODE_FP8) return fail(ANN_EINVAL, "server modes are the dense ones (0..3)");
  if (c.rerank < 0 || c.max_inflight < 1 || c.max_batch < 1 || c.streams < 1 || c.streams > 4 ||
      c.k_max < 1 || c.k_max > ANN_K_MAX || c.ef_max < 1 || c.queue_cap < 1 || c.hbm_budget < 1)
    return fail(ANN_EINVAL, "bad server configuration");
  if (std::max(c.ef_max, c.k_max) > ANN_EF_MAX) return fail(ANN_EBUDGET, "ef_max above ANN_EF_MAX");
  ann_index* ix = const_cast<ann_index*>(cix);
  // a dry batch validates mode, rerank and the on-chip memory for ef_max,
  // and gives the kernel parameters every lane shares
  ann_batch b;
  std::memset(&b, 0, sizeof b);
  b.mode = c.mode; b.rerank = c.rerank; b.nq = 0; b.k_all = 1; b.ef_all = 1;
  b.k_max = c.k_max; b.ef_max = c.ef_max;
  SearchParams P;
  int rc = make_params(ix, &b, &P);
  if (rc) return rc;
  const SearchParams proto = P;
  std::unique_ptr<ann_server> s(new ann_server);
  s->ix = ix;
  s->cfg = c;
  const int64_t max_batch = std::min<int64_t>(c.max_batch, c.max_inflight);
  // device memory of one lane: batch buffers + workspace
  const int64_t batch_bytes = max_batch * ((int64_t)ix->d * 4 + 8 + (int64_t)c.k_max * 12 + 4);
  P.nq = max_batch;
  int64_t slots = pick_slots(ix, P, 0);
  const int64_t per_slot = slot_bytes(ix->n) + (proto.glist ? (int64_t)proto.ef_cap * 16 : 0);
  while (slots > 1 && c.streams * (batch_bytes + slots * per_slot) > c.hbm_budget) slots /= 2;
  if (c.streams * (batch_bytes + slots * per_slot) > c.hbm_budget)
    return fail(ANN_EBUDGET, "hbm_budget %lld too small for one slot per stream", (long long)c.hbm_budget);
  s->slots = slots;
  s->proto = proto;
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  s->lanes.resize(c.streams);
  for (Lane& L : s->lanes) {
    HIP_OR_RETURN(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking), "hipStreamCreate");
    HIP_OR_RETURN(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming), "hipEventCreate");
    if ((rc = ensure_workspace(ix, L.ws, slots, proto.glist ? proto.ef_cap : 0))) {
      s->free_lanes();
      return rc;
    }
    const size_t nb = (size_t)max_batch;
    HIP_OR_RETURN(hipMalloc((void**)&L.dq, sizeof(float) * nb * ix->d), "hipMalloc");
    HIP_OR_RETURN(hipMalloc((void**)&L.dk, sizeof(int32_t) * nb), "hipMalloc");
    HIP_OR_RETURN(hipMalloc((void**)&L.def, sizeof(int32_t) * nb), "hipMalloc");
    HIP_OR_RETURN(hipMalloc((void**)&L.dids, sizeof(int64_t) * nb * c.k_max), "hipMalloc");
    HIP_OR_RETURN(hipMalloc((void**)&L.dd, sizeof(float) * nb * c.k_max), "hipMalloc");
    HIP_OR_RETURN(hipMalloc((void**)&L.dstat, sizeof(int32_t) * nb), "hipMalloc");
    HIP_OR_RETURN(hipHostMalloc((void**)&L.hq, sizeof(float) * nb * ix->d, hipHostMallocDefault), "hipHostMalloc");
    HIP_OR_RETURN(hipHostMalloc((void**)&L.hk, sizeof(int32_t) * nb, hipHostMallocDefault), "hipHostMalloc");
    HIP_OR_RETURN(hipHostMalloc((void**)&L.hef, sizeof(int32_t) * nb, hipHostMallocDefault), "hipHostMalloc");
    HIP_OR_RETURN(hipHostMalloc((void**)&L.hids, sizeof(int64_t) * nb * c.k_max, hipHostMallocDefault), "hipHostMalloc");
    HIP_OR_RETURN(hipHostMalloc((void**)&L.hd, sizeof(float) * nb * c.k_max, hipHostMallocDefault), "hipHostMalloc");
    HIP_OR_RETURN(hipHostMalloc((void**)&L.hstat, sizeof(int32_t) * nb, hipHostMallocDefault), "hipHostMalloc");
    HIP_OR_RETURN(hipMalloc((void**)&L.dnq, sizeof(int32_t)), "hipMalloc");
    HIP_OR_RETURN(hipHostMalloc((void**)&L.hnq, sizeof(int32_t), hipHostMallocDefault), "hipHostMalloc");
  }
  s->cfg.max_batch = (int32_t)max_batch;
  for (Lane& L : s->lanes)
    if ((rc = s->capture(L))) { s->free_lanes(); return rc; }
  ann_server* raw = s.get();
  s->th = std::thread([raw] { raw->loop(); });
  *out = s.release();
  return ANN_OK;
}

int ann_server_submit(ann_server* s, const ann_request* r) {
  if (!s || !r || !r->query) return fail(ANN_EINVAL, "NULL argument");
  if (r->k < 1 || r->k > s->cfg.k_max) return fail(ANN_EINVAL, "k %d outside [1, %d]", r->k, s->cfg.k_max);
  if (r->ef < 1 || r->ef > s->cfg.ef_max) return fail(ANN_EINVAL, "ef %d outside [1, %d]", r->ef, s->cfg.ef_max);
  Req q;
  q.tag = r->tag;
  q.k = r->k;
  q.ef = r->ef;
  q.t_submit = now_s();
  q.q.assign(r->query, r->query + s->ix->d);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(ANN_EINVAL, "server is stopping");
    if ((int64_t)s->queue.size() >= s->cfg.queue_cap) return fail(ANN_EAGAIN, "queue full");
    s->queue.push_back(std::move(q));
  }
  s->cv.notify_one();
  return ANN_OK;
}

int ann_server_poll(ann_server* s, ann_completion* out, int32_t max) {
  if (!s || (!out && max > 0)) return -fail(ANN_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t n = 0;
  while (n < max && !s->done.empty()) {
    Done& c = s->done.front();
    ann_completion& o = out[n++];
    o.tag = c.tag;
    o.status = c.status;
    o.k = c.k;
    for (int j = 0; j < c.k && j < (int)c.ids.size(); ++j) { o.ids[j] = c.ids[j]; o.dists[j] = c.dists[j]; }
    o.t_submit = c.t_submit;
    o.t_start = c.t_start;
    o.t_done = c.t_done;
    s->done.pop_front();
  }
  return n;
}

int ann_server_destroy(ann_server* s) {
  if (!s) return ANN_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();   // not yet admitted: cancelled
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  s->free_lanes();
  const int err = s->loop_error;
  delete s;
  return err;
}

}  // extern "C"
