// Continuous batching over the persistent search kernel, admitted per slot.
//
// The server keeps one persistent search kernel on the device whose
// workgroups ("slots") take requests one at a time from a ring in pinned
// host memory (RingArgs in search_kernels.h).  A host thread moves submitted
// requests into free ring entries and publishes them; the first slot that
// is free claims the next published request, so a request that arrives while
// others run starts as soon as any one slot is free, without waiting for a
// batch to end, and its work overlaps theirs on the device.  Results are
// written by the kernel straight into the ring entry (host memory) with a
// completion flag; the host thread collects them.
//
// The kernel ends as a whole when nothing has been claimed or published for
// idle_us and no request is in flight (or when the server stops); the host
// thread launches it again when new requests are waiting.  Results do not depend on which slot serves a
// request or on what else runs: every key is evaluated in the fixed order.
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
  uint64_t tag = 0;
  int32_t k = 0, ef = 0;
  double t_submit = 0.0, t_start = 0.0;
  std::vector<float> q;
};

struct Done {
  uint64_t tag;
  int32_t status, k, slot;
  std::vector<int64_t> ids;
  std::vector<float> dists;
  double t_submit, t_start, t_done, d_start, d_done;
};

constexpr double kPollUs = 2.0;     // how often one waiting slot reads the host's ring tail

}  // namespace

struct ann_server {
  ann_index* ix = nullptr;
  ann_server_cfg cfg{};
  int64_t slots = 0;
  int64_t R = 0;                     // ring entries
  SearchParams P{};
  Workspace ws;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  bool running = false;
  double clock_hz = 1e8;
  // ring in pinned host memory (h_*: host addresses, d_*: the same memory as
  // the device addresses it)
  void* hblock = nullptr;
  uint64_t* h_tail = nullptr;
  uint32_t* h_stop = nullptr;
  float* h_q = nullptr;
  int32_t* h_k = nullptr;
  int32_t* h_ef = nullptr;
  int64_t* h_ids = nullptr;
  float* h_d = nullptr;
  int32_t* h_status = nullptr;
  uint64_t* h_done = nullptr;
  uint64_t* h_tstart = nullptr;
  uint64_t* h_tdone = nullptr;
  int32_t* h_served = nullptr;
  uint64_t* d_ctl = nullptr;         // device: head, mirror, last poll, activity, busy
  void* d_stage = nullptr;           // device: each slot's copy of its request and results
  std::vector<int64_t> entry_seq;    // request occupying each entry, -1 when free
  std::vector<Req> entry_req;
  uint64_t next_seq = 0;             // requests published
  uint64_t oldest = 0;               // every request below this one has been collected
  uint64_t completed = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req> queue;
  std::deque<Done> done;
  bool stop = false;
  int loop_error = ANN_OK;
  std::thread th;

  int launch();
  bool collect();
  bool admit();
  void loop();
  void release();
};

int ann_server::launch() {
  const size_t lds = lds_bytes(P);
  const void* fn = kernel_symbol(P);
  if (!fn) return fail(ANN_EUNSUP, "no search kernel for the server's mode");
  if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  ring_rearm(P.ring, st);
  HIP_OR_RETURN(hipGetLastError(), "ring rearm");
  SearchParams arg = P;
  void* args[] = {&arg};
  HIP_OR_RETURN(hipLaunchKernel(fn, dim3((unsigned)slots), dim3(64 * P.waves_per_query), args, lds, st),
                "server kernel launch");
  HIP_OR_RETURN(hipEventRecord(ev, st), "hipEventRecord");
  running = true;
  return ANN_OK;
}

// Moves finished requests from the ring to the completion list.
bool ann_server::collect() {
  bool any = false;
  std::vector<Done> out;
  const double t = now_s();
  for (uint64_t seq = oldest; seq < next_seq; ++seq) {
    const int64_t e = (int64_t)(seq % (uint64_t)R);
    if (entry_seq[e] != (int64_t)seq) continue;
    if (__atomic_load_n(&h_done[e], __ATOMIC_ACQUIRE) != seq + 1) continue;
    Req& r = entry_req[e];
    Done c;
    c.tag = r.tag;
    c.status = h_status[e] == 0 ? ANN_OK : ANN_EBUDGET;
    c.k = r.k;
    c.slot = h_served[e];
    c.ids.assign(h_ids + e * cfg.k_max, h_ids + e * cfg.k_max + r.k);
    c.dists.assign(h_d + e * cfg.k_max, h_d + e * cfg.k_max + r.k);
    c.t_submit = r.t_submit;
    c.t_start = r.t_start;
    c.t_done = t;
    c.d_start = (double)h_tstart[e] / clock_hz;
    c.d_done = (double)h_tdone[e] / clock_hz;
    out.push_back(std::move(c));
    entry_seq[e] = -1;
    ++completed;
    any = true;
  }
  while (oldest < next_seq && entry_seq[oldest % (uint64_t)R] != (int64_t)oldest) ++oldest;
  if (any) {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& c : out) done.push_back(std::move(c));
  }
  return any;
}

// Writes waiting requests into free ring entries and publishes them.
bool ann_server::admit() {
  std::vector<Req> take;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (stop) return false;
    uint64_t seq = next_seq;
    while (!queue.empty() && seq - completed < (uint64_t)R &&
           entry_seq[seq % (uint64_t)R] == -1) {
      take.push_back(std::move(queue.front()));
      queue.pop_front();
      ++seq;
    }
  }
  if (take.empty()) return false;
  const int d = ix->d;
  const double t = now_s();
  for (Req& r : take) {
    const int64_t e = (int64_t)(next_seq % (uint64_t)R);
    std::memcpy(h_q + (size_t)e * d, r.q.data(), sizeof(float) * d);
    h_k[e] = r.k;
    h_ef[e] = r.ef;
    h_done[e] = 0;
    r.t_start = t;
    entry_seq[e] = (int64_t)next_seq;
    entry_req[e] = std::move(r);
    ++next_seq;
  }
  // the entries are written before the tail that publishes them
  __atomic_store_n(h_tail, next_seq, __ATOMIC_RELEASE);
  return true;
}

void ann_server::loop() {
  if (hipSetDevice(ix->device) != hipSuccess) { loop_error = ANN_EHIP; return; }
  while (true) {
    bool progressed = collect();
    if (running) {
      const hipError_t q = hipEventQuery(ev);
      if (q == hipSuccess) {
        running = false;
      } else if (q != hipErrorNotReady) {
        loop_error = hip_fail(q, "server kernel");
        running = false;
      }
    }
    progressed = admit() || progressed;
    bool stopping;
    {
      std::lock_guard<std::mutex> lk(mu);
      stopping = stop;
    }
    if (stopping) {
      // no new work: the running requests finish, waiting ones are dropped
      __atomic_store_n(h_stop, 1u, __ATOMIC_RELEASE);
      if (running) (void)hipEventSynchronize(ev);
      running = false;
      collect();
      return;
    }
    // a published request that no running kernel will claim: (re)launch
    if (!running && next_seq > completed && loop_error == ANN_OK) {
      const int rc = launch();
      if (rc) loop_error = rc;
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait_for(lk, std::chrono::microseconds(next_seq > completed ? 20 : 500));
    }
  }
}

void ann_server::release() {
  if (st) (void)hipStreamSynchronize(st);
  ws.release();
  if (d_ctl) (void)hipFree(d_ctl);
  if (d_stage) (void)hipFree(d_stage);
  d_stage = nullptr;
  if (hblock) (void)hipHostFree(hblock);
  if (ev) (void)hipEventDestroy(ev);
  if (st) (void)hipStreamDestroy(st);
  d_ctl = nullptr;
  hblock = nullptr;
  ev = nullptr;
  st = nullptr;
}

extern "C" {

int ann_server_create(const ann_index* cix, const ann_server_cfg* cfg, ann_server** out) {
  if (!cix || !cfg || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  const ann_server_cfg& c = *cfg;
  if (c.mode < ANN_MODE_F32 || c.mode > ANN_MODE_FP8)
    return fail(ANN_EINVAL, "server modes are the dense ones (0..3)");
  if (c.rerank < 0 || c.max_inflight < 1 || c.slots < 0 || c.k_max < 1 || c.k_max > ANN_K_MAX ||
      c.ef_max < 1 || c.queue_cap < 1 || c.hbm_budget < 1 || c.idle_us < 0)
    return fail(ANN_EINVAL, "bad server configuration");
  if (std::max(c.ef_max, c.k_max) > ANN_EF_MAX) return fail(ANN_EBUDGET, "ef_max above ANN_EF_MAX");
  ann_index* ix = const_cast<ann_index*>(cix);
  // a dry batch validates mode, rerank and the on-chip memory for ef_max and
  // gives the kernel parameters
  ann_batch b;
  std::memset(&b, 0, sizeof b);
  b.mode = c.mode; b.rerank = c.rerank; b.nq = 0; b.k_all = 1; b.ef_all = 1;
  b.k_max = c.k_max; b.ef_max = c.ef_max;
  SearchParams P;
  int rc = make_params(ix, &b, &P);
  if (rc) return rc;
  std::unique_ptr<ann_server> s(new ann_server);
  s->ix = ix;
  s->cfg = c;
  if (!s->cfg.idle_us) s->cfg.idle_us = 2000;
  s->R = c.max_inflight;
  P.nq = c.max_inflight;
  P.ring.cap = s->R;       // the occupancy is the server kernel's
  int64_t slots = pick_slots(ix, P, c.slots);
  const int64_t per_slot = slot_bytes(ix->n) + (P.glist ? (int64_t)P.ef_cap * 16 : 0);
  while (slots > 1 && slots * per_slot > c.hbm_budget) slots /= 2;
  if (slots * per_slot > c.hbm_budget)
    return fail(ANN_EBUDGET, "hbm_budget %lld too small for one slot", (long long)c.hbm_budget);
  s->slots = slots;
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  int rate_khz = 0;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ix->device) == hipSuccess &&
      rate_khz > 0)
    s->clock_hz = 1e3 * rate_khz;
  HIP_OR_RETURN(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking), "hipStreamCreate");
  HIP_OR_RETURN(hipEventCreateWithFlags(&s->ev, hipEventDisableTiming), "hipEventCreate");
  if ((rc = ensure_workspace(ix, s->ws, slots, P.glist ? P.ef_cap : 0))) { s->release(); return rc; }
  // the ring: one pinned, coherent host block
  const size_t Rn = (size_t)s->R, d = (size_t)ix->d, km = (size_t)c.k_max;
  size_t off = 0;
  auto carve = [&](size_t bytes) { const size_t o = off; off += (bytes + 63) & ~size_t(63); return o; };
  const size_t o_tail = carve(8), o_stop = carve(4), o_q = carve(4 * Rn * d), o_k = carve(4 * Rn),
               o_ef = carve(4 * Rn), o_ids = carve(8 * Rn * km), o_d = carve(4 * Rn * km),
               o_status = carve(4 * Rn), o_done = carve(8 * Rn), o_ts = carve(8 * Rn),
               o_td = carve(8 * Rn), o_sv = carve(4 * Rn);
  if (hipHostMalloc(&s->hblock, off, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    s->hblock = nullptr;
    s->release();
    return fail(ANN_ENOMEM, "pinned ring of %zu bytes", off);
  }
  std::memset(s->hblock, 0, off);
  void* dblock = nullptr;
  if (hipHostGetDevicePointer(&dblock, s->hblock, 0) != hipSuccess) {
    s->release();
    return fail(ANN_EHIP, "hipHostGetDevicePointer");
  }
  char* hb = (char*)s->hblock;
  char* db = (char*)dblock;
  s->h_tail = (uint64_t*)(hb + o_tail);
  s->h_stop = (uint32_t*)(hb + o_stop);
  s->h_q = (float*)(hb + o_q);
  s->h_k = (int32_t*)(hb + o_k);
  s->h_ef = (int32_t*)(hb + o_ef);
  s->h_ids = (int64_t*)(hb + o_ids);
  s->h_d = (float*)(hb + o_d);
  s->h_status = (int32_t*)(hb + o_status);
  s->h_done = (uint64_t*)(hb + o_done);
  s->h_tstart = (uint64_t*)(hb + o_ts);
  s->h_tdone = (uint64_t*)(hb + o_td);
  s->h_served = (int32_t*)(hb + o_sv);
  // head, mirror, last poll, activity and busy, 256 bytes apart
  // (separate cache lines)
  if (hipMalloc((void**)&s->d_ctl, 2048) != hipSuccess) { s->d_ctl = nullptr; s->release(); return fail(ANN_ENOMEM, "server control block"); }
  HIP_OR_RETURN(hipMemset(s->d_ctl, 0, 2048), "hipMemset");
  s->entry_seq.assign(Rn, -1);
  s->entry_req.resize(Rn);
  // kernel parameters: each slot searches a copy of its request in device
  // memory (row `slot` of these arrays); the ring entries are in RingArgs
  const size_t sn = (size_t)slots;
  size_t so = 0;
  auto scarve = [&](size_t bytes) { const size_t o = so; so += (bytes + 255) & ~size_t(255); return o; };
  const size_t s_q = scarve(4 * sn * d), s_k = scarve(4 * sn), s_ef = scarve(4 * sn),
               s_ids = scarve(8 * sn * km), s_d = scarve(4 * sn * km), s_st = scarve(4 * sn);
  if (hipMalloc(&s->d_stage, so) != hipSuccess) { s->d_stage = nullptr; s->release(); return fail(ANN_ENOMEM, "server staging"); }
  char* sb = (char*)s->d_stage;
  P.nq = slots;
  P.queries = (const float*)(sb + s_q);
  P.k_arr = (const int32_t*)(sb + s_k);
  P.ef_arr = (const int32_t*)(sb + s_ef);
  P.out_ids = (int64_t*)(sb + s_ids);
  P.out_dists = (float*)(sb + s_d);
  P.out_status = (int32_t*)(sb + s_st);
  bind_workspace(P, s->ws);
  RingArgs& r = P.ring;
  r.cap = s->R;
  r.host_tail = (const uint64_t*)(db + o_tail);
  r.host_stop = (const uint32_t*)(db + o_stop);
  r.head = s->d_ctl;
  r.mirror = s->d_ctl + 32;
  r.last_poll = s->d_ctl + 64;
  r.activity = s->d_ctl + 32 * 4;
  r.busy = (uint32_t*)(s->d_ctl + 32 * 5);
  r.waiting = (uint32_t*)(s->d_ctl + 32 * 6);   // kRingTiers counters, one line
  r.tier_width = std::max(1, ix->cu_count);
  r.e_query = (const float*)(db + o_q);
  r.e_k = (const int32_t*)(db + o_k);
  r.e_ef = (const int32_t*)(db + o_ef);
  r.e_ids = (int64_t*)(db + o_ids);
  r.e_dists = (float*)(db + o_d);
  r.e_status = (int32_t*)(db + o_status);
  r.done = (uint64_t*)(db + o_done);
  r.t_start = (uint64_t*)(db + o_ts);
  r.t_done = (uint64_t*)(db + o_td);
  r.served_by = (int32_t*)(db + o_sv);
  r.idle_ticks = (uint64_t)(s->clock_hz * 1e-6 * s->cfg.idle_us);
  r.poll_ticks = std::max<uint64_t>(1, (uint64_t)(s->clock_hz * 1e-6 * kPollUs));
  r.idle_spins = 64 + s->cfg.idle_us / 3;   // waits last at least 7 us
  s->P = P;
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
    if (s->loop_error) return fail(s->loop_error, "the server's kernel failed earlier (code %d)", s->loop_error);
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
    o.d_start = c.d_start;
    o.d_done = c.d_done;
    o.slot = c.slot;
    o.reserved = 0;
    s->done.pop_front();
  }
  return n;
}

int ann_server_info(const ann_server* s, ann_server_state* out) {
  if (!s || !out) return fail(ANN_EINVAL, "NULL argument");
  ann_server* m = const_cast<ann_server*>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  out->slots = (int32_t)s->slots;
  out->ring = (int32_t)s->R;
  out->waves_per_query = s->P.waves_per_query;
  out->lanes_per_row = s->P.lanes_per_row;
  out->queued = (int64_t)s->queue.size();
  return ANN_OK;
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
  s->release();
  const int err = s->loop_error;
  delete s;
  return err;
}

}  // extern "C"
