// C-ABI of the batched HNSW search library (declared in include/ann.h).
//
// Host side only: argument checks, device-resident index image, per-stream
// workspaces (visited bitsets, logs, the persistent queue counter), launch
// configuration and the autotuner.  All per-query work runs in the kernels
// of search_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ann.h"
#include "internal.h"
#include "search_kernels.h"

using namespace ann;

namespace ann {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(ANN_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(ANN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void Workspace::release() {
  if (bits) (void)hipFree(bits);
  if (vlog) (void)hipFree(vlog);
  if (counter) (void)hipFree(counter);
  if (beam_key) (void)hipFree(beam_key);
  if (beam_id) (void)hipFree(beam_id);
  if (done) (void)hipEventDestroy(done);
  bits = nullptr; vlog = nullptr; counter = nullptr; done = nullptr;
  beam_key = nullptr; beam_id = nullptr;
  slots = 0;
  beam_cap = 0;
  bytes = 0;
}

int64_t slot_bytes(int64_t n) {
  return ((n + 31) / 32) * 4 + 4 * std::max<int64_t>(256, std::min<int64_t>(n / 64, 1 << 20));
}

}  // namespace ann

namespace {

// Beams wider than this get an insert buffer when the launch leaves it to the
// library, and beams wider than kHbmListMinEf keep their list in HBM.
constexpr int kBufferMinEf = 1024;
constexpr int kHbmListMinEf = 4096;

template <class T>
int upload(T** dst, const T* src, size_t count, int64_t* bytes) {
  *dst = nullptr;
  if (!src || count == 0) return ANN_OK;
  HIP_OR_RETURN(hipMalloc((void**)dst, count * sizeof(T)), "hipMalloc (index)");
  HIP_OR_RETURN(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy (index)");
  *bytes += (int64_t)(count * sizeof(T));
  return ANN_OK;
}

int mode_supported(const ann_index* ix, int mode) {
  switch (mode) {
    case ANN_MODE_F32: return ix->x_f32 != nullptr;
    case ANN_MODE_F16: return ix->x_f16 != nullptr;
    case ANN_MODE_BF16: return ix->x_bf16 != nullptr;
    case ANN_MODE_FP8: return ix->x_fp8 != nullptr && ix->fp8_scale != nullptr;
    case ANN_MODE_PQ: return ix->pq_codes != nullptr;
    case ANN_MODE_SPARSE: return ix->sp_ptr != nullptr;
  }
  return 0;
}

int elem_bytes(int mode) {
  switch (mode) {
    case ANN_MODE_F32: return 4;
    case ANN_MODE_F16: case ANN_MODE_BF16: return 2;
    case ANN_MODE_FP8: return 1;
  }
  return 0;
}

bool is_dense(int mode) { return mode <= ANN_MODE_FP8; }

int default_lanes(int mode, int d) {
  if (!is_dense(mode)) return 64;
  const int nchunks = d * elem_bytes(mode) / 16;
  for (int L : {16, 32, 64})
    if (dense_shape_supported(mode, nchunks, L) && nchunks <= 4 * L && nchunks > L / 2) return L;
  return 64;
}

int validate_graph(const ann_index_desc* D) {
  const int64_t n = D->n;
  if (!D->levels || !D->adj0 || !D->upper_off) return fail(ANN_EINVAL, "graph arrays are required");
  if (D->M < 1 || D->M > 64 || D->M0 < 1 || D->M0 > 64)
    return fail(ANN_EFORMAT, "need 1 <= M <= 64 and 1 <= M0 <= 64 (M=%d M0=%d)", D->M, D->M0);
  if (D->entry_point < 0 || D->entry_point >= n)
    return fail(ANN_EFORMAT, "entry point %d outside [0, %lld)", D->entry_point, (long long)n);
  if (D->max_level < 0 || D->levels[D->entry_point] != D->max_level)
    return fail(ANN_EFORMAT, "entry point level %d != max_level %d", D->levels[D->entry_point],
                D->max_level);
  for (int64_t v = 0; v < n; ++v) {
    const int lv = D->levels[v];
    if (lv > D->max_level) return fail(ANN_EFORMAT, "node %lld above max_level", (long long)v);
    const int32_t* a = D->adj0 + v * D->M0;
    bool pad = false;
    for (int j = 0; j < D->M0; ++j) {
      if (a[j] < 0) { if (a[j] != -1) return fail(ANN_EFORMAT, "bad id in adj0"); pad = true; continue; }
      if (pad || a[j] >= n) return fail(ANN_EFORMAT, "adj0 row %lld not -1 padded or id out of range", (long long)v);
    }
    const int32_t off = D->upper_off[v];
    if (lv == 0) {
      if (off != -1) return fail(ANN_EFORMAT, "level-0 node %lld has upper lists", (long long)v);
      continue;
    }
    if (off < 0 || (int64_t)off + lv > D->n_upper_lists || !D->upper_adj)
      return fail(ANN_EFORMAT, "upper_off of node %lld out of range", (long long)v);
    for (int lc = 1; lc <= lv; ++lc) {
      const int32_t* u = D->upper_adj + ((int64_t)off + lc - 1) * D->M;
      bool upad = false;
      for (int j = 0; j < D->M; ++j) {
        if (u[j] < 0) { if (u[j] != -1) return fail(ANN_EFORMAT, "bad id in upper lists"); upad = true; continue; }
        if (upad || u[j] >= n || D->levels[u[j]] < lc)
          return fail(ANN_EFORMAT, "upper list of node %lld level %d invalid", (long long)v, lc);
      }
    }
  }
  return ANN_OK;
}

}  // namespace

namespace ann {

// Every host-side check of ann_index_create (no device involved).
int check_desc(const ann_index_desc* D) {
  if (D->n < 1 || D->n > INT32_MAX - 1) return fail(ANN_EINVAL, "n %lld outside [1, 2^31 - 2]", (long long)D->n);
  if (D->d < 1) return fail(ANN_EINVAL, "d < 1");
  if (D->metric != ANN_METRIC_L2 && D->metric != ANN_METRIC_IP) return fail(ANN_EINVAL, "unknown metric");
  const bool dense = D->x_f32 || D->x_f16 || D->x_bf16 || D->x_fp8 || D->pq_codes;
  if (dense && (D->d % 16 != 0 || D->d > 4096))
    return fail(ANN_EFORMAT, "dense rows need d %% 16 == 0 and d <= 4096 (d=%d)", D->d);
  if (D->x_fp8 && !D->fp8_scale) return fail(ANN_EINVAL, "x_fp8 without fp8_scale");
  if (D->pq_codes || D->pq_codebook) {
    if (!D->pq_codes || !D->pq_codebook || D->pq_ksub != 256 || D->pq_m < 1 || D->pq_m > 64 ||
        D->d % D->pq_m != 0)
      return fail(ANN_EFORMAT, "PQ needs codes, codebook, 256 centroids, 1 <= m <= 64, m | d");
  }
  if (D->sp_indptr) {
    if (!D->sp_ids || !D->sp_vals) return fail(ANN_EINVAL, "sparse arrays incomplete");
    if (D->metric != ANN_METRIC_IP) return fail(ANN_EFORMAT, "sparse rows support inner product only");
    if (D->sp_indptr[0] != 0) return fail(ANN_EFORMAT, "sp_indptr[0] != 0");
    for (int64_t v = 0; v < D->n; ++v)
      if (D->sp_indptr[v + 1] < D->sp_indptr[v]) return fail(ANN_EFORMAT, "sp_indptr not monotone");
    const int64_t nnz = D->sp_indptr[D->n];
    for (int64_t j = 0; j < nnz; ++j)
      if (D->sp_ids[j] >= D->d) return fail(ANN_EFORMAT, "sparse id %d >= vocabulary %d", D->sp_ids[j], D->d);
  }
  return validate_graph(D);
}

int default_waves(const ann_index* ix, const SearchParams& P);

int ensure_workspace(ann_index* ix, Workspace& ws, int64_t slots, int64_t beam_cap) {
  if (ws.slots >= slots && ws.beam_cap >= beam_cap && ws.device == ix->device) return ANN_OK;
  if (ws.done) HIP_OR_RETURN(hipEventSynchronize(ws.done), "hipEventSynchronize");
  slots = std::max(slots, ws.slots);
  beam_cap = std::max(beam_cap, ws.beam_cap);
  ws.release();
  ws.device = ix->device;
  ws.bits_words = (ix->n + 31) / 32;
  ws.vlog_cap = (int)std::max<int64_t>(256, std::min<int64_t>(ix->n / 64, 1 << 20));
  HIP_OR_RETURN(hipMalloc((void**)&ws.bits, (size_t)slots * ws.bits_words * 4), "hipMalloc (visited bits)");
  HIP_OR_RETURN(hipMemset(ws.bits, 0, (size_t)slots * ws.bits_words * 4), "hipMemset (visited bits)");
  HIP_OR_RETURN(hipMalloc((void**)&ws.vlog, (size_t)slots * ws.vlog_cap * 4), "hipMalloc (visited log)");
  HIP_OR_RETURN(hipMalloc((void**)&ws.counter, 64), "hipMalloc (counter)");
  HIP_OR_RETURN(hipEventCreateWithFlags(&ws.done, hipEventDisableTiming), "hipEventCreate");
  if (beam_cap > 0) {
    // two arrays per slot: a buffer flush writes the merged list into the other one
    HIP_OR_RETURN(hipMalloc((void**)&ws.beam_key, (size_t)slots * beam_cap * 8), "hipMalloc (beam keys)");
    HIP_OR_RETURN(hipMalloc((void**)&ws.beam_id, (size_t)slots * beam_cap * 8), "hipMalloc (beam ids)");
  }
  ws.slots = slots;
  ws.beam_cap = beam_cap;
  ws.used = false;
  ws.bytes = slots * ws.bits_words * 4 + slots * (int64_t)ws.vlog_cap * 4 + 64 + slots * beam_cap * 16;
  return ANN_OK;
}

void bind_workspace(SearchParams& P, const Workspace& ws) {
  P.bits = ws.bits;
  P.bits_words = ws.bits_words;
  P.vlog = ws.vlog;
  P.vlog_cap = ws.vlog_cap;
  P.counter = ws.counter;
  P.glist_key = ws.beam_key;
  P.glist_id = ws.beam_id;
}

// Fills the kernel parameters for a batch; checks everything on the host.
int make_params(const ann_index* ix, const ann_batch* b, SearchParams* P) {
  if (!b) return fail(ANN_EINVAL, "batch is NULL");
  const int mode = b->mode;
  if (mode < 0 || mode > ANN_MODE_SPARSE) return fail(ANN_EINVAL, "unknown mode %d", mode);
  if (!mode_supported(ix, mode)) return fail(ANN_EUNSUP, "index has no arrays for mode %d", mode);
  if (b->nq < 0) return fail(ANN_EINVAL, "nq < 0");
  if (b->k_max < 1 || b->k_max > ANN_K_MAX) return fail(ANN_EINVAL, "k_max %d outside [1, %d]", b->k_max, ANN_K_MAX);
  if (b->ef_max < 1) return fail(ANN_EINVAL, "ef_max < 1");
  if (!b->k && (b->k_all < 1 || b->k_all > b->k_max)) return fail(ANN_EINVAL, "k_all %d outside [1, k_max]", b->k_all);
  if (!b->ef && (b->ef_all < 1 || b->ef_all > b->ef_max)) return fail(ANN_EINVAL, "ef_all %d outside [1, ef_max]", b->ef_all);
  const int ef_cap = std::max(b->ef_max, b->k_max);
  if (ef_cap > ANN_EF_MAX) return fail(ANN_EBUDGET, "ef %d above ANN_EF_MAX %d", ef_cap, ANN_EF_MAX);
  if (b->rerank < 0) return fail(ANN_EINVAL, "rerank < 0");
  if (b->rerank > 0 && (!ix->x_f32 || mode == ANN_MODE_SPARSE))
    return fail(ANN_EUNSUP, "rerank needs FP32 rows of a dense index");
  if (b->nq > 0) {
    if (!b->out_ids || !b->out_dists) return fail(ANN_EINVAL, "output pointers are NULL");
    if (mode == ANN_MODE_SPARSE) {
      if (!b->q_indptr || !b->q_ids || !b->q_vals) return fail(ANN_EINVAL, "sparse query arrays are NULL");
    } else if (!b->queries) {
      return fail(ANN_EINVAL, "queries pointer is NULL");
    }
    if (b->out_visited && b->visited_cap < 1) return fail(ANN_EINVAL, "visited_cap < 1");
  }
  if (b->nq > INT32_MAX) return fail(ANN_EINVAL, "nq above 2^31 - 1");
  std::memset(P, 0, sizeof *P);
  P->debug = ix->debug;
  P->mode = mode;
  P->metric = ix->metric;
  P->d = ix->d;
  const ann_launch_cfg& cfg = ix->cfg[mode];
  if (is_dense(mode)) {
    P->nchunks = ix->d * elem_bytes(mode) / 16;
    P->lanes_per_row = cfg.lanes_per_row ? cfg.lanes_per_row : default_lanes(mode, ix->d);
    if (!dense_shape_supported(mode, P->nchunks, P->lanes_per_row))
      return fail(ANN_EBUDGET, "row of %d chunks not supported with %d lanes per row", P->nchunks,
                  P->lanes_per_row);
    P->rows = mode == ANN_MODE_F32 ? (const void*)ix->x_f32
            : mode == ANN_MODE_F16 ? (const void*)ix->x_f16
            : mode == ANN_MODE_BF16 ? (const void*)ix->x_bf16 : (const void*)ix->x_fp8;
  } else if (mode == ANN_MODE_PQ) {
    P->lanes_per_row = cfg.lanes_per_row ? cfg.lanes_per_row : 16;
  } else {
    P->lanes_per_row = 64;
  }
  P->waves_per_query = cfg.waves_per_query ? cfg.waves_per_query : 1;
  P->fp8_scale = ix->fp8_scale;
  P->pq_cb = ix->pq_cb;
  P->pq_codes = ix->pq_codes;
  P->pq_m = ix->pq_m;
  P->pq_dsub = ix->pq_m ? ix->d / ix->pq_m : 0;
  P->pq_stride = ix->pq_stride;
  P->sp_ptr = ix->sp_ptr;
  P->sp_ids = ix->sp_ids;
  P->sp_vals = ix->sp_vals;
  P->x_f32 = ix->x_f32;
  P->n = ix->n;
  P->M = ix->M;
  P->M0 = ix->M0;
  P->max_level = ix->max_level;
  P->entry = ix->entry;
  P->adj0 = ix->adj0;
  P->upper_off = ix->upper_off;
  P->upper_adj = ix->upper_adj;
  P->nq = b->nq;
  P->queries = b->queries;
  P->q_ptr = b->q_indptr;
  P->q_ids = b->q_ids;
  P->q_vals = b->q_vals;
  P->k_arr = b->k;
  P->ef_arr = b->ef;
  P->k_all = b->k_all;
  P->ef_all = b->ef_all;
  P->k_max = b->k_max;
  P->ef_cap = ef_cap;
  P->rerank = b->rerank;
  P->q_lds_floats = (b->rerank > 0 || mode == ANN_MODE_PQ) ? ((ix->d + 3) & ~3) : 0;
  P->out_ids = b->out_ids;
  P->out_dists = b->out_dists;
  P->out_status = b->out_status;
  P->out_stats = b->out_stats;
  P->out_visited = b->out_visited;
  P->visited_cap = b->visited_cap;
  // where the beam lives: its list in LDS, or (wide beams) in HBM with only
  // the insert buffer in LDS
  P->glist = cfg.beam_list == ANN_BEAM_HBM ||
             (cfg.beam_list == ANN_BEAM_AUTO && (ef_cap > kHbmListMinEf || lds_bytes(*P) > ix->lds_limit));
  if (P->glist) {
    if (cfg.beam_buffer == -1)
      return fail(ANN_EINVAL, "a beam list in HBM needs the insert buffer (beam_buffer is -1)");
    P->wbuf = cfg.beam_buffer > 0 ? cfg.beam_buffer : 1024;
    P->wbuf_min_ef = 0;
  } else if (cfg.beam_buffer > 0) {
    P->wbuf = cfg.beam_buffer;
    P->wbuf_min_ef = 0;
  } else if (cfg.beam_buffer == 0 && ef_cap > kBufferMinEf) {
    // an eighth of the beam, 128..1024 entries, halved until it fits
    int wb = 128;
    while (wb < 1024 && wb < ef_cap / 8) wb <<= 1;
    P->wbuf_min_ef = kBufferMinEf;
    for (; wb >= 64; wb >>= 1) {
      P->wbuf = wb;
      if (lds_bytes(*P) <= ix->lds_limit) break;
    }
    if (wb < 64) P->wbuf = 0;
  }
  // a beam list in HBM leaves the LDS nearly free: many queries per compute
  // unit, two waves each (measured best for wide beams)
  if (P->glist && !cfg.waves_per_query) P->waves_per_query = 2;
  if (lds_bytes(*P) > ix->lds_limit)
    return fail(ANN_EBUDGET, "on-chip memory for ef %d in mode %d: %zu bytes > %zu", ef_cap, mode,
                lds_bytes(*P), ix->lds_limit);
  if (!cfg.waves_per_query && !P->glist) P->waves_per_query = default_waves(ix, *P);
  return ANN_OK;
}

// More waves per query when the beam's LDS, not the registers, bounds how
// many queries a compute unit holds: the spare wave slots then gather rows
// for the resident queries.
int default_waves(const ann_index* ix, const SearchParams& P) {
  const void* fn = kernel_symbol(P);
  if (!fn) return 1;
  int with_lds = 0, without = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&with_lds, fn, 64, lds_bytes(P)) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&without, fn, 64, 0) != hipSuccess || with_lds < 1)
    return 1;
  (void)ix;
  const int ratio = without / with_lds;
  return ratio >= 8 ? 8 : ratio >= 4 ? 4 : ratio >= 2 ? 2 : 1;
}

int64_t pick_slots(const ann_index* ix, const SearchParams& P, int64_t requested) {
  int per_cu = 0;
  const void* fn = kernel_symbol(P);
  size_t lds = lds_bytes(P);
  if (fn && hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * P.waves_per_query, lds) !=
                hipSuccess)
    per_cu = 0;
  if (per_cu <= 0) per_cu = 4;
  int64_t slots = requested > 0 ? requested : (int64_t)ix->cu_count * per_cu;
  // bound the visited bitsets (and HBM beam lists) to 4 GiB
  const int64_t per_slot = slot_bytes(ix->n) + (P.glist ? (int64_t)P.ef_cap * 16 : 0);
  slots = std::min<int64_t>(slots, std::max<int64_t>(1, (int64_t(4) << 30) / per_slot));
  slots = std::min<int64_t>(slots, std::max<int64_t>(1, P.nq));
  return std::max<int64_t>(1, slots);
}

int run_batch(ann_index* ix, Workspace& ws, const SearchParams& P0, int64_t slots_req,
              hipStream_t st) {
  if (P0.nq == 0) return ANN_OK;
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  SearchParams P = P0;
  const int64_t slots = pick_slots(ix, P, slots_req);
  int rc = ensure_workspace(ix, ws, slots, P.glist ? P.ef_cap : 0);
  if (rc) return rc;
  if (ws.used) HIP_OR_RETURN(hipStreamWaitEvent(st, ws.done, 0), "hipStreamWaitEvent");
  bind_workspace(P, ws);
  const size_t lds = lds_bytes(P);
  if (lds > 65536) {
    const void* fn = kernel_symbol(P);
    if (fn) hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  HIP_OR_RETURN(launch_search(P, (int)slots, lds, st), "search launch");
  HIP_OR_RETURN(hipEventRecord(ws.done, st), "hipEventRecord");
  ws.used = true;
  return ANN_OK;
}

}  // namespace ann

extern "C" {

const char* ann_last_error(void) { return g_err.c_str(); }

int ann_version(void) { return 1; }

int ann_debug_flags(const ann_index* ix, uint32_t* out, int32_t clear) {
  if (!ix || !out) return fail(ANN_EINVAL, "NULL argument");
#ifdef ANN_DEBUG_CHECKS
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  HIP_OR_RETURN(hipDeviceSynchronize(), "hipDeviceSynchronize");
  HIP_OR_RETURN(hipMemcpy(out, ix->debug, sizeof(uint32_t), hipMemcpyDeviceToHost), "hipMemcpy");
  if (clear) HIP_OR_RETURN(hipMemset(ix->debug, 0, sizeof(uint32_t)), "hipMemset");
  return ANN_OK;
#else
  (void)clear;
  *out = 0;
  return fail(ANN_EUNSUP, "this library was built without ANN_DEBUG_CHECKS");
#endif
}

int ann_device_count(void) {
  int c = 0;
  if (hipGetDeviceCount(&c) != hipSuccess) return 0;
  return c;
}

int ann_index_create(const ann_index_desc* D, int device, ann_index** out) {
  if (!D || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  int rc = check_desc(D);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(ANN_ENODEV, "no GPU visible");
  if (device < 0 || device >= ndev) return fail(ANN_ENODEV, "device %d outside [0, %d)", device, ndev);
  HIP_OR_RETURN(hipSetDevice(device), "hipSetDevice");
  std::unique_ptr<ann_index> ix(new ann_index);
  ix->device = device;
  hipDeviceProp_t prop;
  HIP_OR_RETURN(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
  ix->cu_count = prop.multiProcessorCount;
  ix->lds_limit = prop.sharedMemPerBlock;
  if (prop.maxSharedMemoryPerMultiProcessor > 0)
    ix->lds_limit = std::max(ix->lds_limit, std::min<size_t>(prop.maxSharedMemoryPerMultiProcessor, 160 * 1024));
  HIP_OR_RETURN(hipStreamCreateWithFlags(&ix->stream, hipStreamNonBlocking), "hipStreamCreate");
#ifdef ANN_DEBUG_CHECKS
  HIP_OR_RETURN(hipMalloc((void**)&ix->debug, sizeof(uint32_t)), "hipMalloc");
  HIP_OR_RETURN(hipMemset(ix->debug, 0, sizeof(uint32_t)), "hipMemset");
#endif
  ix->n = D->n; ix->d = D->d; ix->metric = D->metric; ix->M = D->M; ix->M0 = D->M0;
  ix->max_level = D->max_level; ix->entry = D->entry_point; ix->n_upper_lists = D->n_upper_lists;
  const size_t n = (size_t)D->n, d = (size_t)D->d;
  int64_t* by = &ix->device_bytes;
  if ((rc = upload(&ix->adj0, D->adj0, n * D->M0, by))) return rc;
  if ((rc = upload(&ix->upper_off, D->upper_off, n, by))) return rc;
  if ((rc = upload(&ix->upper_adj, D->upper_adj, (size_t)D->n_upper_lists * D->M, by))) return rc;
  if (!ix->upper_adj) {
    // keep a valid pointer for graphs without upper layers
    HIP_OR_RETURN(hipMalloc((void**)&ix->upper_adj, 64), "hipMalloc");
  }
  if ((rc = upload(&ix->x_f32, D->x_f32, n * d, by))) return rc;
  if (D->x_f32) {
    double xmax = 0.0, x2max = 0.0;
    for (size_t v = 0; v < n; ++v) {
      double s2 = 0.0;
      for (size_t i = 0; i < d; ++i) {
        const double x = D->x_f32[v * d + i];
        xmax = std::max(xmax, std::fabs(x));
        s2 += x * x;
      }
      x2max = std::max(x2max, s2);
    }
    // rounded up so that the bounds stay bounds
    ix->xmax = (float)(xmax * (1.0 + 1e-6));
    ix->x2max = (float)(x2max * (1.0 + 1e-6));
  }
  if ((rc = upload(&ix->x_f16, D->x_f16, n * d, by))) return rc;
  if ((rc = upload(&ix->x_bf16, D->x_bf16, n * d, by))) return rc;
  if ((rc = upload(&ix->x_fp8, D->x_fp8, n * d, by))) return rc;
  if ((rc = upload(&ix->fp8_scale, D->fp8_scale, n, by))) return rc;
  if (D->pq_codes) {
    ix->pq_m = D->pq_m;
    ix->pq_stride = (D->pq_m + 15) & ~15;
    if ((rc = upload(&ix->pq_cb, D->pq_codebook, (size_t)D->pq_m * 256 * (d / D->pq_m), by))) return rc;
    std::vector<uint8_t> padded(n * ix->pq_stride, 0);
    for (size_t v = 0; v < n; ++v)
      std::memcpy(&padded[v * ix->pq_stride], D->pq_codes + v * D->pq_m, D->pq_m);
    if ((rc = upload(&ix->pq_codes, padded.data(), padded.size(), by))) return rc;
  }
  if (D->sp_indptr) {
    const size_t nnz = (size_t)D->sp_indptr[n];
    if ((rc = upload(&ix->sp_ptr, D->sp_indptr, n + 1, by))) return rc;
    // one spare element so that empty rows still have valid pointers
    std::vector<uint16_t> ids(D->sp_ids, D->sp_ids + nnz); ids.push_back(0);
    std::vector<float> vals(D->sp_vals, D->sp_vals + nnz); vals.push_back(0.f);
    if ((rc = upload(&ix->sp_ids, ids.data(), ids.size(), by))) return rc;
    if ((rc = upload(&ix->sp_vals, vals.data(), vals.size(), by))) return rc;
  }
  *out = ix.release();
  return ANN_OK;
}

int ann_index_free(ann_index* ix) {
  if (!ix) return ANN_OK;
  hipSetDevice(ix->device);
  hipDeviceSynchronize();
  ix->ws.release();
  if (ix->bf_scratch) (void)hipFree(ix->bf_scratch);
  if (ix->bf_xh) (void)hipFree(ix->bf_xh);
  if (ix->debug) (void)hipFree(ix->debug);
  if (ix->bf_done) (void)hipEventDestroy(ix->bf_done);
  void* ptrs[] = {ix->adj0, ix->upper_off, ix->upper_adj, ix->x_f32, ix->x_f16, ix->x_bf16,
                  ix->x_fp8, ix->fp8_scale, ix->pq_cb, ix->pq_codes, ix->sp_ptr, ix->sp_ids,
                  ix->sp_vals};
  for (void* p : ptrs)
    if (p) hipFree(p);
  if (ix->stream) hipStreamDestroy(ix->stream);
  delete ix;
  return ANN_OK;
}

int ann_index_info_get(const ann_index* ix, ann_info* out) { return ann_index_info(ix, out); }

int ann_index_info(const ann_index* ix, ann_info* out) {
  if (!ix || !out) return fail(ANN_EINVAL, "NULL argument");
  out->n = ix->n; out->d = ix->d; out->metric = ix->metric; out->M = ix->M; out->M0 = ix->M0;
  out->max_level = ix->max_level; out->entry_point = ix->entry;
  out->modes = 0;
  for (int m = 0; m <= ANN_MODE_SPARSE; ++m)
    if (mode_supported(ix, m)) out->modes |= 1 << m;
  out->device = ix->device;
  out->device_bytes = ix->device_bytes;
  return ANN_OK;
}

int ann_search_ex(const ann_index* cix, const ann_batch* b, void* stream) {
  if (!cix) return fail(ANN_EINVAL, "index is NULL");
  ann_index* ix = const_cast<ann_index*>(cix);
  SearchParams P;
  int rc = make_params(ix, b, &P);
  if (rc) return rc;
  if (b->nq == 0) return ANN_OK;
  std::lock_guard<std::mutex> lock(ix->mu);
  hipStream_t st = stream ? (hipStream_t)stream : ix->stream;
  rc = run_batch(ix, ix->ws, P, ix->cfg[b->mode].slots, st);
  if (rc) return rc;
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "search kernel");
  return ANN_OK;
}

int ann_search(const ann_index* ix, const float* queries, int64_t nq, int32_t k, int32_t ef,
               int64_t* out_ids, float* out_dists) {
  ann_batch b;
  std::memset(&b, 0, sizeof b);
  b.mode = ANN_MODE_F32;
  b.nq = nq;
  b.queries = queries;
  b.k_all = k; b.ef_all = std::max(ef, 1);
  b.k_max = k; b.ef_max = std::max(ef, k);
  if (k < 1) return fail(ANN_EINVAL, "k < 1");
  if (ef < 1) return fail(ANN_EINVAL, "ef < 1");
  b.out_ids = out_ids; b.out_dists = out_dists;
  return ann_search_ex(ix, &b, nullptr);
}

int ann_search_sparse(const ann_index* ix, const int64_t* q_indptr, const uint16_t* q_ids,
                      const float* q_vals, int64_t nq, int32_t k, int32_t ef,
                      int64_t* out_ids, float* out_dists) {
  ann_batch b;
  std::memset(&b, 0, sizeof b);
  b.mode = ANN_MODE_SPARSE;
  b.nq = nq;
  b.q_indptr = q_indptr; b.q_ids = q_ids; b.q_vals = q_vals;
  if (k < 1) return fail(ANN_EINVAL, "k < 1");
  if (ef < 1) return fail(ANN_EINVAL, "ef < 1");
  b.k_all = k; b.ef_all = ef; b.k_max = k; b.ef_max = std::max(ef, k);
  b.out_ids = out_ids; b.out_dists = out_dists;
  return ann_search_ex(ix, &b, nullptr);
}

int ann_set_launch(ann_index* ix, int32_t mode, const ann_launch_cfg* cfg) {
  if (!ix || !cfg) return fail(ANN_EINVAL, "NULL argument");
  if (mode < 0 || mode > ANN_MODE_SPARSE) return fail(ANN_EINVAL, "unknown mode");
  if (cfg->slots < 0) return fail(ANN_EINVAL, "slots < 0");
  if (cfg->waves_per_query != 0 && cfg->waves_per_query != 1 && cfg->waves_per_query != 2 &&
      cfg->waves_per_query != 4 && cfg->waves_per_query != 8)
    return fail(ANN_EINVAL, "waves_per_query must be 0, 1, 2, 4 or 8");
  if (cfg->beam_buffer != 0 && cfg->beam_buffer != -1 &&
      (cfg->beam_buffer < 64 || cfg->beam_buffer > 4096))
    return fail(ANN_EINVAL, "beam_buffer must be 0, -1 or in [64, 4096]");
  if (cfg->beam_list != ANN_BEAM_AUTO && cfg->beam_list != ANN_BEAM_LDS && cfg->beam_list != ANN_BEAM_HBM)
    return fail(ANN_EINVAL, "beam_list must be ANN_BEAM_AUTO, ANN_BEAM_LDS or ANN_BEAM_HBM");
  if (cfg->lanes_per_row != 0 && mode == ANN_MODE_PQ) {
    if (cfg->lanes_per_row != 16 && cfg->lanes_per_row != 32 && cfg->lanes_per_row != 64)
      return fail(ANN_EINVAL, "PQ takes 16, 32 or 64 lanes per candidate");
  } else if (cfg->lanes_per_row != 0) {
    if (!is_dense(mode)) return fail(ANN_EINVAL, "lanes_per_row applies to dense and PQ modes");
    if (!dense_shape_supported(mode, ix->d * elem_bytes(mode) / 16, cfg->lanes_per_row))
      return fail(ANN_EBUDGET, "lanes_per_row %d not supported for d=%d", cfg->lanes_per_row, ix->d);
  }
  std::lock_guard<std::mutex> lock(ix->mu);
  ix->cfg[mode] = *cfg;
  return ANN_OK;
}

int ann_get_launch(const ann_index* ix, int32_t mode, ann_launch_cfg* out) {
  if (!ix || !out) return fail(ANN_EINVAL, "NULL argument");
  if (mode < 0 || mode > ANN_MODE_SPARSE) return fail(ANN_EINVAL, "unknown mode");
  *out = ix->cfg[mode];
  if (out->lanes_per_row == 0 && is_dense(mode)) out->lanes_per_row = default_lanes(mode, ix->d);
  if (out->lanes_per_row == 0 && mode == ANN_MODE_PQ) out->lanes_per_row = 16;
  return ANN_OK;
}

int ann_autotune(ann_index* ix, const ann_batch* b, ann_launch_cfg* best) {
  if (!ix || !b) return fail(ANN_EINVAL, "NULL argument");
  SearchParams P;
  int rc = make_params(ix, b, &P);
  if (rc) return rc;
  if (b->nq == 0) return fail(ANN_EINVAL, "autotune needs a non-empty batch");
  const int mode = b->mode;
  std::lock_guard<std::mutex> lock(ix->mu);
  // events and the configuration under test are restored on every exit
  struct Guard {
    ann_index* ix;
    int mode;
    ann_launch_cfg saved;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Guard() {
      ix->cfg[mode] = saved;
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } g{ix, mode, ix->cfg[mode]};
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  HIP_OR_RETURN(hipEventCreate(&g.e0), "hipEventCreate");
  HIP_OR_RETURN(hipEventCreate(&g.e1), "hipEventCreate");
  // one warm-up run (caches, workspace growth), then one timed run
  auto time_cfg = [&](const ann_launch_cfg& c, float* ms) -> int {
    ix->cfg[mode] = c;
    SearchParams Q;
    int r = make_params(ix, b, &Q);
    if (r) return r;
    for (int rep = 0; rep < 2; ++rep) {
      HIP_OR_RETURN(hipEventRecord(g.e0, ix->stream), "hipEventRecord");
      r = run_batch(ix, ix->ws, Q, c.slots, ix->stream);
      if (r) return r;
      HIP_OR_RETURN(hipEventRecord(g.e1, ix->stream), "hipEventRecord");
      HIP_OR_RETURN(hipEventSynchronize(g.e1), "autotune run");
      HIP_OR_RETURN(hipEventElapsedTime(ms, g.e0, g.e1), "hipEventElapsedTime");
    }
    return ANN_OK;
  };
  std::vector<int> lanes;
  if (is_dense(mode)) {
    for (int L : {16, 32, 64})
      if (dense_shape_supported(mode, P.nchunks, L)) lanes.push_back(L);
  } else if (mode == ANN_MODE_PQ) {
    lanes = {16, 32, 64};
  } else {
    lanes = {0};
  }
  float best_ms = 1e30f;
  ann_launch_cfg pick = g.saved;
  // 1. lanes per row x waves per query, slots from the occupancy
  for (int L : lanes) {
    for (int nw : {1, 2, 4, 8}) {
      ann_launch_cfg c = g.saved;
      c.slots = 0;
      c.lanes_per_row = L;
      c.waves_per_query = nw;
      float ms = 0.f;
      rc = time_cfg(c, &ms);
      if (rc == ANN_EBUDGET) continue;     // this shape does not fit on chip
      if (rc) return rc;
      if (ms < best_ms) { best_ms = ms; pick = c; }
    }
  }
  if (best_ms >= 1e30f) return fail(ANN_EBUDGET, "no launch shape fits this batch");
  // 2. a wide beam's list in the other place (on chip it costs LDS, which
  //    bounds the queries per compute unit; in HBM it costs a round trip
  //    per expansion), with every waves-per-query count at the best lanes
  {
    ix->cfg[mode] = pick;
    SearchParams Q;
    if ((rc = make_params(ix, b, &Q))) return rc;
    if (Q.wbuf > 0) {
      for (int nw : {1, 2, 4, 8}) {
        ann_launch_cfg c = pick;
        c.beam_list = Q.glist ? ANN_BEAM_LDS : ANN_BEAM_HBM;
        c.waves_per_query = nw;
        float ms = 0.f;
        rc = time_cfg(c, &ms);
        if (rc == ANN_EBUDGET) continue;
        if (rc) return rc;
        if (ms < best_ms) { best_ms = ms; pick = c; }
      }
    }
  }
  // 3. the insert buffer of a wide beam: larger means rarer flushes into the
  //    sorted list but longer merges into the buffer, for the best shape
  {
    ix->cfg[mode] = pick;
    SearchParams Q;
    if ((rc = make_params(ix, b, &Q))) return rc;
    if (Q.wbuf > 0) {
      for (int wb : {Q.wbuf / 2, Q.wbuf * 2}) {
        if (wb < 64 || wb > 4096) continue;
        ann_launch_cfg c = pick;
        c.beam_buffer = wb;
        float ms = 0.f;
        rc = time_cfg(c, &ms);
        if (rc == ANN_EBUDGET) continue;
        if (rc) return rc;
        if (ms < best_ms) { best_ms = ms; pick = c; }
      }
    }
  }
  // 4. fewer slots than the occupancy allows (less contention for the
  //    caches and the memory system), for the best shape
  {
    ix->cfg[mode] = pick;
    SearchParams Q;
    if ((rc = make_params(ix, b, &Q))) return rc;
    const int64_t full = pick_slots(ix, Q, 0);
    for (int64_t sl : {full * 3 / 4, full / 2}) {
      if (sl < 1) continue;
      ann_launch_cfg c = pick;
      c.slots = (int32_t)sl;
      float ms = 0.f;
      if ((rc = time_cfg(c, &ms))) return rc;
      if (ms < best_ms) { best_ms = ms; pick = c; }
    }
  }
  g.saved = pick;   // the guard installs the winner
  if (best) *best = pick;
  return ANN_OK;
}

}  // extern "C"
