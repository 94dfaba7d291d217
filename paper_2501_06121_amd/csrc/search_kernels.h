// Internal interface between the C-ABI host code and the search kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ann {

enum { MODE_F32 = 0, MODE_F16 = 1, MODE_BF16 = 2, MODE_FP8 = 3, MODE_PQ = 4, MODE_SPARSE = 5 };
enum { METRIC_L2 = 0, METRIC_IP = 1 };

// Request ring of a server (ring.cap > 0): the persistent kernel's
// workgroups claim requests one at a time, in publication order, from a ring
// in host memory instead of taking queries from a batch.  The host writes an
// entry (query, k, ef), then publishes it by raising *host_tail; one waiting
// workgroup at a time copies *host_tail into *mirror every poll_ticks, the
// others read the mirror (device memory), and a workgroup claims request
// `seq` by advancing *head from seq to seq + 1.  When a request is done its
// results are in host memory and done[seq % cap] = seq + 1.
// The kernel ends as a whole, never one workgroup at a time (that would
// leave fewer slots for the requests still to come): when nothing has been
// claimed or published for idle_ticks (or idle_spins waits) and no request
// is in flight, a waiting workgroup sets kRingDrain in *head, after which no
// claim can succeed (claims and the drain are compare-and-swaps of the same
// word) and every workgroup leaves; the host clears the bit before it
// launches the kernel again.  *host_stop ends it at
// once for the workgroups that are waiting: the poller that sees it sets
// kRingStop in *head.
// Waiting workgroups look at the claim word and the mirror (two relaxed
// loads; an acquire would invalidate the L2) and back off from about 7 to
// about 220 us between looks while nothing arrives: hundreds of idle slots
// reading the same few control words would otherwise load the memory channel
// that holds them, under the busy slots' row gathers (measured: service
// times twice as long at half load as at full load before the backoff).
// Requests are spread over the compute units: workgroup b belongs to tier
// b / tier_width (tier_width = the compute units, so the dispatch that hands
// consecutive workgroups to different compute units puts one workgroup of
// each tier on each), and a workgroup claims only when no workgroup of a
// lower tier is waiting.  Without that the slots that have just finished a
// request (and look most often) take the next ones, and the requests pile up
// on a few compute units.
constexpr uint64_t kRingDrain = 1ull << 63;
constexpr uint64_t kRingStop = 1ull << 62;
constexpr uint64_t kRingFlags = kRingDrain | kRingStop;
constexpr int kRingTiers = 8;

struct RingArgs {
  int64_t cap;                      // entries; 0: no ring (batch mode)
  const uint64_t* host_tail;        // host memory: requests published
  const uint32_t* host_stop;        // host memory: nonzero asks the kernel to end
  uint64_t* head;                   // device: requests claimed | kRingDrain | kRingStop
  uint64_t* mirror;                 // device: the last host_tail read
  uint64_t* last_poll;              // device: clock of the last read of host_tail
  uint64_t* activity;               // device: clock of the last claim or new tail
  uint32_t* busy;                   // device: requests claimed (or being claimed), not done
  uint32_t* waiting;                // device [kRingTiers]: workgroups of each tier waiting
  int32_t tier_width;               // workgroups per tier (the last tier takes the rest)
  // the entries in host memory: read and written with system-scope atomic
  // loads and stores (coherent per access, so no fence has to invalidate or
  // write back a whole cache); the search itself runs on a per-workgroup copy
  // in device memory (SearchParams queries / k_arr / ef_arr / out_*, indexed
  // by the workgroup)
  const float* e_query;             // [cap][d]
  const int32_t* e_k;               // [cap]
  const int32_t* e_ef;              // [cap]
  int64_t* e_ids;                   // [cap][k_max]
  float* e_dists;                   // [cap][k_max]
  int32_t* e_status;                // [cap]
  uint64_t* done;                   // host memory [cap]: seq + 1 once request seq is done
  uint64_t* t_start;                // host memory [cap]: device clock at claim
  uint64_t* t_done;                 // host memory [cap]: device clock at completion
  int32_t* served_by;               // host memory [cap]: the workgroup that served it
  uint64_t idle_ticks, poll_ticks;  // device clock ticks
  int64_t idle_spins;               // the idle bound counted in waits (at least 6.8 us each)
};

// Clears the drain bit and restarts the idle clock before the server's
// kernel is launched again (one thread).
void ring_rearm(const RingArgs& r, hipStream_t st);

struct SearchParams {
  int mode, metric;
  int d, nchunks, lanes_per_row;
  int waves_per_query;              // wavefronts of one workgroup (1, 2 or 4)
  // representation searched
  const void* rows;
  const float* fp8_scale;
  const float* pq_cb;
  const uint8_t* pq_codes;
  int pq_m, pq_dsub, pq_stride;
  const int64_t* sp_ptr;
  const uint16_t* sp_ids;
  const float* sp_vals;
  const float* x_f32;               // rerank rows
  // graph
  int64_t n;
  int M, M0, max_level, entry;
  const int32_t* adj0;
  const int32_t* upper_off;
  const int32_t* upper_adj;
  // batch (nq_dev, when set, holds the query count on the device and
  // overrides nq, so that a captured launch can serve batches of any size)
  int64_t nq;
  const int32_t* nq_dev;
  const float* queries;
  const int64_t* q_ptr;
  const uint16_t* q_ids;
  const float* q_vals;
  const int32_t* k_arr;
  const int32_t* ef_arr;
  int k_all, ef_all, k_max, ef_cap, rerank;
  int q_lds_floats;
  int wbuf;                         // insert-buffer entries of a large beam (0: none)
  int wbuf_min_ef;                  // queries with ef above this use the buffer
  int glist;                        // beam list in HBM (glist_key/glist_id) instead of LDS
  float* glist_key;                 // [slots][2][ef_cap] (two arrays per slot)
  uint32_t* glist_id;               // [slots][2][ef_cap]
  int64_t* out_ids;
  float* out_dists;
  int32_t* out_status;
  int32_t* out_stats;
  int32_t* out_visited;
  int64_t visited_cap;
  // workspace
  uint32_t* bits;
  int64_t bits_words;
  int32_t* vlog;
  int vlog_cap;
  int32_t* counter;
  RingArgs ring;
  uint32_t* debug;       // builds with ANN_DEBUG_CHECKS: invariant violations (bits), else unused
};

// Entries of the sparse query's hash table in LDS (at most half filled).
constexpr int kSparseHashSlots = 512;
// Entries of a beam list's tail that each wave copies to LDS when the list is in HBM.
constexpr int kListTailCache = 256;

// Rerank keys held at once: R_eff <= min(max(R, k_max), ef_cap).
__host__ __device__ inline int rerank_slots(const SearchParams& p) {
  if (p.rerank <= 0) return 0;
  const int r = p.rerank > p.k_max ? p.rerank : p.k_max;
  return r < p.ef_cap ? r : p.ef_cap;
}

hipError_t launch_search(const SearchParams& p, int slots, size_t lds, hipStream_t st);
size_t lds_bytes(const SearchParams& p);
const void* kernel_symbol(const SearchParams& p);
bool dense_shape_supported(int mode, int nchunks, int lanes_per_row);

// kernel of a batch, one function per storage mode (search_<mode>.hip)
const void* symbol_f32(const SearchParams& p);
const void* symbol_f16(const SearchParams& p);
const void* symbol_bf16(const SearchParams& p);
const void* symbol_fp8(const SearchParams& p);
const void* symbol_pq(const SearchParams& p);
const void* symbol_sparse(const SearchParams& p);


}  // namespace ann
