// Internal interface between the C-ABI host code and the search kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ann {

enum { MODE_F32 = 0, MODE_F16 = 1, MODE_BF16 = 2, MODE_FP8 = 3, MODE_PQ = 4, MODE_SPARSE = 5 };
enum { METRIC_L2 = 0, METRIC_IP = 1 };

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
