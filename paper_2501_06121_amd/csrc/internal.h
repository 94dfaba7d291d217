// Internal host-side state shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ann.h"
#include "search_kernels.h"

namespace ann {

// Sets the calling thread's error text; returns `code`.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

#define HIP_OR_RETURN(expr, what)                    \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return ::ann::hip_fail(_e, what); \
  } while (0)

// One set of per-slot scratch arrays.  A launch owns a workspace until its
// kernels finish; `done` is recorded after them so that the next user (on any
// stream) waits for it on the device.
struct Workspace {
  int device = -1;
  int64_t slots = 0;
  int64_t bits_words = 0;
  int vlog_cap = 0;
  uint32_t* bits = nullptr;
  int32_t* vlog = nullptr;
  int32_t* counter = nullptr;
  int64_t beam_cap = 0;              // beam-list entries per slot held in HBM
  float* beam_key = nullptr;
  uint32_t* beam_id = nullptr;
  hipEvent_t done = nullptr;
  bool used = false;
  int64_t bytes = 0;
  void release();
};

// Bytes of one slot's visited bitset and log for an index of n nodes.
int64_t slot_bytes(int64_t n);

}  // namespace ann

struct ann_index {
  int device = 0;
  int cu_count = 0;
  size_t lds_limit = 65536;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  int d = 0, metric = 0, M = 0, M0 = 0, max_level = 0, entry = 0;
  int64_t n_upper_lists = 0;
  int32_t* adj0 = nullptr;
  int32_t* upper_off = nullptr;
  int32_t* upper_adj = nullptr;
  float* x_f32 = nullptr;
  uint16_t* x_f16 = nullptr;
  uint16_t* x_bf16 = nullptr;
  uint8_t* x_fp8 = nullptr;
  float* fp8_scale = nullptr;
  float* pq_cb = nullptr;
  uint8_t* pq_codes = nullptr;
  int pq_m = 0, pq_stride = 0;
  int64_t* sp_ptr = nullptr;
  uint16_t* sp_ids = nullptr;
  float* sp_vals = nullptr;
  int64_t device_bytes = 0;
  float xmax = 0.f;                  // max |x_ij| of the FP32 rows
  float x2max = 0.f;                 // max squared row norm
  void* bf_scratch = nullptr;        // brute-force candidates and row norms
  size_t bf_scratch_bytes = 0;
  bool bf_norms_ready = false;
  hipEvent_t bf_done = nullptr;      // recorded after the last brute-force call's kernels
  bool bf_used = false;
  void* bf_xh = nullptr;             // the rows' FP16 copy for the half-precision brute-force pass
  uint32_t* debug = nullptr;         // ANN_DEBUG_CHECKS builds: the kernels' invariant-violation bits
  ann_launch_cfg cfg[6] = {};
  std::mutex mu;
  ann::Workspace ws;                 // used by ann_search / ann_search_ex
};

namespace ann {

// Every host-side check ann_index_create makes on a description (array
// sizes, graph validity); no device is touched.
int check_desc(const ann_index_desc* D);
// Kernel parameters for a batch; every argument is checked on the host.
int make_params(const ann_index* ix, const ann_batch* b, SearchParams* P);
// Allocates (or grows) a workspace for `slots` slots, with room for beam
// lists of `beam_cap` entries per slot in HBM (0: none).
int ensure_workspace(ann_index* ix, Workspace& ws, int64_t slots, int64_t beam_cap);
// Points the kernel parameters at a workspace's arrays.
void bind_workspace(SearchParams& P, const Workspace& ws);
// Launches one batch with workspace `ws` on stream `st` (asynchronous).
// slots_req = 0 picks the default (occupancy x CUs, bounded by memory).
int run_batch(ann_index* ix, Workspace& ws, const SearchParams& P, int64_t slots_req,
              hipStream_t st);
// The slot count run_batch would use.
int64_t pick_slots(const ann_index* ix, const SearchParams& P, int64_t requested);

}  // namespace ann
