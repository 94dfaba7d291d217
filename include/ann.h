/*
 * ann.h -- C interface of the MI355X (gfx950) batched HNSW search library.
 *
 * The library answers k-nearest-neighbour queries over a dataset of
 * d-dimensional vectors (arXiv 2501.06121, Section 1) with the HNSW index
 * (Section 2: "The indexing method currently implemented ... is HNSW"):
 * a greedy descent through the upper layers, then an ef-wide beam search on
 * layer 0, over one of these representations:
 *   - dense FP32 rows (the Identity quantizer, Section 2), or FP16, BF16 or
 *     FP8-E4M3 (per-row scale) storage copies, with FP32 arithmetic;
 *   - Product Quantization codes with asymmetric distances from per-query
 *     lookup tables (Section 2: "Product Quantization");
 *   - sparse vectors (Section 3, Table 1: the sparse dataset, inner product).
 * The graph is always one built on the original vectors (Section 3.1,
 * "Performance": the graph is built on the original representations, not on
 * the quantized ones); the library only searches it.
 *
 * Keys ("distances", smaller is better): squared L2, or the negated inner
 * product.  Ties are broken by the id: results are ordered by (key, id).
 *
 * Arithmetic order.  Every key is evaluated in one fixed FP32 order, so a
 * result does not depend on the launch shape: 64 partial sums start at +0;
 * element i belongs to chunk i / c (c = 16 bytes / element size: FP32 4,
 * FP16 and BF16 8, FP8 16; sparse: c = 1 over the document's stored
 * positions); chunk g feeds partial g mod 64 with one fused multiply-add per
 * element in ascending i (L2: the difference is rounded first, then squared
 * by the fma); the partials are then folded as p[l] += p[l ^ s] for
 * s = 32, 16, 8, 4, 2, 1 and the key is +-p[0].  PQ: each lookup-table entry
 * is one ascending fma chain over its subvector, and the per-subspace entries
 * are folded by the same tree.  FP8: the IP key is -(scale * p[0]); the L2
 * key squares q_i - fl(scale * x_i).
 *
 * Conventions for every entry point:
 *   - Return value: ANN_OK (0) or one of the ANN_E* codes; the text of the
 *     last error of the calling thread is in ann_last_error().
 *   - Pointers documented as "device" are HIP device pointers (for example
 *     torch tensor data pointers); "host" pointers are ordinary memory.  The
 *     library never keeps a caller pointer after a call returns, except that
 *     asynchronous calls read and write the device buffers until the stream
 *     reaches the call's completion.
 *   - nq == 0 is a successful no-op.  Invalid arguments are detected on the
 *     host before anything is launched.
 */
#ifndef ANN_H_
#define ANN_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define ANN_OK 0
#define ANN_EINVAL 1   /* bad argument: null pointer, k < 1, ef < 1, sizes */
#define ANN_ENODEV 2   /* no usable GPU / bad device ordinal */
#define ANN_ENOMEM 3   /* device allocation failed */
#define ANN_EBUDGET 4  /* request beyond a compiled or configured capacity */
#define ANN_EFORMAT 5  /* malformed index description or index file (graph, arrays, checksums) */
#define ANN_EHIP 6     /* HIP runtime error; text in ann_last_error() */
#define ANN_EUNSUP 7   /* the index lacks the arrays the requested mode needs */
#define ANN_EAGAIN 8   /* serving queue full, try again later */

/* ---- enums ------------------------------------------------------------- */
enum ann_metric { ANN_METRIC_L2 = 0, ANN_METRIC_IP = 1 };

enum ann_mode {
  ANN_MODE_F32 = 0,    /* FP32 rows */
  ANN_MODE_F16 = 1,    /* FP16 rows, FP32 arithmetic */
  ANN_MODE_BF16 = 2,   /* BF16 rows, FP32 arithmetic */
  ANN_MODE_FP8 = 3,    /* OCP E4M3 rows with one FP32 scale per row */
  ANN_MODE_PQ = 4,     /* PQ codes, per-query lookup tables */
  ANN_MODE_SPARSE = 5  /* sparse rows (CSR), inner product */
};

/* Largest ef (after ef_eff = max(ef, k)) one search can use.  A beam costs 8
 * bytes per entry: in on-chip memory (LDS, 160 KB per compute unit) up to
 * about 20,000 entries fit, wider beams keep their sorted list in device
 * memory (see ann_launch_cfg.beam_list).  Larger requests fail with
 * ANN_EBUDGET, as do requests whose on-chip footprint (beam list when in LDS,
 * insert buffer, rerank keys, PQ table) exceeds the LDS. */
#define ANN_EF_MAX 65536
/* Largest k and largest rerank depth. */
#define ANN_K_MAX 1024

/* ---- index ------------------------------------------------------------- */

/*
 * Everything the library needs to search, as HOST arrays.  The library
 * copies them to the device at ann_index_create(); the caller may free them
 * afterwards.  Arrays a mode does not use may be NULL.
 *
 * Graph (HNSW, Section 2 and its citation): n nodes, level[v] in 0..max_level,
 * layer 0 lists of at most M0 ids, upper-layer lists of at most M ids.
 *   levels      u8[n]
 *   adj0        i32[n][M0]   layer-0 neighbours, valid ids first, then -1
 *   upper_off   i32[n]       for level[v] >= 1: index (in lists) of v's
 *                            level-1 list in upper_adj, its levels 2..level[v]
 *                            lists follow; -1 for level-0 nodes
 *   upper_adj   i32[n_upper_lists][M]   -1 padded
 *   entry_point the node searched first, level[entry_point] == max_level
 * Dense rows (row-major, n x d; d a multiple of 16):
 *   x_f32 f32, x_f16 / x_bf16 u16 bit patterns, x_fp8 u8 E4M3 codes with
 *   fp8_scale f32[n].
 * PQ (pq_m subspaces of d / pq_m contiguous dimensions, 256 centroids):
 *   pq_codebook f32[pq_m][256][d / pq_m], pq_codes u8[n][pq_m]; pq_m <= 64.
 * Sparse (CSR over a vocabulary of `d` terms, ids strictly increasing per row):
 *   sp_indptr i64[n + 1], sp_ids u16[nnz], sp_vals f32[nnz].
 */
typedef struct ann_index_desc {
  int64_t n;
  int32_t d;
  int32_t metric;       /* enum ann_metric; sparse requires ANN_METRIC_IP */
  int32_t M;
  int32_t M0;           /* <= 64 */
  int32_t max_level;
  int32_t entry_point;
  int64_t n_upper_lists;
  const uint8_t* levels;
  const int32_t* adj0;
  const int32_t* upper_off;
  const int32_t* upper_adj;
  const float* x_f32;
  const uint16_t* x_f16;
  const uint16_t* x_bf16;
  const uint8_t* x_fp8;
  const float* fp8_scale;
  int32_t pq_m;
  int32_t pq_ksub;      /* must be 256 when PQ arrays are given */
  const float* pq_codebook;
  const uint8_t* pq_codes;
  const int64_t* sp_indptr;
  const uint16_t* sp_ids;
  const float* sp_vals;
} ann_index_desc;

typedef struct ann_index ann_index; /* opaque, device-resident */

/* Validates `desc`, allocates device memory on GPU `device`, copies every
 * given array and returns the handle in *out.  The graph is checked on the
 * host (ids in range, lists -1 padded, entry point at max_level):
 * ANN_EFORMAT if not.  ANN_ENOMEM if the device is out of memory. */
int ann_index_create(const ann_index_desc* desc, int device, ann_index** out);

/* Frees the index and its device memory (waits for the device first). */
int ann_index_free(ann_index* ix);

/* What an index (or an index file) holds. */
typedef struct ann_info {
  int64_t n;
  int32_t d, metric, M, M0, max_level, entry_point;
  int32_t modes;       /* bit (1 << mode) set for every searchable mode */
  int32_t device;      /* -1 for a file */
  int64_t device_bytes;  /* device memory of the index (of a file: of its arrays) */
} ann_info;

int ann_index_info(const ann_index* ix, ann_info* out);
/* The same, under the name of an earlier version of this header. */
int ann_index_info_get(const ann_index* ix, ann_info* out);

/* ---- index files --------------------------------------------------------- */

/*
 * One file holds everything an ann_index_desc describes: the graph and every
 * stored representation (the Dataset component of the paper, Section 2 and
 * Figure 1: the data an index is built over and searched with).  Version 1,
 * little-endian:
 *
 *   header, bytes 0..127
 *      0  u8[8]  magic "ANNINDEX"
 *      8  u32    version (1)
 *     12  u32    section count S (1..14)
 *     16  i64    n
 *     24  i32    d                 28  i32  metric
 *     32  i32    M                 36  i32  M0
 *     40  i32    max_level         44  i32  entry_point
 *     48  i64    n_upper_lists
 *     56  i32    pq_m (0: no PQ)   60  i32  pq_ksub (0 or 256)
 *     64  i64    nnz (sparse nonzeros; 0: no sparse rows)
 *     72  u8[52] zero
 *    124  u32    CRC-32 of bytes 0..123
 *   section table, bytes 128 .. 128 + 32 S, one entry per section:
 *      0  u32 id   4  u32 CRC-32 of the section's bytes
 *      8  u64 offset (from the start of the file)   16  u64 size   24  u64 zero
 *   then a u32 CRC-32 of the table's 32 S bytes.
 *   sections, in ascending id, each starting at the first multiple of 64 at
 *   or after the end of what precedes it (zero bytes in between); the file
 *   ends with the last section.
 *
 *   id  section       type, size            id  section       type, size
 *    1  levels        u8[n]                  8  x_fp8         u8[n][d]
 *    2  adj0          i32[n][M0]             9  fp8_scale     f32[n]
 *    3  upper_off     i32[n]                10  pq_codebook   f32[pq_m][256][d/pq_m]
 *    4  upper_adj     i32[n_upper_lists][M] 11  pq_codes      u8[n][pq_m]
 *    5  x_f32         f32[n][d]             12  sp_indptr     i64[n + 1]
 *    6  x_f16         u16[n][d]             13  sp_ids        u16[nnz]
 *    7  x_bf16        u16[n][d]             14  sp_vals       f32[nnz]
 *   Sections 1-3 are required, 4 iff n_upper_lists > 0; 8 and 9 go together,
 *   10 and 11 iff pq_m > 0, 12-14 iff nnz > 0.  The arrays have the layout
 *   and meaning of the ann_index_desc fields of the same names.  CRC-32 is
 *   the IEEE 802.3 one (reflected polynomial 0xEDB88320, initial value and
 *   final xor 0xFFFFFFFF; "123456789" gives 0xCBF43926).
 *
 * ann_index_file_info reads and checks a file on the host only (no GPU):
 * magic, version, every CRC, the section table (known ids, ascending,
 * aligned, non-overlapping, inside the file, the sizes above, the required
 * and paired sections) and then every check of ann_index_create on the
 * arrays.  Returns ANN_EFORMAT with the reason in ann_last_error() for a
 * file that fails any of them (corrupt, truncated, another version),
 * ANN_EINVAL if the file cannot be opened.  On success *out describes the
 * file (device = -1).
 *
 * ann_index_load does the same checks, then ann_index_create with the file's
 * arrays on GPU `device` (ANN_ENODEV without one).  The file is mapped, not
 * copied, on the host.
 *
 * ann_index_save writes the arrays of a description to `path` in this
 * format (after the checks of ann_index_create; ANN_EINVAL if the file
 * cannot be written).  Host only.
 */
int ann_index_file_info(const char* path, ann_info* out);
int ann_index_load(const char* path, int device, ann_index** out);
int ann_index_save(const ann_index_desc* desc, const char* path);

/* ---- search ------------------------------------------------------------ */

/*
 * HNSW search (the citation's Algorithm 5: greedy descent on layers
 * max_level..1, then the ef-wide beam on layer 0), FP32 rows, one k and one
 * ef for every query, on the index's own stream; returns when done.
 *   queries    device f32[nq][d]
 *   out_ids    device i64[nq][k]   ascending (key, id); -1 when fewer than k
 *                                  nodes were reached
 *   out_dists  device f32[nq][k]   the keys; +inf with id -1
 * ef_eff = max(ef, k) must not exceed ANN_EF_MAX (ANN_EBUDGET).
 */
int ann_search(const ann_index* ix, const float* queries, int64_t nq, int32_t k, int32_t ef,
               int64_t* out_ids, float* out_dists);

/*
 * A batch with per-query k and ef, a representation and an optional exact
 * rerank, asynchronous on `stream` (a hipStream_t; NULL = the index's own
 * stream, and then the call waits for completion).
 *
 *   mode           enum ann_mode of the traversal keys
 *   rerank         R >= 0.  If R > 0, the first R_eff = min(max(R, k), |W|)
 *                  entries of the final layer-0 beam W are re-scored with the
 *                  FP32 rows in the fixed FP32 order above, re-sorted by
 *                  (key, id) and the first k returned.  Needs x_f32.
 *   queries        device f32[nq][d] (dense and PQ modes)
 *   q_indptr, q_ids, q_vals   device CSR of the sparse queries (sparse mode):
 *                  i64[nq + 1], u16, f32; ids strictly increasing per query.
 *                  The device keeps at most 256 nonzeros of a query (in an
 *                  LDS hash table); a longer query is cut to its first 256
 *                  and flagged in out_status (bit 1)
 *   k, ef          device i32[nq] per-query values, or NULL to use k_all /
 *                  ef_all for every query
 *   k_max, ef_max  host-side upper bounds of the per-query values (they size
 *                  on-chip memory and the output rows); a query whose k or ef
 *                  exceeds them is clamped and flagged in out_status
 *   out_ids        device i64[nq][k_max]; columns >= k of a row are -1
 *   out_dists      device f32[nq][k_max]; +inf where the id is -1
 *   out_status     optional device i32[nq], bit flags (0 = ok): bit 0 (1) =
 *                  k or ef clamped to k_max / ef_max; bit 1 (2) = a sparse
 *                  query with more than 256 nonzeros was searched with its
 *                  first 256 (by position) only
 *   out_stats      optional device i32[nq][4]: distance evaluations (all
 *                  layers), layer-0 expansions, layer-0 visited count, |W|
 *   out_visited    optional device i32[nq][visited_cap]: the layer-0 visited
 *                  ids in the order they were first reached (-1 padded,
 *                  truncated to visited_cap); for testing
 */
typedef struct ann_batch {
  int32_t mode;
  int32_t rerank;
  int64_t nq;
  const float* queries;
  const int64_t* q_indptr;
  const uint16_t* q_ids;
  const float* q_vals;
  const int32_t* k;
  const int32_t* ef;
  int32_t k_all, ef_all;
  int32_t k_max, ef_max;
  int64_t* out_ids;
  float* out_dists;
  int32_t* out_status;
  int32_t* out_stats;
  int32_t* out_visited;
  int64_t visited_cap;
} ann_batch;

int ann_search_ex(const ann_index* ix, const ann_batch* b, void* stream);

/* Sparse convenience form of ann_search_ex (mode ANN_MODE_SPARSE), blocking. */
int ann_search_sparse(const ann_index* ix, const int64_t* q_indptr, const uint16_t* q_ids,
                      const float* q_vals, int64_t nq, int32_t k, int32_t ef,
                      int64_t* out_ids, float* out_dists);

/* ---- launch configuration ------------------------------------------------ */

/*
 * The traversal kernel is persistent: `slots` workgroups pull query indices
 * from a device counter, one query per workgroup at a time.  A workgroup has
 * waves_per_query wavefronts (1, 2, 4 or 8): they share the query's beam in
 * LDS, split the row gathers of each expansion and merge new entries into the
 * beam together, so a large beam (whose LDS limits the queries per compute
 * unit) still keeps many rows in flight.
 * lanes_per_row (16, 32 or 64) is how many lanes evaluate one dense row
 * together, or, in PQ mode, one candidate of a short run (each lane looks
 * up 64 / lanes_per_row of its table entries; default 16).  beam_buffer is the capacity of the sorted insert buffer that a
 * large beam uses in front of its sorted list (new entries are merged into
 * the buffer, the buffer into the list only when it fills): 0 lets the
 * library decide (queries with ef above 1024 use one sized from ef and the
 * free LDS), -1 turns it off, and a value in [64, 4096] makes every query use
 * a buffer of that size.  Zeros select the built-in defaults (or the
 * autotuned values, once ann_autotune has run).  Results do not depend on
 * these settings.
 * beam_list says where the beam's sorted list lives: ANN_BEAM_LDS (on chip,
 * which bounds ef by the LDS size and the queries per compute unit by the
 * beam's footprint), ANN_BEAM_HBM (a per-slot array in device memory; only
 * the insert buffer stays in LDS, so wide beams keep several queries per
 * compute unit and ef may reach ANN_EF_MAX), or ANN_BEAM_AUTO (HBM for ef
 * above 4096 or when the list does not fit in LDS).
 */
#define ANN_BEAM_AUTO 0
#define ANN_BEAM_LDS 1
#define ANN_BEAM_HBM 2

typedef struct ann_launch_cfg {
  int32_t slots;
  int32_t lanes_per_row;
  int32_t waves_per_query;
  int32_t beam_buffer;
  int32_t beam_list;
} ann_launch_cfg;

int ann_set_launch(ann_index* ix, int32_t mode, const ann_launch_cfg* cfg);
int ann_get_launch(const ann_index* ix, int32_t mode, ann_launch_cfg* out);

/*
 * Times candidate launch shapes on the given batch (as for ann_search_ex;
 * the outputs are written by every run) on the index stream and keeps the
 * fastest for b->mode: lanes per row (16 / 32 / 64 where the mode supports
 * them) x waves per query (1 / 2 / 4 / 8) with slots from the occupancy;
 * then, for a wide beam (one with an insert buffer), its list in the other
 * place (LDS or HBM) at every waves-per-query count, and half and twice
 * the insert buffer of the best shape; then 3/4 and 1/2 of its slots.  Each
 * candidate runs twice and the second run is timed.  Shapes whose on-chip
 * memory does not fit are skipped.
 * Results are identical for every shape (the arithmetic order is fixed);
 * only speed differs.  The chosen configuration is written to *best when not
 * NULL.  Blocking; ANN_EBUDGET if no shape fits.
 */
int ann_autotune(ann_index* ix, const ann_batch* b, ann_launch_cfg* best);

/* ---- captured batches (HIP graphs) ---------------------------------------- */

/*
 * A plan records one batch shape as a HIP graph: the same search as
 * ann_search_ex, with the buffers of `b` fixed (queries, per-query k / ef
 * arrays, outputs) and the number of queries of each replay read from
 * device memory at *nq_dev when the replay runs (values outside [0, b->nq]
 * are clamped to it).  The caller refills the fixed buffers and *nq_dev on
 * the device between replays; a serving loop then costs one graph launch per
 * batch and no host-side argument work.  For callers that replay the same
 * batch shape many times (the paper's one-query-at-a-time search, Section 3,
 * batched for a GPU).
 *   b        as for ann_search_ex; b->nq is the capacity (>= 1); the launch
 *            shape is the index's current one for b->mode (ann_set_launch,
 *            ann_autotune) and stays fixed in the plan
 *   nq_dev   device i32: the batch size of each replay
 *   out      the plan.  It owns its own workspace (visited bitsets, beam
 *            lists), so replays never share scratch memory with other calls;
 *            replays of one plan run one after the other on the device
 *            whatever streams they use.
 * ann_plan_launch replays the graph on `stream` (NULL: the index stream,
 * and the call waits).  ann_plan_info gives the recorded launch shape (slots
 * resolved).  ann_plan_free waits for the last replay and frees the plan;
 * the index must outlive its plans.  Results equal ann_search_ex's for the
 * same queries bit for bit.  Errors as for ann_search_ex.
 */
typedef struct ann_plan ann_plan;
int ann_plan_create(const ann_index* ix, const ann_batch* b, const int32_t* nq_dev, ann_plan** out);
int ann_plan_launch(ann_plan* plan, void* stream);
int ann_plan_info(const ann_plan* plan, ann_launch_cfg* out);
int ann_plan_free(ann_plan* plan);

/* ---- exact search on matrix cores ---------------------------------------- */

/*
 * Exact k-NN by a full scan (the k-nearest-neighbour problem of Section 1),
 * for ground truth.  Matrix-core tiles of Q x X^T preselect 64 candidates per
 * query and row range; the best k + 16 are then re-scored with the FP32 rows
 * in the fixed FP32 order above and sorted by (key, id).  The preselection
 * runs first on FP16 copies of the rows and queries (v_mfma_f32_16x16x32_f16;
 * the rows' copy, 2 n d bytes, is made on the first call and kept by the
 * index) when d is a multiple of 8 and every row value is inside the FP16
 * range; queries whose result that pass cannot certify are scanned again
 * with FP32 tiles (v_mfma_f32_16x16x4_f32), which is also the only pass
 * otherwise.  Either way a certified result is the exact top-k.
 *   queries        device f32[nq][d]
 *   out_ids        device i64[nq][k], out_dists device f32[nq][k]
 *   out_certified  optional device i32[nq]: nonzero when the result is
 *                  provably the exact top-k under the fixed-order keys (the
 *                  gap to every candidate not re-scored exceeds the worst-
 *                  case difference between the preselection's and the
 *                  fixed-order keys): 2 when the FP16 pass certified it, 1
 *                  when the FP32 pass did; else 0
 * 1 <= k <= 48.  Needs x_f32.  Asynchronous on `stream` (NULL: the index
 * stream, blocking).  Uses a scratch buffer the index keeps (grown on
 * demand): the kernels of calls on one index run one call after the other
 * on the device, whatever streams the calls use (each call's stream waits
 * for an event recorded after the previous call's kernels).
 */
int ann_bruteforce(const ann_index* ix, const float* queries, int64_t nq, int32_t k,
                   int64_t* out_ids, float* out_dists, int32_t* out_certified, void* stream);

/*
 * ann_bruteforce with no device allocation, for callers that cannot
 * allocate memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and errors as
 * ann_bruteforce, and the same ids and keys, bit for bit, for every query
 * that both certify; it runs the FP32 tiles only (out_certified 0 or 1),
 * since the rows' FP16 copy would be an allocation.  Its scratch (the row norms and the candidate
 * lists: 4 n + 512 nq r bytes, each rounded up to 256, where r is the
 * number of row ranges the scan splits the rows into, at most 32) lives in
 * a fixed device array of ANN_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends; a call whose scratch would
 * not fit returns ANN_EBUDGET (split the batch).  Every call on one GPU
 * uses that GPU's one array: calls that overlap on a GPU (other streams,
 * other threads, other indexes) race and must be ordered by the caller.
 */
#define ANN_NOALLOC_SCRATCH_BYTES (32 << 20)
int ann_bruteforce_noalloc(const ann_index* ix, const float* queries, int64_t nq, int32_t k,
                           int64_t* out_ids, float* out_dists, int32_t* out_certified, void* stream);

/* ---- HNSW construction on the device ------------------------------------- */

/*
 * Builds the HNSW graph (the paper's index, Section 2, built as its
 * citation's Algorithms 1 and 4 describe) over dense FP32 rows, with every
 * key in the fixed FP32 order above.  Levels: l_i = min(floor(-ln(1 - u_i) /
 * ln M), 30).  Nodes are inserted in batches: the first seq_prefix one at a
 * time, then batches of max(1, min(batch_cap, floor(done * batch_frac)))
 * (batch_frac = 0: one at a time throughout).  Every node of a batch searches
 * the graph as it was before the batch: greedy descent (ef = 1) down to its
 * level, then on each layer from min(max level, l_i) to 0 a beam search of
 * width efc from the previous layer's result, whose best entries are thinned
 * by the neighbour heuristic (keep a candidate iff it is strictly closer to
 * the new node than to every kept one; M per layer, layer 0 included).  Then
 * the batch's reverse links are added, grouped by (target, layer) with the
 * sources in node order; a list that would exceed 2M entries (layer 0) or M
 * (above) is sorted by key to its node and cut back by the same heuristic.
 *   X          device f32[n][d], d a multiple of 4, at most 1024
 *   u          host f64[n] level uniforms in [0, 1)
 *   M          2..32 (layer 0 keeps up to 2M)
 *   efc        1..4096
 *   out        receives a host-side graph; read it with ann_graph_info
 *              (n, M, 2M, max level, entry point, number of upper lists)
 *              and ann_graph_export (the layout of ann_index_desc), free it
 *              with ann_graph_free.
 * Synchronizes `stream` (NULL: the null stream).  Allocates its device
 * arrays (graph, per-node visited bitsets of the largest batch) and frees
 * them before returning.
 */
typedef struct ann_graph ann_graph;
int ann_hnsw_build(const float* X, int64_t n, int32_t d, int32_t metric, int32_t M, int32_t efc,
                   const double* u, int64_t seq_prefix, double batch_frac, int64_t batch_cap,
                   ann_graph** out, void* stream);
int ann_graph_info(const ann_graph* g, int64_t* info);
int ann_graph_export(const ann_graph* g, uint8_t* levels, int32_t* adj0, int32_t* upper_off,
                     int32_t* upper_adj);
int ann_graph_free(ann_graph* g);

/* ---- product quantization on the device -------------------------------- */

/*
 * Product Quantization (Section 2 of the paper and its citation, Jegou et
 * al.): the d dimensions are split into m contiguous subspaces of d/m
 * dimensions (d/m <= 32), each quantized to one of ksub <= 256 centroids.
 * Distances are squared L2, summed in FP64 from the FP32 inputs in ascending
 * dimension order (one multiply and one add per dimension); the nearest
 * centroid is the first minimum (lower index on ties).  The results are
 * fixed bit for bit by the inputs.
 *
 * ann_pq_train: Lloyd's k-means per subspace on the sample rows.  Centroid j
 * starts at sample point init[j]; each iteration assigns every sample point,
 * stops a subspace when no assignment changed, and otherwise replaces each
 * centroid by the FP64 mean of its points (summed in ascending sample order,
 * rounded once to FP32).  An empty cluster takes the sample point with the
 * largest error of that iteration (lower sample position on ties, each point
 * at most once per iteration), clusters in ascending order.
 *   X              device f32[n][d]
 *   sample         device i64[ns], row ids into X (ns >= ksub)
 *   init           device i64[ksub], positions into sample
 *   out_codebook   device f32[m][ksub][d/m]
 *   out_iters      optional host i32: iterations run (the largest over the
 *                  subspaces; max_iter when some subspace never settled)
 * Allocates its scratch (assignments and errors, 12 bytes per sample point
 * and subspace) and frees it before returning; synchronizes `stream`.
 *
 * ann_pq_encode: codes[r][s] = the nearest centroid of subspace s of row r.
 *   X device f32[n][d], codebook device f32[m][ksub][d/m], out_codes device
 *   u8[n][m].  Asynchronous on `stream` (NULL: the null stream, blocking).
 */
int ann_pq_train(const float* X, int64_t n, int32_t d, const int64_t* sample, int64_t ns,
                 const int64_t* init, int32_t m, int32_t ksub, int32_t max_iter,
                 float* out_codebook, int32_t* out_iters, void* stream);
int ann_pq_encode(const float* X, int64_t n, int32_t d, const float* codebook, int32_t m,
                  int32_t ksub, uint8_t* out_codes, void* stream);

/* ---- FP8 storage copy on the device -------------------------------------- */

/*
 * The FP8-E4M3 copy of dense rows that ANN_MODE_FP8 searches: row r gets the
 * scale s_r = max_i |x_ri| / 448 (1 for an all-zero row) and the codes
 * E4M3(x_ri / s_r), both quotients in FP32; OCP E4M3 (bias 7, 3 mantissa
 * bits, no infinities, largest finite 448), rounded to nearest even,
 * saturating at +-448, NaN to 0x7F with its sign.
 *   X          device f32[n][d]
 *   out_codes  device u8[n][d]
 *   out_scale  device f32[n]
 * Asynchronous on `stream` (NULL: the null stream, blocking).
 */
int ann_encode_fp8(const float* X, int64_t n, int32_t d, uint8_t* out_codes, float* out_scale,
                   void* stream);

/* ---- IVF index (inverted lists over a coarse quantizer) ------------------ */

/*
 * An inverted-file index, the index family the paper names beside graphs
 * (Section 1) and plans to add (Section 4, Conclusions and Future Work).  The coarse quantizer is a set of
 * nlist FP32 centroids (k-means over whole vectors: ann_ivf_train below);
 * list l holds the rows whose nearest centroid is l.  The IVF index searches
 * the rows (or PQ codes) of an existing ann_index, which must outlive it; it
 * adds only the centroids and the lists to device memory.
 *
 * ann_ivf_create (host arrays, copied; the caller may free them afterwards):
 *   centroids  f32[nlist][d], finite; 1 <= nlist <= 8192, d a multiple of 4
 *              and at most 1024
 *   list_off   i64[nlist + 1], list_off[0] = 0, non-decreasing, list_off[nlist] = n
 *   list_ids   i32[n]: list l is list_ids[list_off[l] .. list_off[l+1]); every
 *              row 0..n-1 exactly once (any order inside a list)
 * ANN_EFORMAT when the lists are not a partition of the rows.
 *
 * ann_ivf_search: for each query, the probe keys are the squared L2 distances
 * from the FP32 query to the centroids, in the fixed FP32 order of a dense
 * FP32 row; the lists of the min(nprobe, nlist) smallest (key, list id) are
 * scanned; each of their rows is keyed like the HNSW search keys it in
 * `mode` (the index metric); the candidates are ordered by (key, id).  With
 * rerank R > 0 the first min(max(R, k), #candidates) are re-keyed on the
 * FP32 rows and re-sorted.  The first k are returned.
 *   mode         ANN_MODE_F32 / F16 / BF16 / FP8 / PQ (not SPARSE)
 *   rerank       0 .. ANN_K_MAX (needs x_f32 when > 0)
 *   queries      device f32[nq][d]
 *   k            1 .. ANN_K_MAX;  nprobe >= 1 (values above nlist scan all)
 *   out_ids      device i64[nq][k], ascending (key, id), -1 padded when the
 *                probed lists hold fewer than k rows
 *   out_dists    device f32[nq][k], +inf with id -1
 *   out_probes   optional device i32[nq][nprobe]: the probed lists in probe
 *                order, -1 beyond nlist
 *   out_stats    optional device i32[nq][2]: distance evaluations (rows
 *                scanned), lists probed
 *   group        queries per workgroup of the list scan, 0..16.  0: the
 *                default, 8 in the dense modes when nprobe > nlist / 4, else
 *                1.  With group > 1 (dense modes only) the workgroup stages
 *                each list probed by any of its queries in LDS once and every
 *                query that probes it scores it from there; with 1 each query
 *                reads its rows from device memory.  The results are the
 *                same for every group.
 * Asynchronous on `stream` (NULL: the index's stream, and the call waits).
 * Without out_probes the probe lists go to a scratch buffer the IVF object
 * owns (4 bytes per query and probe, grown on demand); batches on different
 * streams are ordered on it by an event, and calls on one IVF object are
 * serialized by the library.  Errors: ANN_EINVAL (arguments, group > 1 in PQ
 * mode), ANN_EUNSUP (sparse mode, missing arrays), ANN_EBUDGET (an explicit
 * group whose tiles and lists do not fit the LDS), ANN_ENOMEM, ANN_EHIP.
 *
 * ann_ivf_free waits for the device and frees the IVF object's memory (not
 * the index's).
 */
typedef struct ann_ivf ann_ivf;
typedef struct ann_ivf_batch {
  int32_t mode;
  int32_t rerank;
  int64_t nq;
  const float* queries;
  int32_t k;
  int32_t nprobe;
  int64_t* out_ids;
  float* out_dists;
  int32_t* out_probes;
  int32_t* out_stats;
  int32_t group;
} ann_ivf_batch;

/*
 * Construction of the lists on the device (k-means over whole vectors, the
 * procedure ann_pq_train applies per subspace, with the same arithmetic and
 * rules: FP64 squared L2 distances in ascending dimension order, first
 * minimum, FP64 means in ascending sample order rounded once, empty clusters
 * re-seeded by error).  The results are fixed bit for bit by the inputs.
 *
 * ann_ivf_train: Lloyd's iterations on the sample rows; centroid j starts at
 * sample point init[j].
 *   X              device f32[n][d]
 *   sample         device i64[ns], row ids into X (ns >= nlist; checked on
 *                  the host, which copies them once)
 *   init           device i64[nlist], positions into sample
 *   out_centroids  device f32[nlist][d]; 1 <= nlist <= 8192
 *   out_iters      optional host i32: iterations run (max_iter when the
 *                  assignment never settled)
 * Allocates its scratch (12 bytes per sample point) and frees it before
 * returning; synchronizes `stream`.
 *
 * ann_ivf_assign: out_list[r] = the nearest centroid of row r.  X device
 * f32[n][d], centroids device f32[nlist][d], out_list device i32[n].
 * Asynchronous on `stream` (NULL: the null stream, blocking).
 *
 * ann_ivf_group (host only): the lists of an assignment, ids ascending inside
 * each list.  list host i32[n] with values in [0, nlist); list_off host
 * i64[nlist + 1]; list_ids host i32[n].
 */
int ann_ivf_train(const float* X, int64_t n, int32_t d, const int64_t* sample, int64_t ns,
                  const int64_t* init, int32_t nlist, int32_t max_iter, float* out_centroids,
                  int32_t* out_iters, void* stream);
int ann_ivf_assign(const float* X, int64_t n, int32_t d, const float* centroids, int32_t nlist,
                   int32_t* out_list, void* stream);
int ann_ivf_group(const int32_t* list, int64_t n, int32_t nlist, int64_t* list_off,
                  int32_t* list_ids);

int ann_ivf_create(ann_index* ix, int32_t nlist, const float* centroids, const int64_t* list_off,
                   const int32_t* list_ids, ann_ivf** out);
int ann_ivf_free(ann_ivf* v);
int ann_ivf_search(ann_ivf* v, const ann_ivf_batch* b, void* stream);

/* ---- serving: continuous batching ------------------------------------------ */

/*
 * A server keeps the index resident and answers single requests (one query
 * each, with its own k and ef) submitted from any host thread, with the
 * search above (the paper answers one query at a time, Section 3; here the
 * requests in flight share the GPU).
 *
 * Admission is per slot.  One persistent search kernel runs `slots`
 * workgroups ("slots", each serving one request at a time).  Submitted
 * requests wait in a host queue (at most queue_cap) until a ring entry in
 * pinned host memory is free (at most max_inflight requests on the device,
 * running or waiting for a slot); the server's host thread writes them into
 * the ring and publishes them in submission order.  The first slot that is
 * free claims the next published request, so a request that arrives while
 * others run starts as soon as any slot is free, and its work overlaps
 * theirs on the device.  The kernel writes each result into its ring entry
 * with a completion flag, and the host thread moves it to the completion
 * list.  When nothing has been published for idle_us the kernel ends, and
 * the next request launches it again.
 *
 * Results equal ann_search_ex's for the same query, k, ef, mode and rerank,
 * bit for bit, whatever else is in flight.
 *
 * ann_server_cfg:
 *   mode, rerank   as in ann_batch (dense modes); the launch shape (waves
 *                  per query, lanes per row, beam layout) is the index's for
 *                  `mode` (ann_set_launch) when the server is created
 *   max_inflight   ring entries, >= 1 (host memory: 4 d + 12 k_max + 40 bytes each)
 *   slots          workgroups of the kernel; 0: what the compute units hold
 *                  at once (occupancy), halved until the visited bitsets and
 *                  beam lists fit hbm_budget
 *   k_max, ef_max  bounds of the requests' k and ef
 *   queue_cap      waiting requests before ann_server_submit returns ANN_EAGAIN
 *   idle_us        the kernel ends after this long without a new request;
 *                  0: 2,000
 *   hbm_budget     bytes of device memory the slots' workspace may use
 */
typedef struct ann_server ann_server;

typedef struct ann_server_cfg {
  int32_t mode;
  int32_t rerank;
  int32_t max_inflight;
  int32_t slots;
  int32_t k_max;
  int32_t ef_max;
  int32_t queue_cap;
  int32_t idle_us;
  int64_t hbm_budget;
} ann_server_cfg;

typedef struct ann_request {
  uint64_t tag;          /* returned in the completion */
  const float* query;    /* host f32[d]; copied at submit */
  int32_t k, ef;
} ann_request;

/* A finished request.  t_*: host steady clock in seconds (submitted, written
 * into the ring, seen done); d_*: the device clock in seconds (claimed by a
 * slot, finished), comparable between the requests of one server; slot: the
 * workgroup that served it. */
typedef struct ann_completion {
  uint64_t tag;
  int32_t status;        /* ANN_OK, or ANN_EBUDGET if k or ef had to be clamped */
  int32_t k;
  int64_t ids[ANN_K_MAX];
  float dists[ANN_K_MAX];
  double t_submit, t_start, t_done;
  double d_start, d_done;
  int32_t slot;
  int32_t reserved;
} ann_completion;

/* What a server runs with. */
typedef struct ann_server_state {
  int32_t slots;
  int32_t ring;
  int32_t waves_per_query;
  int32_t lanes_per_row;
  int64_t queued;        /* requests waiting for a ring entry */
} ann_server_state;

/* Validates cfg, allocates the slots' workspace (device) and the ring
 * (pinned host memory), starts the host thread.  ANN_EBUDGET if one slot does
 * not fit hbm_budget or ef_max does not fit on chip. */
int ann_server_create(const ann_index* ix, const ann_server_cfg* cfg, ann_server** out);
/* Copies the request into the queue; ANN_EAGAIN if the queue is full,
 * ANN_EINVAL for k or ef outside the bounds. */
int ann_server_submit(ann_server* s, const ann_request* r);
/* Moves up to `max` finished requests into out[]; returns how many (>= 0),
 * or a negative error code.  Non-blocking. */
int ann_server_poll(ann_server* s, ann_completion* out, int32_t max);
int ann_server_info(const ann_server* s, ann_server_state* out);
/* Stops admitting: requests not yet claimed by a slot are dropped, running
 * ones finish; then frees the server.  Returns the first error of the
 * server's host thread, if any. */
int ann_server_destroy(ann_server* s);

/* ---- misc -------------------------------------------------------------- */

/* Text of the calling thread's last error ("" if none). */
const char* ann_last_error(void);
/* Library version, e.g. 1. */
int ann_version(void);
/* Number of visible GPUs (0 if none); does not fail. */
int ann_device_count(void);

/*
 * Invariant checks of the search kernels, in a library built with
 * ANN_DEBUG_CHECKS (libann_debug.so beside libann.so; slower, for tests).
 * Between expansions every workgroup checks its beam (the sorted list and
 * insert buffer of the layer-0 search): each strictly ascending in (key, id),
 * so its ids unique; |W| <= ef after the cut; every id inside [0, n); every
 * entry before the scan position expanded; an expansion's candidate counts
 * at most 64.  A violation sets a bit of a word the index holds (1 size, 2
 * list order, 4 buffer order, 8 id range, 16 scan position, 32 counts); the
 * kernels never trap.  ann_debug_flags waits for the device, copies the word
 * to *out and, when clear is nonzero, zeroes it.  Without ANN_DEBUG_CHECKS it
 * returns ANN_EUNSUP with *out = 0.
 */
int ann_debug_flags(const ann_index* ix, uint32_t* out, int32_t clear);

#ifdef __cplusplus
}
#endif

#endif /* ANN_H_ */
