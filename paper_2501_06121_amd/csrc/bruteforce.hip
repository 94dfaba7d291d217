// Exact k-nearest neighbours on matrix cores (MFMA), used as ground truth.
//
// The k-NN problem of the paper (Section 1: the k nearest neighbours of a
// query among a dataset X of d-dimensional vectors) solved by a full scan:
//
// Stage 1 (bf_tiles): a workgroup of 4 wavefronts owns 128 queries and a
//   contiguous range of base rows.  For each tile of 128 base rows it forms
//   the 128 x 128 block of dot products with v_mfma_f32_16x16x4_f32, each
//   wave a 64 x 64 quarter (16 accumulator tiles).  Operands pass through LDS
//   in stages of 32 dimensions, stored k-major so that the MFMA operand reads
//   are free of bank conflicts; the next stage is loaded into registers while
//   the current one is multiplied.  The block becomes approximate keys (-dot,
//   or |x|^2 - 2 dot for L2: |q|^2 is the same for every row of a query) in a
//   tile that reuses the stage buffers, and each query merges the rows that
//   beat the (k + 17)-th entry of its sorted list (64 entries, in LDS) into
//   it.  At the end the lists go to scratch memory: 64 candidates per (query,
//   range), of which the first k + 17 are exact.
// Stage 2 (bf_finish): one wavefront per query merges the candidate lists of
//   all ranges into the approximate top-64, re-scores the best k + 16 with the
//   FP32 rows in the same fixed order as the search kernel, sorts them by
//   (key, id) and writes the first k.  The result is certified exact when the
//   k-th exact key plus the worst-case difference between the MFMA and the
//   fixed-order evaluations stays below the approximate key of every
//   candidate that was not re-scored.
//
// Half-precision preselection (bf_tiles_h): the same scan with FP16 copies
// of the rows and queries (rounded to nearest even from the FP32 values) on
// v_mfma_f32_16x16x32_f16, eight times the FP32 matrix rate and half the
// bytes per row.  Its certificate adds the rounding of the operands to the
// bound.  Queries it cannot certify are scanned again by the FP32 tiles
// (whose workgroups skip query blocks with nothing to redo), so the call
// returns the same exact top-k either way.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "ann.h"
#include "internal.h"
#include "search_kernels.h"

namespace ann {
namespace {

constexpr int BM = 128;     // queries per workgroup
constexpr int BN = 128;     // base rows per tile
constexpr int BK = 32;      // dimensions per stage
constexpr int KC = 64;      // candidates kept per query and range
constexpr int kRescore = 16;
constexpr int LDA = BM + 16;   // k-major stage rows (16 mod 32 banks: conflict-free reads)
constexpr int LDB = BN + 16;
constexpr int TLT = BM + 4;    // key tile column length (a multiple of 4: 16-byte stores)
constexpr int kStageFloats = 2 * BK * (LDA + LDB);
static_assert(BN * TLT <= kStageFloats, "the key tile reuses the stage buffers");

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool kid_less(float ka, int ia, float kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// Merge 64 candidates held one per lane (unsorted, +inf = empty) into the
// sorted list (lk, li)[0..KC) in LDS, keeping the best KC.
__device__ void merge_list(float* lk, int* li, float k, int id) {
  const int lane = threadIdx.x & 63;
  // bitonic sort of the 64 lanes
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const float ok = __shfl_xor(k, stride, 64);
      const int oi = __shfl_xor(id, stride, 64);
      const bool lower = (lane & stride) == 0;
      const bool asc = (lane & size) == 0;
      const bool take = (lower == asc) ? kid_less(ok, oi, k, id) : kid_less(k, id, ok, oi);
      if (take) { k = ok; id = oi; }
    }
  }
  // rank of each new entry among the list and of each list entry among the new
  const float ek = lk[lane];
  const int ei = li[lane];
  int lo = 0, hi = KC;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kid_less(lk[mid], li[mid], k, id)) lo = mid + 1; else hi = mid;
  }
  const int pos_new = lo + lane;
  int lo2 = 0, hi2 = 64;
  while (lo2 < hi2) {   // new entries below the list entry: new is sorted
    const int mid = (lo2 + hi2) >> 1;
    const float mk = __shfl(k, mid, 64);
    const int mi = __shfl(id, mid, 64);
    if (kid_less(mk, mi, ek, ei)) lo2 = mid + 1; else hi2 = mid;
  }
  const int pos_old = lane + lo2;
  // one wavefront owns the list: its LDS reads above complete before the
  // writes below (in-order LDS queue); the wave barrier keeps the compiler
  // from moving them
  __builtin_amdgcn_wave_barrier();
  if (pos_old < KC) { lk[pos_old] = ek; li[pos_old] = ei; }
  if (pos_new < KC) { lk[pos_new] = k; li[pos_new] = id; }
  __builtin_amdgcn_wave_barrier();
}

// Insert the few candidates of lanes `mask` into the sorted list (lk, li)[0..KC)
// one at a time: the list sits one entry per lane, each candidate's rank is
// the number of entries below it, and the entries from that rank on move up
// one lane (the last one drops out).
__device__ void insert_few(float* lk, int* li, float k, int id, uint64_t mask) {
  const int lane = threadIdx.x & 63;
  float ek = lk[lane];
  int ei = li[lane];
  for (uint64_t m = mask; m; m &= m - 1) {
    const int b = __builtin_ctzll(m);
    const float ck = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(k), b));
    const int ci = __builtin_amdgcn_readlane(id, b);
    const float wk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ek), KC - 1));
    const int wi = __builtin_amdgcn_readlane(ei, KC - 1);
    if (!kid_less(ck, ci, wk, wi)) continue;        // the list has tightened meanwhile
    const int rank = __builtin_popcountll(__ballot(kid_less(ek, ei, ck, ci)));
    const float uk = __shfl_up(ek, 1, 64);
    const int ui = __shfl_up(ei, 1, 64);
    if (lane > rank) { ek = uk; ei = ui; }
    if (lane == rank) { ek = ck; ei = ci; }
  }
  __builtin_amdgcn_wave_barrier();
  lk[lane] = ek;
  li[lane] = ei;
  __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(64) bf_norms(const float* X, int64_t n, int d, float* x2) {
  const int64_t r = blockIdx.x;
  if (r >= n) return;
  float acc = 0.0f;
  for (int i = threadIdx.x; i < d; i += 64) {
    const float v = X[r * d + i];
    acc = __builtin_fmaf(v, v, acc);
  }
  for (int s = 32; s >= 1; s >>= 1) acc += __shfl_down(acc, s, 64);
  if (threadIdx.x == 0) x2[r] = acc;
}

struct BfParams {
  const float* X;
  const float* x2;       // squared row norms (L2 only)
  int64_t n;
  int d;                 // multiple of 4
  int metric;
  const float* Q;
  int64_t nq;
  int64_t rows_per_range;
  int nranges;
  int admit;             // a row enters a list when it beats the list's admit-th entry
  float* cand_key;       // [nq][nranges][KC]
  int32_t* cand_id;
  const int32_t* redo;   // optional [nq]: only blocks with a query whose flag is 0 are scanned
  const uint16_t* Xh;    // FP16 copies (bf_tiles_h): rows [n][d], queries [nq][d]
  const uint16_t* Qh;
  uint32_t* bound;       // optional [nq]: shared admission bounds (ordered key bits, see below)
};

// Shared admission bounds.  A range's list, once it holds `admit` entries,
// has its admit-th key at or above the admit-th best key over all rows, so
// the smallest such key published by the workgroups scanning the same
// queries in other ranges bounds what any range still needs: a row whose key
// is not below it can be left out (it sorts after the merged list's admit-th
// entry, which the certificate already accounts for).  Keys are kept as
// order-preserving unsigned bits so that atomicMin applies; all ones (the
// initial fill) means no bound.
__device__ __forceinline__ uint32_t key_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float bits_key(uint32_t o) {
  if (o == 0xFFFFFFFFu) return __builtin_inff();
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// Whether this workgroup's block of BM queries has work: without a redo mask
// always; with one, when some query of the block was not certified.
__device__ __forceinline__ bool block_has_work(const BfParams& p, int64_t q0) {
  if (!p.redo) return true;
  const int tid = threadIdx.x;
  const int64_t q = q0 + tid;
  const int need = (tid < BM && q < p.nq && p.redo[q] == 0) ? 1 : 0;
  return __syncthreads_or(need) != 0;
}

// One stage (32 dimensions from k0) of the query block and of a base tile:
// 4 float4 of each per thread.  The loads are unconditional (rows past the
// matrices read their last row, dimensions past d read dimension 0): a load
// under a per-lane condition makes the compiler wait for it on the spot,
// which would serialise the prefetch.  Rows past the matrices are never
// used (their keys are +inf, their lists are not written); dimensions past
// d are zeroed when the stage is stored.
struct StageRegs {
  float4 q[4];
  float4 x[4];
};

__device__ __forceinline__ void load_stage(const BfParams& p, int64_t q0, int64_t t0,
                                           int64_t r_end, int k0, StageRegs& r) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = tid + 256 * u;       // 1024 float4 per operand: row idx / 8, float4 idx % 8
    const int row = idx >> 3;
    int k = k0 + 4 * (idx & 7);
    k = k < p.d ? k : 0;
    const int64_t qi = q0 + row < p.nq ? q0 + row : p.nq - 1;
    const int64_t xi = t0 + row < r_end ? t0 + row : r_end - 1;
    r.q[u] = *(const float4*)(p.Q + qi * p.d + k);
    r.x[u] = *(const float4*)(p.X + xi * p.d + k);
  }
}

__device__ __forceinline__ void store_stage(float* sa, float* sb, const StageRegs& r, int k0, int d) {
  const int tid = threadIdx.x;
  // the thread's dimensions are the same in every u (256 u is a multiple of 8)
  const bool in = k0 + 4 * (tid & 7) < d;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = tid + 256 * u;
    const int row = idx >> 3;
    const int kk = 4 * (idx & 7);
    const float4 q = in ? r.q[u] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 x = in ? r.x[u] : make_float4(0.f, 0.f, 0.f, 0.f);
    sa[(kk + 0) * LDA + row] = q.x;
    sa[(kk + 1) * LDA + row] = q.y;
    sa[(kk + 2) * LDA + row] = q.z;
    sa[(kk + 3) * LDA + row] = q.w;
    sb[(kk + 0) * LDB + row] = x.x;
    sb[(kk + 1) * LDB + row] = x.y;
    sb[(kk + 2) * LDB + row] = x.z;
    sb[(kk + 3) * LDB + row] = x.w;
  }
}

// The 128 x 128 block of a tile (accumulators of the four waves: row
// wq + 16 rb + 4 (lane / 16) + r, column wx + 16 cb + lane % 16) as
// approximate keys in the LDS tile, stored by column: tile[col * TLT + row].
// A lane's four rows of one column are one 16-byte store, and the 16 lanes
// of a store row fill the 64 banks once.
__device__ __forceinline__ void tile_keys(const BfParams& p, const floatx4 (&acc)[4][4], float* tile,
                                          int64_t t0, int64_t r_end, int wq, int wx, int lane) {
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int col = wx + cb * 16 + (lane & 15);
    const int64_t xi = t0 + col;
    const bool in = xi < r_end;
    const float x2 = (p.metric == METRIC_IP || !in) ? 0.0f : p.x2[xi];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int row0 = wq + rb * 16 + 4 * (lane >> 4);
      float4 k4;
      const floatx4 a = acc[rb][cb];
      if (p.metric == METRIC_IP) {
        k4 = make_float4(-a[0], -a[1], -a[2], -a[3]);
      } else {
        k4 = make_float4(x2 - 2.0f * a[0], x2 - 2.0f * a[1], x2 - 2.0f * a[2], x2 - 2.0f * a[3]);
      }
      if (!in) k4 = make_float4(__builtin_inff(), __builtin_inff(), __builtin_inff(), __builtin_inff());
      *(float4*)(tile + col * TLT + row0) = k4;
    }
  }
}

// Merge the key tile into the per-query lists (each wave its 32 queries).
// bnd: the shared bound of this lane's query (row wave * 32 + lane % 32), +inf
// without one; rows need a key strictly below it as well.
__device__ __forceinline__ void tile_merge(const BfParams& p, const float* tile, float (*lk)[KC],
                                           int (*li)[KC], int64_t q0, int64_t t0, int64_t r_end,
                                           int wave, int lane, float bnd = __builtin_inff()) {
  // First every lane screens one (query, half tile) against that query's
  // admission entry: lane l takes query row wave * 32 + l % 32 and half
  // l / 32, the second half starting 8 columns on so that the two halves
  // read different banks.  Only the flagged pairs take the wave-wide path
  // (a later merge only lowers the entry, so an unflagged pair stays out).
  static_assert(BN == 128 && BM / 4 == 32, "one lane per (query, half tile) of the wave");
  bool hit = false;
  {
    const int row = wave * (BM / 4) + (lane & 31);
    const int half = lane >> 5;
    if (q0 + row < p.nq) {
      const float thr_k = lk[row][p.admit - 1];
      const int thr_i = li[row][p.admit - 1];
      for (int c = 0; c < 64; ++c) {
        const int col = half * 64 + ((c + 8 * half) & 63);
        const int id = (t0 + col < r_end) ? (int)(t0 + col) : 0x7FFFFFFF;
        const float key = tile[col * TLT + row];
        hit = hit | (kid_less(key, id, thr_k, thr_i) && key < bnd);
      }
    }
  }
  for (uint64_t todo = __ballot(hit); todo; todo &= todo - 1) {
    const int j = __builtin_ctzll(todo);
    const int row = wave * (BM / 4) + (j & 31);
    const int col = (j >> 5) * 64 + lane;
    const float thr_k = lk[row][p.admit - 1];
    const int thr_i = li[row][p.admit - 1];
    const float rb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bnd), j & 31));
    float k = tile[col * TLT + row];
    // columns past the range are empty entries (+inf, largest id)
    int id = (t0 + col < r_end) ? (int)(t0 + col) : 0x7FFFFFFF;
    const bool keep = kid_less(k, id, thr_k, thr_i) && k < rb;
    const uint64_t km = __ballot(keep);
    if (!km) continue;
    if (__builtin_popcountll(km) > 8) {
      if (!keep) { k = __builtin_inff(); id = 0x7FFFFFFF; }
      merge_list(lk[row], li[row], k, id);
    } else {
      insert_few(lk[row], li[row], k, id, km);
    }
  }
}

// The lists of a workgroup's queries out to the candidate arrays.
__device__ __forceinline__ void lists_out(const BfParams& p, float (*lk)[KC], int (*li)[KC], int64_t q0,
                                          int range) {
  for (int i = threadIdx.x; i < BM * KC; i += blockDim.x) {
    const int r = i / KC, c = i % KC;
    const int64_t qi = q0 + r;
    if (qi < p.nq) {
      const size_t o = ((size_t)qi * p.nranges + range) * KC + c;
      p.cand_key[o] = lk[r][c];
      p.cand_id[o] = li[r][c];
    }
  }
}

__global__ void __launch_bounds__(256) bf_tiles(BfParams p) {
  __shared__ __align__(16) float stage[kStageFloats];   // [2][BK][LDA] queries, [2][BK][LDB] rows; later the key tile
  __shared__ float lk[BM][KC];
  __shared__ int li[BM][KC];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int wq = (wave & 1) * 64;         // this wave's 64 queries of the block
  const int wx = (wave >> 1) * 64;        // and 64 rows of the tile
  const int64_t q0 = (int64_t)blockIdx.x * BM;
  const int range = blockIdx.y;
  const int64_t r_begin = (int64_t)range * p.rows_per_range;
  const int64_t r_end = r_begin + p.rows_per_range < p.n ? r_begin + p.rows_per_range : p.n;
  float* const sa = stage;                  // stage buffer b of the queries: sa + b * BK * LDA
  float* const sb = stage + 2 * BK * LDA;   // of the rows: sb + b * BK * LDB
  float* const tile = stage;
  const int nst = (p.d + BK - 1) / BK;
  if (!block_has_work(p, q0)) return;

  for (int i = tid; i < BM * KC; i += 256) {
    lk[i / KC][i % KC] = __builtin_inff();
    li[i / KC][i % KC] = 0x7FFFFFFF;
  }

  StageRegs regs;
  if (r_begin < r_end) load_stage(p, q0, r_begin, r_end, 0, regs);
  for (int64_t t0 = r_begin; t0 < r_end; t0 += BN) {
    __syncthreads();                      // the previous tile's keys have been read
    store_stage(sa, sb, regs, 0, p.d);
    __syncthreads();
    floatx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < nst; ++s) {
      const int buf = s & 1;
      if (s + 1 < nst) load_stage(p, q0, t0, r_end, (s + 1) * BK, regs);
      const float* A = sa + buf * (BK * LDA);
      const float* B = sb + buf * (BK * LDB);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        float av[4], bv[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) av[rb] = A[kr * LDA + wq + rb * 16 + (lane & 15)];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) bv[cb] = B[kr * LDB + wx + cb * 16 + (lane & 15)];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb], bv[cb], acc[rb][cb], 0, 0, 0);
      }
      if (s + 1 < nst) store_stage(sa + (buf ^ 1) * (BK * LDA), sb + (buf ^ 1) * (BK * LDB), regs, (s + 1) * BK, p.d);
      __syncthreads();
    }
    tile_keys(p, acc, tile, t0, r_end, wq, wx, lane);
    __syncthreads();
    // the next tile's first stage is in flight while the lists are merged
    if (t0 + BN < r_end) load_stage(p, q0, t0 + BN, r_end, 0, regs);
    tile_merge(p, tile, lk, li, q0, t0, r_end, wave, lane);
  }
  __syncthreads();
  lists_out(p, lk, li, q0, range);
}

// ---- half-precision preselection ---------------------------------------

constexpr int BKH = 64;         // dimensions per stage
constexpr int LDH = BKH + 8;    // row stride in halves: 144 B, so 16 rows of a 16-byte
                                // read start on 16 different 4-bank groups
static_assert(2 * 2 * BM * LDH * 2 <= kStageFloats * 4, "two half stages fit the stage buffers");

typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// FP16 copy, rounded to nearest even; values beyond the FP16 range saturate
// (the finishing kernel refuses to certify a query that needed it).
__global__ void bf_half(const float* src, int64_t count, uint16_t* dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = fminf(fmaxf(src[i], -65504.0f), 65504.0f);
    dst[i] = __builtin_bit_cast(uint16_t, (_Float16)v);
  }
}

// One stage (64 dimensions from k0) of the query block and a base tile: 256
// rows (queries first) of 8 16-byte chunks, 8 chunks per thread (d is a
// multiple of 8: a chunk is wholly in or out).  Unconditional loads as in
// load_stage: rows past the matrices read their last row, chunks past d
// chunk 0, zeroed when stored.
struct StageRegsH {
  uint4 v[8];
};

__device__ __forceinline__ void load_stage_h(const BfParams& p, int64_t q0, int64_t t0,
                                             int64_t r_end, int k0, StageRegsH& r) {
  int k = k0 + 8 * (threadIdx.x & 7);     // the same in every u
  k = k < p.d ? k : 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int row = (int)(threadIdx.x + 256 * u) >> 3;   // u < 4: queries, else rows
    const uint16_t* src;
    if (u < 4) {
      const int64_t qi = q0 + row < p.nq ? q0 + row : p.nq - 1;
      src = p.Qh + qi * p.d + k;
    } else {
      const int64_t xi = t0 + (row - BM) < r_end ? t0 + (row - BM) : r_end - 1;
      src = p.Xh + xi * p.d + k;
    }
    r.v[u] = *(const uint4*)src;
  }
}

__device__ __forceinline__ void store_stage_h(uint16_t* sbuf, const StageRegsH& r, int k0, int d) {
  const bool in = k0 + 8 * (threadIdx.x & 7) < d;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int idx = threadIdx.x + 256 * u;
    *(uint4*)(sbuf + (idx >> 3) * LDH + 8 * (idx & 7)) = in ? r.v[u] : make_uint4(0u, 0u, 0u, 0u);
  }
}

// bf_tiles with FP16 operands on v_mfma_f32_16x16x32_f16: the same blocks,
// lists, admission and output, 64 dimensions per stage.
// Hits of one tile, found in registers: the (query row, column, key) of every
// key at or below its query's threshold (list admission entry and shared
// bound of the previous tile: a superset of what the lists admit now).
constexpr int kHitCap = 1024;

__global__ void __launch_bounds__(256) bf_tiles_h(BfParams p) {
  __shared__ __align__(16) float stage[kStageFloats];   // [2][256 rows][LDH] halves; later the key tile
  __shared__ float lk[BM][KC];
  __shared__ int li[BM][KC];
  __shared__ float thr_s[BM];             // per query row: min(admission key, shared bound)
  __shared__ int hit_n;
  __shared__ int hit_rc[kHitCap];         // row * BN + column
  __shared__ float hit_k[kHitCap];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int wq = (wave & 1) * 64;
  const int wx = (wave >> 1) * 64;
  const int64_t q0 = (int64_t)blockIdx.x * BM;
  const int range = blockIdx.y;
  const int64_t r_begin = (int64_t)range * p.rows_per_range;
  const int64_t r_end = r_begin + p.rows_per_range < p.n ? r_begin + p.rows_per_range : p.n;
  uint16_t* const sh = (uint16_t*)stage;   // stage buffer b: sh + b * 2 * BM * LDH
  float* const tile = stage;
  const int nst = (p.d + BKH - 1) / BKH;
  if (!block_has_work(p, q0)) return;

  for (int i = tid; i < BM * KC; i += 256) {
    lk[i / KC][i % KC] = __builtin_inff();
    li[i / KC][i % KC] = 0x7FFFFFFF;
  }
  if (tid < BM) thr_s[tid] = __builtin_inff();
  if (tid == 0) hit_n = 0;

  StageRegsH regs;
  if (r_begin < r_end) load_stage_h(p, q0, r_begin, r_end, 0, regs);
  for (int64_t t0 = r_begin; t0 < r_end; t0 += BN) {
    __syncthreads();                      // the previous tile's keys have been read
    store_stage_h(sh, regs, 0, p.d);
    __syncthreads();
    floatx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int st = 0; st < nst; ++st) {
      const int buf = st & 1;
      if (st + 1 < nst) load_stage_h(p, q0, t0, r_end, (st + 1) * BKH, regs);
      const uint16_t* S = sh + buf * (2 * BM * LDH);
#pragma unroll
      for (int j = 0; j < BKH / 32; ++j) {
        // lane: row lane % 16 of each 16-row block, dimensions 8 (lane / 16) ..
        // of this 32-dimension step; queries and rows take the same
        // dimensions, so each product sums over all 32 of them
        const int ko = 32 * j + 8 * (lane >> 4);
        halfx8 av[4], bv[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
          av[rb] = *(const halfx8*)(S + (wq + rb * 16 + (lane & 15)) * LDH + ko);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          bv[cb] = *(const halfx8*)(S + (BM + wx + cb * 16 + (lane & 15)) * LDH + ko);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[rb], bv[cb], acc[rb][cb], 0, 0, 0);
      }
      if (st + 1 < nst) store_stage_h(sh + (buf ^ 1) * (2 * BM * LDH), regs, (st + 1) * BKH, p.d);
      __syncthreads();
    }
    // the shared bound of this lane's query, read before the next stage's
    // loads are issued (a load waited for after them would wait for them too)
    const int brow = wave * (BM / 4) + (lane & 31);
    const int64_t bq = q0 + brow < p.nq ? q0 + brow : p.nq - 1;
    const uint32_t bseen = p.bound ? p.bound[bq] : 0xFFFFFFFFu;
    const float bnd = bits_key(bseen);
    // the keys that may enter a list go to the hit list; the rest of the
    // tile is never written out
    float th[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) th[rb][r] = thr_s[wq + rb * 16 + 4 * (lane >> 4) + r];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = wx + cb * 16 + (lane & 15);
      const int64_t xi = t0 + col;
      const bool in = xi < r_end;
      const float x2 = (p.metric == METRIC_IP || !in) ? 0.0f : p.x2[xi];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wq + rb * 16 + 4 * (lane >> 4) + r;
          const float dot = acc[rb][cb][r];
          const float key = (p.metric == METRIC_IP) ? -dot : x2 - 2.0f * dot;
          if (in && key <= th[rb][r]) {
            const int slot = atomicAdd(&hit_n, 1);
            if (slot < kHitCap) { hit_rc[slot] = row * BN + col; hit_k[slot] = key; }
          }
        }
    }
    __syncthreads();
    const int nh = hit_n;
    if (nh > kHitCap) {
      // too many for the list (the first tiles of a range): the whole tile
      // through LDS as before
      tile_keys(p, acc, tile, t0, r_end, wq, wx, lane);
      __syncthreads();
      if (t0 + BN < r_end) load_stage_h(p, q0, t0 + BN, r_end, 0, regs);
      tile_merge(p, tile, lk, li, q0, t0, r_end, wave, lane, bnd);
    } else {
      if (t0 + BN < r_end) load_stage_h(p, q0, t0 + BN, r_end, 0, regs);
      // each wave inserts the hits of its 32 query rows, one row at a time
      for (int base = 0; base < nh; base += 64) {
        const int i = base + lane;
        int row = -1;
        float k = __builtin_inff();
        int id = 0x7FFFFFFF;
        if (i < nh) {
          const int rc = hit_rc[i];
          if ((rc / BN) / (BM / 4) == wave) {
            row = rc / BN;
            k = hit_k[i];
            id = (int)(t0 + rc % BN);
          }
        }
        for (uint64_t todo = __ballot(row >= 0); todo;) {
          const int j = __builtin_ctzll(todo);
          const int r = __builtin_amdgcn_readlane(row, j);
          const uint64_t same = __ballot(row == r);
          todo &= ~same;
          const float rb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bnd), r & 31));
          const bool keep = row == r && kid_less(k, id, lk[r][p.admit - 1], li[r][p.admit - 1]) && k < rb;
          const uint64_t km = __ballot(keep);
          if (!km) continue;
          if (__builtin_popcountll(km) > 8) {
            merge_list(lk[r], li[r], keep ? k : __builtin_inff(), keep ? id : 0x7FFFFFFF);
          } else {
            insert_few(lk[r], li[r], k, id, km);
          }
        }
      }
    }
    // publish this range's admit-th key where it lowers the bound, and the
    // threshold of the next tile's hit search
    if (lane < 32) {
      const float ka = lk[brow][p.admit - 1];
      uint32_t nb = bseen;
      if (p.bound && q0 + brow < p.nq && ka < __builtin_inff() && key_bits(ka) < bseen) {
        atomicMin(&p.bound[bq], key_bits(ka));
        nb = key_bits(ka);
      }
      thr_s[brow] = fminf(ka, bits_key(nb));
    }
    __syncthreads();
    if (tid == 0) hit_n = 0;
  }
  __syncthreads();
  lists_out(p, lk, li, q0, range);
}

struct BfFinish {
  const float* X;
  int64_t n;
  int d;
  int metric;
  const float* Q;
  int64_t nq;
  int nranges;
  const float* cand_key;
  const int32_t* cand_id;
  int k;
  float xmax, x2max;
  int half;              // the candidates come from bf_tiles_h: its operand rounding joins the bound
  const int32_t* redo;   // optional [nq]: queries flagged 1 are done (certified by the half pass)
  int64_t* out_ids;
  float* out_dists;
  int32_t* out_certified;
};

__global__ void __launch_bounds__(64) bf_finish(BfFinish p) {
  __shared__ float lk[KC];
  __shared__ int li[KC];
  __shared__ float ek[KC];
  const int lane = threadIdx.x;
  const int64_t q = blockIdx.x;
  if (q >= p.nq) return;
  if (p.redo && p.redo[q]) {
    if (lane == 0 && p.out_certified) p.out_certified[q] = 2;   // certified by the half pass
    return;
  }
  lk[lane] = __builtin_inff();
  li[lane] = 0x7FFFFFFF;
  __syncthreads();
  for (int r = 0; r < p.nranges; ++r) {
    const size_t o = ((size_t)q * p.nranges + r) * KC + lane;
    merge_list(lk, li, p.cand_key[o], p.cand_id[o]);
  }
  const float* qr = p.Q + q * p.d;
  // |q|_1 and |q|^2 for the error bound and the L2 offset
  float a1 = 0.f, q2 = 0.f, qm = 0.f;
  for (int i = lane; i < p.d; i += 64) {
    a1 += fabsf(qr[i]);
    q2 = __builtin_fmaf(qr[i], qr[i], q2);
    qm = fmaxf(qm, fabsf(qr[i]));
  }
  for (int s = 32; s >= 1; s >>= 1) {
    a1 += __shfl_xor(a1, s, 64);
    q2 += __shfl_xor(q2, s, 64);
    qm = fmaxf(qm, __shfl_xor(qm, s, 64));
  }
  // exact re-score of the best R candidates: 64 lanes per row, the fixed
  // FP32 order (chunk g of 4 floats feeds partial g mod 64 = lane)
  const int R = p.k + kRescore < KC ? p.k + kRescore : KC;
  const int nch = p.d / 4;
  for (int j = 0; j < R; ++j) {
    const int id = li[j];
    float acc = 0.0f;
    if (id >= 0 && id < p.n) {
      const float* xr = p.X + (size_t)id * p.d;
      for (int g = lane; g < nch; g += 64) {
        const float4 xv = *(const float4*)(xr + 4 * g);
        const float4 qv = *(const float4*)(qr + 4 * g);
        if (p.metric == METRIC_IP) {
          acc = __builtin_fmaf(qv.x, xv.x, acc);
          acc = __builtin_fmaf(qv.y, xv.y, acc);
          acc = __builtin_fmaf(qv.z, xv.z, acc);
          acc = __builtin_fmaf(qv.w, xv.w, acc);
        } else {
          const float t0 = qv.x - xv.x, t1 = qv.y - xv.y, t2 = qv.z - xv.z, t3 = qv.w - xv.w;
          acc = __builtin_fmaf(t0, t0, acc);
          acc = __builtin_fmaf(t1, t1, acc);
          acc = __builtin_fmaf(t2, t2, acc);
          acc = __builtin_fmaf(t3, t3, acc);
        }
      }
      for (int s = 32; s >= 1; s >>= 1) acc = acc + __shfl_down(acc, s, 64);
    }
    if (lane == 0) ek[j] = (id >= 0 && id < p.n) ? (p.metric == METRIC_IP ? -acc : acc) : __builtin_inff();
  }
  __syncthreads();
  // rank the re-scored candidates by (exact key, id)
  float kx = lane < R ? ek[lane] : __builtin_inff();
  int ix = lane < R ? li[lane] : 0x7FFFFFFF;
  int rank = 0;
  for (int j = 0; j < R; ++j) rank += kid_less(ek[j], li[j], kx, ix) ? 1 : 0;
  const bool valid = lane < R && kx != __builtin_inff();
  const int nvalid = __builtin_popcountll(__ballot(valid));
  if (valid && rank < p.k) {
    p.out_ids[q * p.k + rank] = ix;
    p.out_dists[q * p.k + rank] = kx;
  }
  if (lane >= nvalid && lane < p.k) {      // fewer than k rows: padding
    p.out_ids[q * p.k + lane] = -1;
    p.out_dists[q * p.k + lane] = __builtin_inff();
  }
  // certificate: every candidate not re-scored has approximate key >= lk[R-1]
  // (and every row never kept has one >= its range's 64th); the approximate
  // and the fixed-order keys differ by at most E
  const float u = 0x1p-24f;
  float E = 2.0f * (float)(p.d + 16) * u;
  if (!p.half) {
    E *= (p.metric == METRIC_IP) ? a1 * p.xmax : 2.0f * a1 * p.xmax + p.x2max + q2;
  } else {
    // S bounds sum |q_i x_i| for every row: by |q|_1 max|x_ij| or by Cauchy-
    // Schwarz (|q|_2 max |x|_2), with 0.1% for the rounding of a1, q2, x2max
    const float S = fminf(a1 * p.xmax, sqrtf(q2) * sqrtf(p.x2max)) * 1.001f;
    E *= (p.metric == METRIC_IP) ? S : 2.0f * S + p.x2max + q2;
    // FP16 operands: each factor within a relative 2^-11 (round to nearest
    // even) or an absolute 2^-25 (subnormals) of its FP32 value; the product
    // of two such within (2^-10 + 2^-22) |q_i x_i| + 2^-25 (1 + 2^-11)(|q_i| + |x_i|) + 2^-50
    const float eh = (0x1p-10f + 0x1p-22f) * S +
                     0x1p-25f * (1.0f + 0x1p-11f) * (a1 + (float)p.d * p.xmax) + (float)p.d * 0x1p-50f;
    E = (E * (1.0f + 0x1p-9f) + ((p.metric == METRIC_IP) ? eh : 2.0f * eh)) * (1.0f + 0x1p-16f);
  }
  float kth = __shfl(kx, 0, 64);
  for (int j = 0; j < 64; ++j) {
    const int rj = __shfl(rank, j, 64);
    if (rj == p.k - 1) kth = __shfl(kx, j, 64);
  }
  // every candidate not re-scored sorts after lk[R] (R < KC), and every row
  // outside the merged list after lk[KC - 1] (each range's list holds its
  // best KC, and the merged list the best KC of those)
  float thr = (R < KC) ? lk[R] : lk[KC - 1];
  if (p.metric != METRIC_IP) thr += q2;
  // a query beyond the FP16 range was saturated: no bound holds for it
  const bool in_range = !p.half || qm <= 65504.0f;
  if (lane == 0 && p.out_certified) p.out_certified[q] = in_range && (kth + E < thr) ? 1 : 0;
}

}  // namespace

// Base-row ranges per query block: the workgroups (query blocks x ranges)
// should fill whole rounds of the compute units.  Picks the smallest range
// count with the least time, counting time as rounds x rows per range, with
// ranges of at least 4 tiles.
static int bf_ranges(int64_t n, int64_t nq, int cu) {
  const int64_t qb = (nq + BM - 1) / BM;
  int best = 1;
  double best_t = 1e300;
  for (int r = 1; r <= 32; ++r) {
    if (r > 1 && n / r < 4 * BN) break;
    const int64_t rounds = (qb * r + cu - 1) / cu;
    const double t = (double)rounds * (double)((n + r - 1) / r);
    if (t < best_t * 0.99) { best_t = t; best = r; }
  }
  return best;
}

static size_t bruteforce_scratch_bytes(int64_t n, int64_t nq, int nranges) {
  return (size_t)nq * nranges * KC * 8 + (((size_t)n * 4 + 255) & ~size_t(255)) + 256;
}

}  // namespace ann

using namespace ann;

namespace {

// Checks shared by both entry points.
int bf_check(const ann_index* ix, const float* queries, int64_t nq, int32_t k, const int64_t* out_ids,
             const float* out_dists) {
  if (!ix) return fail(ANN_EINVAL, "index is NULL");
  if (!ix->x_f32) return fail(ANN_EUNSUP, "brute force needs the FP32 rows");
  if (k < 1 || k > KC - kRescore) return fail(ANN_EINVAL, "k %d outside [1, %d]", k, KC - kRescore);
  if (ix->d % 4 != 0) return fail(ANN_EUNSUP, "brute force needs d %% 4 == 0 (d=%d)", ix->d);
  if (nq < 0) return fail(ANN_EINVAL, "nq < 0");
  if (nq > 0 && (!queries || !out_ids || !out_dists)) return fail(ANN_EINVAL, "NULL pointer");
  return ANN_OK;
}

// The three kernels of one call, with the row norms (x2, written first when
// norms is set) and the candidate lists (ckey, cid) at the given addresses.
// With xh (the rows' FP16 copy), qh and hcert (scratch for the queries' FP16
// copy and the half pass's certificates), the half-precision pass runs first
// and the FP32 tiles redo only the queries it could not certify.
int bf_launch(const ann_index* ix, const float* queries, int64_t nq, int32_t k, int64_t* out_ids,
              float* out_dists, int32_t* out_certified, hipStream_t st, int nranges, float* x2,
              float* ckey, int32_t* cid, bool norms, const uint16_t* xh = nullptr,
              uint16_t* qh = nullptr, int32_t* hcert = nullptr, uint32_t* bound = nullptr) {
  if (norms) {
    hipLaunchKernelGGL(bf_norms, dim3((unsigned)ix->n), dim3(64), 0, st, ix->x_f32, ix->n, ix->d, x2);
    HIP_OR_RETURN(hipGetLastError(), "bf_norms launch");
  }
  BfParams p;
  p.X = ix->x_f32; p.x2 = x2; p.n = ix->n; p.d = ix->d; p.metric = ix->metric;
  p.Q = queries; p.nq = nq; p.nranges = nranges;
  p.rows_per_range = (ix->n + nranges - 1) / nranges;
  // bf_finish re-scores the best k + 16 of the merged lists and certifies
  // them against the next one, so each range needs its exact best k + 17
  // only: rows that do not beat the (k + 17)-th entry of their range's list
  // are not inserted (entries further down may then be stale).
  p.admit = std::min(KC, k + kRescore + 1);
  p.cand_key = ckey; p.cand_id = cid;
  p.redo = nullptr; p.Xh = nullptr; p.Qh = nullptr; p.bound = nullptr;
  const dim3 grid((unsigned)((nq + BM - 1) / BM), (unsigned)nranges);
  BfFinish f;
  f.X = ix->x_f32; f.n = ix->n; f.d = ix->d; f.metric = ix->metric; f.Q = queries; f.nq = nq;
  f.nranges = nranges; f.cand_key = ckey; f.cand_id = cid; f.k = k;
  f.xmax = ix->xmax; f.x2max = ix->x2max;
  f.out_ids = out_ids; f.out_dists = out_dists;
  if (xh) {
    const int64_t cnt = nq * ix->d;
    hipLaunchKernelGGL(bf_half, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 16384)), dim3(256), 0,
                       st, queries, cnt, qh);
    HIP_OR_RETURN(hipGetLastError(), "bf_half launch");
    p.Xh = xh; p.Qh = qh;
    // no bound yet for any query (the FP32 pass below keeps none: its keys
    // round differently)
    HIP_OR_RETURN(hipMemsetAsync(bound, 0xFF, (size_t)nq * 4, st), "hipMemsetAsync");
    p.bound = bound;
    hipLaunchKernelGGL(bf_tiles_h, grid, dim3(256), 0, st, p);
    HIP_OR_RETURN(hipGetLastError(), "bf_tiles_h launch");
    p.bound = nullptr;
    f.half = 1; f.redo = nullptr; f.out_certified = hcert;
    hipLaunchKernelGGL(bf_finish, dim3((unsigned)nq), dim3(64), 0, st, f);
    HIP_OR_RETURN(hipGetLastError(), "bf_finish launch");
    p.redo = hcert;
    f.redo = hcert;
  } else {
    f.redo = nullptr;
  }
  hipLaunchKernelGGL(bf_tiles, grid, dim3(256), 0, st, p);
  HIP_OR_RETURN(hipGetLastError(), "bf_tiles launch");
  f.half = 0; f.out_certified = out_certified;
  hipLaunchKernelGGL(bf_finish, dim3((unsigned)nq), dim3(64), 0, st, f);
  HIP_OR_RETURN(hipGetLastError(), "bf_finish launch");
  return ANN_OK;
}

// The rows' FP16 copy for the half-precision pass, made once per index; null
// (FP32 tiles only) when the rows do not suit it (d not a multiple of 8,
// values beyond the FP16 range) or the memory is not there.
const uint16_t* half_rows(ann_index* ix, hipStream_t st) {
  if (ix->d % 8 != 0 || !(ix->xmax < 65504.0f)) return nullptr;
  if (!ix->bf_xh) {
    const size_t bytes = (size_t)ix->n * ix->d * 2;
    if (hipMalloc(&ix->bf_xh, bytes) != hipSuccess) {
      (void)hipGetLastError();
      ix->bf_xh = nullptr;
      return nullptr;
    }
    const int64_t cnt = ix->n * ix->d;
    hipLaunchKernelGGL(bf_half, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 16384)), dim3(256), 0,
                       st, ix->x_f32, cnt, (uint16_t*)ix->bf_xh);
    if (hipGetLastError() != hipSuccess) {
      (void)hipFree(ix->bf_xh);
      ix->bf_xh = nullptr;
      return nullptr;
    }
  }
  return (const uint16_t*)ix->bf_xh;
}

}  // namespace

extern "C" int ann_bruteforce(const ann_index* cix, const float* queries, int64_t nq, int32_t k,
                              int64_t* out_ids, float* out_dists, int32_t* out_certified,
                              void* stream) {
  int rc = bf_check(cix, queries, nq, k, out_ids, out_dists);
  if (rc) return rc;
  if (nq == 0) return ANN_OK;
  ann_index* ix = const_cast<ann_index*>(cix);
  std::lock_guard<std::mutex> lock(ix->mu);
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  hipStream_t st = stream ? (hipStream_t)stream : ix->stream;
  const int nranges = bf_ranges(ix->n, nq, ix->cu_count > 0 ? ix->cu_count : 256);
  // the half pass's extra scratch: the queries' FP16 copy and its certificates
  const size_t half_extra = (((size_t)nq * ix->d * 2 + 255) & ~size_t(255)) + (((size_t)nq * 4 + 255) & ~size_t(255)) +
                            (size_t)nq * 4;
  const size_t need = bruteforce_scratch_bytes(ix->n, nq, nranges) + half_extra;
  if (!ix->bf_done)
    HIP_OR_RETURN(hipEventCreateWithFlags(&ix->bf_done, hipEventDisableTiming), "hipEventCreate");
  if (ix->bf_scratch_bytes < need) {
    if (ix->bf_scratch) {
      // the previous call (on whatever stream) is done with the old buffer
      if (ix->bf_used) HIP_OR_RETURN(hipEventSynchronize(ix->bf_done), "hipEventSynchronize");
      (void)hipFree(ix->bf_scratch);
      ix->bf_scratch = nullptr;
      ix->bf_scratch_bytes = 0;
    }
    HIP_OR_RETURN(hipMalloc(&ix->bf_scratch, need), "hipMalloc (brute-force scratch)");
    ix->bf_scratch_bytes = need;
    ix->bf_norms_ready = false;
  }
  // the scratch is shared by every call on this index: this call's kernels
  // start after the previous call's, whatever streams the two use
  if (ix->bf_used) HIP_OR_RETURN(hipStreamWaitEvent(st, ix->bf_done, 0), "hipStreamWaitEvent");
  char* base = (char*)ix->bf_scratch;
  float* x2 = (float*)base;
  float* ckey = (float*)(base + (((size_t)ix->n * 4 + 255) & ~size_t(255)));
  int32_t* cid = (int32_t*)(ckey + (size_t)nq * nranges * KC);
  uint16_t* qh = (uint16_t*)(base + bruteforce_scratch_bytes(ix->n, nq, nranges));
  int32_t* hcert = (int32_t*)((char*)qh + (((size_t)nq * ix->d * 2 + 255) & ~size_t(255)));
  uint32_t* bound = (uint32_t*)((char*)hcert + (((size_t)nq * 4 + 255) & ~size_t(255)));
  const uint16_t* xh = half_rows(ix, st);
  rc = bf_launch(ix, queries, nq, k, out_ids, out_dists, out_certified, st, nranges, x2, ckey, cid,
                 !ix->bf_norms_ready, xh, xh ? qh : nullptr, xh ? hcert : nullptr, xh ? bound : nullptr);
  if (rc) return rc;
  ix->bf_norms_ready = true;
  HIP_OR_RETURN(hipEventRecord(ix->bf_done, st), "hipEventRecord");
  ix->bf_used = true;
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "brute force");
  return ANN_OK;
}

// ---- the variant that allocates nothing ------------------------------------
//
// Its scratch (row norms and candidate lists) is a file-scope device array,
// one per GPU the library runs on, held until the process ends.  In host
// code `bf_static_scratch` names a host-side stand-in, not device memory:
// each device's address comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is handed to the
// kernels.
namespace {

__device__ __align__(256) char bf_static_scratch[ANN_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

// The device address of this device's array (the device must be current).
int static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(ANN_ENODEV, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(bf_static_scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress (static scratch)");
    g_static_ptr[device] = p;
  }
  *out = g_static_ptr[device];
  return ANN_OK;
}

}  // namespace

extern "C" int ann_bruteforce_noalloc(const ann_index* cix, const float* queries, int64_t nq,
                                      int32_t k, int64_t* out_ids, float* out_dists,
                                      int32_t* out_certified, void* stream) {
  int rc = bf_check(cix, queries, nq, k, out_ids, out_dists);
  if (rc) return rc;
  if (nq == 0) return ANN_OK;
  const ann_index* ix = cix;
  const int nranges = bf_ranges(ix->n, nq, ix->cu_count > 0 ? ix->cu_count : 256);
  const size_t need = bruteforce_scratch_bytes(ix->n, nq, nranges);
  if (need > (size_t)ANN_NOALLOC_SCRATCH_BYTES)
    return fail(ANN_EBUDGET, "%lld queries over %lld rows need %zu bytes of scratch, above the %d "
                "of ann_bruteforce_noalloc; split the batch", (long long)nq, (long long)ix->n, need,
                ANN_NOALLOC_SCRATCH_BYTES);
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  void* base_v = nullptr;
  if ((rc = static_scratch(ix->device, &base_v))) return rc;
  hipStream_t st = stream ? (hipStream_t)stream : ix->stream;
  char* base = (char*)base_v;
  float* x2 = (float*)base;
  float* ckey = (float*)(base + (((size_t)ix->n * 4 + 255) & ~size_t(255)));
  int32_t* cid = (int32_t*)(ckey + (size_t)nq * nranges * KC);
  // the array keeps whatever the last call left: the norms are recomputed
  // (L2 only), and every candidate list is written before it is read
  rc = bf_launch(ix, queries, nq, k, out_ids, out_dists, out_certified, st, nranges, x2, ckey, cid,
                 ix->metric != METRIC_IP);
  if (rc) return rc;
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "brute force");
  return ANN_OK;
}
