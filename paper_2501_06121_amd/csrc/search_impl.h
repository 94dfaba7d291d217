// Device code of the batched HNSW search on gfx950, included by one
// translation unit per storage mode (search_<mode>.hip), which instantiates
// the kernels.  Persistent grid: one workgroup of 1-8 wavefronts per query at
// a time, pulling query indices from a counter.
//
// What the workgroup does for one query (HNSW, the paper's index of Section 2
// and its citation's Algorithm 5):
//   1. query prep: the query's chunks into registers (dense), the PQ lookup
//      table into LDS, or the sparse query into an LDS hash table;
//   2. greedy descent through layers max_level..1 (ef = 1);
//   3. the layer-0 beam W of width ef, sorted by (key, id), with an
//      "expanded" bit per entry: repeatedly expand the best unexpanded entry,
//      gather its neighbour list, drop visited ids (a per-slot bitset in HBM),
//      gather and score the new rows, and merge them into W keeping the best
//      ef.  Under the (key, id) total order this is the citation's
//      Algorithm 2 with the candidate queue folded into W: the queue's minimum
//      is W's best unexpanded entry until none is left, which is exactly when
//      Algorithm 2 stops.  W is one sorted list, or a list plus a short
//      sorted insert buffer for wide beams (see "beam maintenance");
//   4. optional exact FP32 re-score of the first R entries of W;
//   5. the first k by (key, id) to the output rows.
//
// Every key uses the fixed FP32 order documented in include/ann.h, so the
// visited sets, the beam and the output are independent of the launch shape.
//
// Memory layout in HBM (written once by ann_index_create):
//   rows       n x d elements, row-major, 16-byte chunks
//   adj0       n x M0 i32, -1 padded (one 256-byte line for M0 = 64)
//   upper      per upper node, one M-wide list per level >= 1
//   bits       per slot, ceil(n / 32) u32 visited words
//   vlog       per slot, the ids set in `bits` (to clear them afterwards)
//   beam list  per slot, ef_cap keys and ids, when the list is kept in HBM
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "search_kernels.h"

namespace ann {

// 16-byte chunks each lane keeps in flight while scoring rows (4 VGPRs each).
#ifndef ANN_ROW_CHUNKS
#define ANN_ROW_CHUNKS 12
#endif

constexpr uint32_t kExpanded = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;
constexpr int kHashSlots = kSparseHashSlots;  // sparse query table (<= 256 terms)
constexpr int kTailCache = kListTailCache;    // entries of an HBM list's tail kept per wave
constexpr uint32_t kHashEmpty = 0xFFFFFFFFu;

// ----------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }
__device__ __forceinline__ int num_waves() { return (int)(blockDim.x >> 6); }

// Ordering point inside one wavefront: its LDS instructions execute in issue
// order, and the fence keeps the compiler from moving accesses across.  Used
// where only one wave of the workgroup runs (the other waves wait at a
// workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// strict (key, id) order; -0 and +0 compare equal, as in IEEE
__device__ __forceinline__ bool kid_lt(float ka, uint32_t ia, float kb, uint32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ float f16_bits_to_f32(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) {
  return __uint_as_float(h << 16);
}

// OCP E4M3: exponent bias 7, 3 mantissa bits; subnormals are m * 2^-9.
__device__ __forceinline__ float e4m3_bits_to_f32(uint32_t b) {
  const uint32_t em = b & 0x7Fu;
  const float mag = (em >= 8u) ? __uint_as_float((((em >> 3) + 120u) << 23) | ((em & 7u) << 20))
                               : (float)em * 0x1p-9f;
  return __uint_as_float(__float_as_uint(mag) | ((b & 0x80u) << 24));
}

// Cross-lane levels s = L/2 .. 1 of the fixed fold inside groups of L lanes:
// afterwards lane 0 of each group holds the group's sum.  At level s lane j
// (j < s) adds the value of lane j + s: DPP row shifts for s <= 8 (rows of 16
// lanes), a swizzle (xor 16 inside 32 lanes) for s = 16, a permute for s = 32.
template <int L>
__device__ __forceinline__ float fold_lanes(float v) {
  if constexpr (L >= 64) v = v + __shfl_down(v, 32, 64);
  if constexpr (L >= 32)
    v = v + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), (0x10 << 10) | 0x1F));
  if constexpr (L >= 16)
    v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x108, 0xF, 0xF, true));
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x104, 0xF, 0xF, true));
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x102, 0xF, 0xF, true));
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, true));
  return v;
}

// ----------------------------------------------------------------------------
// shared-memory layout of one wave (dynamic LDS)
// ----------------------------------------------------------------------------

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct Lds {
  float* wkey;       // [ef_cap]
  uint32_t* wid;     // [ef_cap] id | kExpanded
  int32_t* cid;      // [64] candidate ids of one expansion
  float* ckey;       // [64] their keys
  int32_t* rnk;      // [64] insertion ranks
  float* bkey;       // [wbuf] insert buffer of a large beam
  uint32_t* bid;     // [wbuf] id | kExpanded
  float* tck;        // [waves][kTailCache] per-wave copy of an HBM list's tail
  uint32_t* tci;     // [waves][kTailCache] (ids without the expanded bit)
  float* q;          // [d_pad] FP32 query (rerank, PQ tables)
  float* rk;         // [ef_cap] rerank keys
  float* lut;        // [pq_m * 256] PQ lookup table
  uint2* htab;       // [kHashSlots] sparse query terms: (term, weight bits)
  int64_t* sb;       // [64] sparse row extents of one expansion
  int64_t* se;       // [64]
  int32_t* ctl;      // [16] values wave 0 publishes to the other waves
};

// CTL_M and CTL_M_ODD carry an expansion's candidate counts, alternating by
// the parity of the expansion: a wave that has not yet read the count of one
// expansion (no barrier follows an expansion without new entries) never sees
// it overwritten by the next one.
enum { CTL_QUERY = 0, CTL_M = 1, CTL_W = 2, CTL_HINT = 3, CTL_VISITED = 4, CTL_VLOG = 5,
       CTL_VLOG_OVF = 6, CTL_FLUSH = 7, CTL_R0 = 8, CTL_M_ODD = 9, CTL_SEQ_LO = 10,
       CTL_SEQ_HI = 11, CTL_BACKOFF = 12 };

__device__ Lds carve(char* base, const SearchParams& p) {
  Lds s;
  size_t off = 0;
  auto take = [&](size_t bytes) { char* r = base + off; off += (bytes + 15) & ~size_t(15); return r; };
  const size_t list = p.glist ? 0 : (size_t)p.ef_cap;   // an HBM list takes no LDS
  s.wkey = (float*)take(sizeof(float) * list);
  s.wid = (uint32_t*)take(sizeof(uint32_t) * list);
  s.cid = (int32_t*)take(sizeof(int32_t) * 64);
  s.ckey = (float*)take(sizeof(float) * 64);
  s.rnk = (int32_t*)take(sizeof(int32_t) * 64);
  s.bkey = (float*)take(sizeof(float) * p.wbuf);
  s.bid = (uint32_t*)take(sizeof(uint32_t) * p.wbuf);
  const size_t tail = p.glist ? (size_t)kTailCache * p.waves_per_query : 0;
  s.tck = (float*)take(sizeof(float) * tail);
  s.tci = (uint32_t*)take(sizeof(uint32_t) * tail);
  s.q = (float*)take(sizeof(float) * p.q_lds_floats);
  s.rk = (float*)take(sizeof(float) * rerank_slots(p));
  s.lut = (float*)take(sizeof(float) * (p.mode == MODE_PQ ? p.pq_m * 256 : 0));
  s.htab = (uint2*)take(sizeof(uint2) * (p.mode == MODE_SPARSE ? kHashSlots : 0));
  s.sb = (int64_t*)take(sizeof(int64_t) * (p.mode == MODE_SPARSE ? 64 : 0));
  s.se = (int64_t*)take(sizeof(int64_t) * (p.mode == MODE_SPARSE ? 64 : 0));
  s.ctl = (int32_t*)take(sizeof(int32_t) * 16);
  return s;
}

// ----------------------------------------------------------------------------
// dense rows: chunk = 16 bytes; lane j of an L-lane group takes chunks
// g = j + L * t and feeds partial (g mod 64), held as virtual partial
// v = t mod (64 / L) of the lane.
// ----------------------------------------------------------------------------

template <int MODE> struct ElemsPerChunk;
template <> struct ElemsPerChunk<MODE_F32> { static constexpr int value = 4; };
template <> struct ElemsPerChunk<MODE_F16> { static constexpr int value = 8; };
template <> struct ElemsPerChunk<MODE_BF16> { static constexpr int value = 8; };
template <> struct ElemsPerChunk<MODE_FP8> { static constexpr int value = 16; };

template <int MODE>
__device__ __forceinline__ float chunk_elem(const uint4& r, int e) {
  const uint32_t w[4] = {r.x, r.y, r.z, r.w};
  if constexpr (MODE == MODE_F32) {
    return __uint_as_float(w[e]);
  } else if constexpr (MODE == MODE_F16) {
    return f16_bits_to_f32((w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
  } else if constexpr (MODE == MODE_BF16) {
    return bf16_bits_to_f32((w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
  } else {
    // gfx950 converts OCP E4M3 in hardware, exactly (checked against the
    // bit-level decode above on all 254 finite codes)
    const int word = (int)w[e >> 2];
    switch (e & 3) {             // the byte selector is an immediate operand
      case 0: return __builtin_amdgcn_cvt_f32_fp8(word, 0);
      case 1: return __builtin_amdgcn_cvt_f32_fp8(word, 1);
      case 2: return __builtin_amdgcn_cvt_f32_fp8(word, 2);
      default: return __builtin_amdgcn_cvt_f32_fp8(word, 3);
    }
  }
}

// One chunk folded into an accumulator, elements in ascending order.
template <int MODE, bool IP>
__device__ __forceinline__ float fold_chunk(float acc, const uint4& raw, const float* qc, float scale) {
  constexpr int C = ElemsPerChunk<MODE>::value;
#pragma unroll
  for (int e = 0; e < C; ++e) {
    float x = chunk_elem<MODE>(raw, e);
    if constexpr (IP) {
      acc = __builtin_fmaf(qc[e], x, acc);
    } else {
      if constexpr (MODE == MODE_FP8) x = scale * x;
      const float t = qc[e] - x;
      acc = __builtin_fmaf(t, t, acc);
    }
  }
  return acc;
}

// Dense scoring policy.  L lanes per row, CPL chunks per lane.
template <int MODE, int L, int CPL>
struct Dense {
  static constexpr int C = ElemsPerChunk<MODE>::value;
  static constexpr int G = 64 / L;          // rows per pass
  static constexpr int V = 64 / L;          // virtual partials per lane
  static constexpr int U = (ANN_ROW_CHUNKS / CPL) > 0 ? ANN_ROW_CHUNKS / CPL : 1;  // passes in flight
  float qreg[CPL][C];

  __device__ __forceinline__ bool prep(const SearchParams& p, const Lds& s, int64_t q) {
    const int j = lane_id() & (L - 1);
    const float* qrow = p.queries + (size_t)q * p.d;
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const int g = j + L * t;
#pragma unroll
      for (int e = 0; e < C; ++e) {
        const int i = g * C + e;
        qreg[t][e] = (g < p.nchunks) ? qrow[i] : 0.0f;
      }
    }
    return true;
  }

  // keys of the candidate rows s.cid[lo..hi) into s.ckey[lo..hi), by the
  // calling wave; row r is read at rows + r * 16 * nchunks (its FP8 scale at
  // scale[r])
  template <bool IP>
  __device__ __forceinline__ void score_impl(const SearchParams& p, const Lds& s, int lo, int hi,
                                             const void* rows_base, const float* scale_base) {
    const int lane = lane_id();
    const int j = lane & (L - 1);
    const int grp = lane / L;
    const size_t row_bytes = (size_t)p.nchunks * 16;
    const char* rows = (const char*)rows_base;
    for (int base = lo; base < hi; base += G * U) {
      uint4 raw[U][CPL];
      int rid[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int ci = base + u * G + grp;
        rid[u] = (ci < hi) ? s.cid[ci] : -1;
        const char* rp = rows + (size_t)(rid[u] < 0 ? 0 : rid[u]) * row_bytes;
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
          const int g = j + L * t;
          // rows are read once per query: streaming (nontemporal) loads
          // leave the caches to the lists and bitsets (+0.5% measured)
          if (rid[u] >= 0 && g < p.nchunks) {
            const u32x4 v = __builtin_nontemporal_load((const u32x4*)(rp + (size_t)g * 16));
            raw[u][t] = make_uint4(v[0], v[1], v[2], v[3]);
          } else {
            raw[u][t] = make_uint4(0u, 0u, 0u, 0u);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (base + u * G >= hi) break;
        const float scale = (MODE == MODE_FP8 && rid[u] >= 0) ? scale_base[rid[u]] : 1.0f;
        float acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0.0f;
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
          const int g = j + L * t;
          if (g < p.nchunks) acc[t % V] = fold_chunk<MODE, IP>(acc[t % V], raw[u][t], qreg[t], scale);
        }
        // tree levels s = 32 .. L inside the lane
#pragma unroll
        for (int h = V / 2; h >= 1; h >>= 1)
#pragma unroll
          for (int v = 0; v < h; ++v) acc[v] = acc[v] + acc[v + h];
        // levels s = L/2 .. 1 across the lanes of the group
        float val = fold_lanes<L>(acc[0]);
        const int ci = base + u * G + grp;
        if (j == 0 && ci < hi) {
          float key;
          if constexpr (IP) {
            if constexpr (MODE == MODE_FP8) val = scale * val;
            key = -val;
          } else {
            key = val;
          }
          s.ckey[ci] = key;
        }
      }
    }
  }

  // keys of the m candidate ids in s.cid[] into s.ckey[]; the waves of the
  // workgroup take contiguous shares of the rows
  __device__ __forceinline__ void score(const SearchParams& p, const Lds& s, int m) {
    const int per = (m + num_waves() - 1) / num_waves();
    const int lo = wave_id() * per;
    const int hi = lo + per < m ? lo + per : m;
    score_rows(p, s, lo, hi, p.rows, p.fp8_scale);
  }

  // the same for rows s.cid[lo..hi) of another row array, by the calling wave
  __device__ __forceinline__ void score_rows(const SearchParams& p, const Lds& s, int lo, int hi,
                                             const void* rows, const float* scale) {
    if (p.metric == METRIC_IP) score_impl<true>(p, s, lo, hi, rows, scale);
    else score_impl<false>(p, s, lo, hi, rows, scale);
  }
};

// ----------------------------------------------------------------------------
// PQ asymmetric distance: LUT[m][j] in LDS.  The key of a row is the fixed
// fold of its per-subspace entries p[m] = LUT[m][code_m] (m < 64, +0 beyond
// pq_m).  Two schedules give the same bits:
//   - few candidates (an HNSW expansion, about 6 new rows): L lanes per
//     candidate, lane j of a group holding the entries m = j + L v (one LDS
//     lookup each); the fold levels s >= L run in registers, the levels
//     s < L across the group's lanes;
//   - long runs (a 64-row chunk of an IVF list): one lane per candidate, all
//     64 entries and the whole fold in registers.
// ----------------------------------------------------------------------------

template <int L>
struct PQ {
  static constexpr int V = 64 / L;   // entries per lane
  static constexpr int G = 64 / L;   // candidates per pass of the wave
  static constexpr int U = 2;        // passes whose codes are in flight together

  __device__ __forceinline__ bool prep(const SearchParams& p, const Lds& s, int64_t q) {
    const int ds = p.pq_dsub;
    const int entries = p.pq_m * 256;
    const bool ip = p.metric == METRIC_IP;
    for (int e = threadIdx.x; e < entries; e += blockDim.x) {
      const int m = e >> 8;
      const float* c = p.pq_cb + (size_t)e * ds;
      const float* qs = s.q + m * ds;
      float acc = 0.0f;
      for (int t = 0; t < ds; ++t) {
        if (ip) {
          acc = __builtin_fmaf(qs[t], c[t], acc);
        } else {
          const float u = qs[t] - c[t];
          acc = __builtin_fmaf(u, u, acc);
        }
      }
      s.lut[e] = acc;
    }
    __syncthreads();
    return true;
  }

  // candidates s.cid[lo..hi) by the calling wave, one lane each
  __device__ __forceinline__ void score_lanes(const SearchParams& p, const Lds& s, int lo, int hi) {
    for (int ci = lo + lane_id(); ci < hi; ci += 64) {
      const int64_t r = s.cid[ci];
      const uint4* cp = (const uint4*)(p.pq_codes + (size_t)r * p.pq_stride);
      float part[64];
      uint4 w4[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) w4[b] = (b * 16 < p.pq_m) ? cp[b] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (int mm = 0; mm < 64; ++mm) {
        const uint4 w = w4[mm >> 4];
        const uint32_t word = ((mm >> 2) & 3) == 0 ? w.x : ((mm >> 2) & 3) == 1 ? w.y
                              : ((mm >> 2) & 3) == 2 ? w.z : w.w;
        const uint32_t code = (word >> (8 * (mm & 3))) & 0xFFu;
        part[mm] = (mm < p.pq_m) ? s.lut[mm * 256 + code] : 0.0f;
      }
#pragma unroll
      for (int h = 32; h >= 1; h >>= 1)
#pragma unroll
        for (int v = 0; v < h; ++v) part[v] = part[v] + part[v + h];
      s.ckey[ci] = (p.metric == METRIC_IP) ? -part[0] : part[0];
    }
  }

  // candidates s.cid[lo..hi) by the calling wave, L lanes each
  __device__ __forceinline__ void score_groups(const SearchParams& p, const Lds& s, int lo, int hi) {
    const int lane = lane_id();
    const int j = lane & (L - 1);
    const int grp = lane / L;
    for (int base = lo; base < hi; base += G * U) {
      uint32_t code[U][V];
      int rid[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int ci = base + u * G + grp;
        rid[u] = (ci < hi) ? s.cid[ci] : -1;
        const uint8_t* cp = p.pq_codes + (size_t)(rid[u] < 0 ? 0 : rid[u]) * p.pq_stride;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          // unconditional (row 0, entry 0 where there is none; the code is
          // then not used), so that the loads stay in flight together
          const int m = j + L * v;
          code[u][v] = (uint32_t)cp[m < p.pq_m ? m : 0];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (base + u * G >= hi) break;
        float acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int m = j + L * v;
          acc[v] = (rid[u] >= 0 && m < p.pq_m) ? s.lut[m * 256 + (int)code[u][v]] : 0.0f;
        }
        // levels s = 32 .. L inside the lane, then s = L/2 .. 1 across the group
#pragma unroll
        for (int h = V / 2; h >= 1; h >>= 1)
#pragma unroll
          for (int v = 0; v < h; ++v) acc[v] = acc[v] + acc[v + h];
        const float val = fold_lanes<L>(acc[0]);
        const int ci = base + u * G + grp;
        if (j == 0 && ci < hi) s.ckey[ci] = (p.metric == METRIC_IP) ? -val : val;
      }
    }
  }

  // keys of the m candidate ids in s.cid[] into s.ckey[]; the waves of the
  // workgroup take contiguous shares
  __device__ __forceinline__ void score(const SearchParams& p, const Lds& s, int m) {
    const int per = (m + num_waves() - 1) / num_waves();
    const int lo = wave_id() * per;
    const int hi = lo + per < m ? lo + per : m;
    if (hi - lo > 16) score_lanes(p, s, lo, hi);
    else if (hi > lo) score_groups(p, s, lo, hi);
  }
};

// ----------------------------------------------------------------------------
// Sparse inner product: the query in an LDS hash table, 64 lanes per document
// (position j of the document feeds partial j mod 64).
// ----------------------------------------------------------------------------

__device__ __forceinline__ uint32_t hash_slot(uint32_t t) {
  return (t * 2654435761u) >> (32 - 9);
}

struct Sparse {
  __device__ __forceinline__ bool prep(const SearchParams& p, const Lds& s, int64_t q) {
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) s.htab[i] = make_uint2(kHashEmpty, 0u);
    __syncthreads();
    const int64_t b = p.q_ptr[q];
    int64_t e = p.q_ptr[q + 1];
    const bool ok = e - b <= kHashSlots / 2;
    if (!ok) e = b + kHashSlots / 2;     // keeps the table at most half full
    for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) {
      const uint32_t t = p.q_ids[j];
      const float w = p.q_vals[j];
      uint32_t h = hash_slot(t);
      while (true) {
        const uint32_t prev = atomicCAS(&s.htab[h].x, kHashEmpty, t);
        if (prev == kHashEmpty || prev == t) { s.htab[h].y = __float_as_uint(w); break; }
        h = (h + 1) & (kHashSlots - 1);
      }
    }
    __syncthreads();
    return ok;
  }

  // The weight of term t when its first probe, slot h, held another term:
  // the probe walks on to t or to an empty slot (0: t is not in the query).
  __device__ __forceinline__ float weight_after(const Lds& s, uint32_t t, uint32_t h) const {
    while (true) {
      h = (h + 1) & (kHashSlots - 1);
      const uint2 e = s.htab[h];
      if (e.x == t) return __uint_as_float(e.y);
      if (e.x == kHashEmpty) return 0.0f;
    }
  }

  __device__ __forceinline__ void score(const SearchParams& p, const Lds& s, int m) {
    const int lane = lane_id();
    constexpr int U = 8;   // documents in flight
    // every candidate's extent in one round trip
    if ((int)threadIdx.x < m) {
      const int64_t r = s.cid[threadIdx.x];
      s.sb[threadIdx.x] = p.sp_ptr[r];
      s.se[threadIdx.x] = p.sp_ptr[r + 1];
    }
    __syncthreads();
    const int per = (m + num_waves() - 1) / num_waves();
    const int lo = wave_id() * per;
    const int hi = lo + per < m ? lo + per : m;
    for (int base = lo; base < hi; base += U) {
      float acc[U];
      int64_t b[U], e[U];
      int64_t most = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc[u] = 0.0f;
        const int ci = base + u;
        b[u] = (ci < hi) ? s.sb[ci] : 0;
        e[u] = (ci < hi) ? s.se[ci] : 0;
        most = (e[u] - b[u] > most) ? e[u] - b[u] : most;
      }
      for (int64_t off = lane; off < most; off += 64) {
        uint32_t tid[U];
        float val[U];
        // every load is issued unconditionally (past a document's end it
        // reads a valid entry that is then ignored): loads under a per-lane
        // condition are each waited for on the spot, which kept only one
        // document's entries in flight
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = b[u] + off;
          const int64_t jc = j < e[u] ? j : (e[u] > b[u] ? e[u] - 1 : 0);
          tid[u] = (uint32_t)p.sp_ids[jc];
          val[u] = p.sp_vals[jc];
        }
        // the first probe of every document's term at once (one LDS wait,
        // not one per document); only a collision walks on
        uint32_t hs[U];
        uint2 ent[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          hs[u] = hash_slot(tid[u]);
          ent[u] = s.htab[hs[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (b[u] + off < e[u]) {
            float w = ent[u].x == tid[u] ? __uint_as_float(ent[u].y) : 0.0f;
            if (ent[u].x != tid[u] && ent[u].x != kHashEmpty) w = weight_after(s, tid[u], hs[u]);
            acc[u] = __builtin_fmaf(w, val[u], acc[u]);
          }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (base + u >= hi) break;
        const float val = fold_lanes<64>(acc[u]);
        if (lane == 0) s.ckey[base + u] = -val;
      }
    }
  }
};

// ----------------------------------------------------------------------------
// beam maintenance
//
// The beam W is the best ef entries seen so far, each (key, id | kExpanded).
// Small beams are one sorted list.  Large beams add a sorted insert buffer
// in LDS (bkey/bid, capacity p.wbuf): new entries are merged into the short
// buffer, and the buffer into the long list only when it fills, so that an
// expansion moves O(wbuf) entries instead of O(ef).  W is then the best ef
// entries of list and buffer together; the worse ones are cut from the two
// tails as soon as they fall out.  The list lives in LDS, or, for beams too
// wide to keep several queries per compute unit, in a per-slot HBM array
// (every access is then a global one; the buffer stays in LDS).  All layouts
// hold the same W.
// ----------------------------------------------------------------------------

// The sorted list [0, w) of a beam, in LDS or in HBM.
struct List {
  float* key;
  uint32_t* id;
};

// first entry of ids[0, w) at or after `from` without the expanded bit, or -1
__device__ int next_unexpanded(const uint32_t* ids, int from, int w) {
  for (int j0 = from; j0 < w; j0 += 64) {
    const int j = j0 + lane_id();
    const bool un = j < w && !(ids[j] & kExpanded);
    const uint64_t mk = ballot(un);
    if (mk) return j0 + __builtin_ctzll(mk);
  }
  return -1;
}

// number of entries of a sorted run keys/ids[0, n) strictly below (k, id)
// (the ids may carry the expanded bit)
__device__ __forceinline__ int count_below(const float* keys, const uint32_t* ids, int n, float k,
                                           uint32_t id) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kid_lt(keys[mid], ids[mid] & kIdMask, k, id)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Merge the sorted run nkey/nid[0, mnew) (mnew >= 1, no entry equal to one
// of the list) into the sorted list dkey/did[0, w), in place, keeping the
// first `cap`; every thread of the workgroup takes part.
//
// With a_j = #{new < old_j}, old entry j moves to j + a_j and the new entries
// i in [a_j, a_{j+1}) land at j + 1 + i (a_w = mnew); new entries below old
// entry 0 stay at i.  Each thread owns E consecutive old entries of a chunk
// of E x nthr; chunks go from the highest down, each read completely (with
// the entry just above it) before it is written.  Writes of a chunk land at
// or above its own entries' positions, so nothing a lower chunk still reads
// is overwritten, and the entry above a chunk is read back unchanged.  The
// walk stops at the chunk holding the place of the smallest new entry; the
// entries below it do not move.
//
// *r0 receives the position of new entry 0.  When `hint` is given it is a
// position of the list before which every entry is expanded, and on return a
// position of the merged list with the same property: the smallest of where
// old entry *hint went and where each new entry without the expanded bit
// went (tracked with atomicMin in *hmin, which must hold INT32_MAX).
// Returns the new size.
template <int E>
__device__ __forceinline__ int merge_sorted(float* dkey, uint32_t* did, int w, int cap, const float* nkey,
                            const uint32_t* nid, int mnew, int32_t* r0, int* hint, int32_t* hmin) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int h = hint ? *hint : 0;
  int lowest = w;
  if (w == 0) {
    for (int i = tid; i < mnew && i < cap; i += nthr) {
      dkey[i] = nkey[i];
      did[i] = nid[i];
      if (hint && !(nid[i] & kExpanded)) atomicMin(hmin, i);
    }
    if (tid == 0) *r0 = 0;
    __syncthreads();
  } else {
    const float k0 = nkey[0];
    const uint32_t i0 = nid[0] & kIdMask;
    const int CH = E * nthr;
    for (int j0 = ((w - 1) / CH) * CH; j0 >= 0; j0 -= CH) {
      const int jb = j0 + tid * E;
      float ok[E];
      uint32_t oi[E];
      int a[E + 1];
      // read unconditionally (entry w - 1 past the end; those values are
      // not used), so that the reads are waited for together, not one by one
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int jj = jb + e < w ? jb + e : w - 1;
        ok[e] = dkey[jj];
        oi[e] = did[jj];
      }
      const bool has_next = jb + E < w;
      const float nk = dkey[has_next ? jb + E : w - 1];
      const uint32_t ni = did[has_next ? jb + E : w - 1] & kIdMask;
      // a[e]: new entries below old entry jb + e; a[E]: below the entry after the block
      int c = jb < w ? count_below(nkey, nid, mnew, ok[0], oi[0] & kIdMask) : 0;
      a[0] = c;
#pragma unroll
      for (int e = 1; e < E; ++e) {
        if (jb + e < w)
          while (c < mnew && kid_lt(nkey[c], nid[c] & kIdMask, ok[e], oi[e] & kIdMask)) ++c;
        a[e] = c;
      }
      if (has_next) {
        while (c < mnew && kid_lt(nkey[c], nid[c] & kIdMask, nk, ni)) ++c;
        a[E] = c;
      } else {
        a[E] = mnew;
      }
      const bool more = j0 > 0 && !kid_lt(dkey[j0], did[j0] & kIdMask, k0, i0);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int j = jb + e;
        if (j < w) {
          const int ae = a[e];
          const int be = j + 1 < w ? a[e + 1] : mnew;
          if (j + ae < cap) { dkey[j + ae] = ok[e]; did[j + ae] = oi[e]; }
          if (hint && j == h) atomicMin(hmin, j + ae);
          for (int i = ae; i < be; ++i) {
            const int pos = j + 1 + i;
            if (pos < cap) {
              dkey[pos] = nkey[i];
              did[pos] = nid[i];
              if (hint && !(nid[i] & kExpanded)) atomicMin(hmin, pos);
            }
          }
          if (ae == 0 && be > 0) *r0 = j + 1;
          if (j == 0) {
            for (int i = 0; i < ae && i < cap; ++i) {
              dkey[i] = nkey[i];
              did[i] = nid[i];
              if (hint && !(nid[i] & kExpanded)) atomicMin(hmin, i);
            }
            if (ae > 0) *r0 = 0;
          }
        }
      }
      __syncthreads();
      lowest = j0;
      if (!more) break;
    }
  }
  const int nw = w + mnew < cap ? w + mnew : cap;
  if (hint) {
    int hm = *hmin;
    if (h >= w) hm = hm < w + mnew ? hm : w + mnew;   // every old entry was expanded
    else if (h < lowest) hm = hm < h ? hm : h;         // old entry h did not move
    *hint = hm < nw ? hm : nw;
  }
  return nw;
}

// Merge the sorted list skey/sid[0, w) and the sorted run nkey/nid[0, mnew)
// into another array dkey/did, keeping the first `cap` (the buffer flush of a
// beam list in HBM, which alternates between two arrays).  The placement is
// that of merge_sorted; source and destination differ, so no chunk order is
// needed: each thread walks its blocks of E entries (stride E x nthr) with
// the next block's loads in flight.  `hint` is carried over as in
// merge_sorted (*hmin must hold INT32_MAX).  Returns the new size.
template <int E>
__device__ __forceinline__ int merge_copy(const float* skey, const uint32_t* sid, int w, float* dkey,
                                          uint32_t* did, int cap, const float* nkey,
                                          const uint32_t* nid, int mnew, int* hint, int32_t* hmin) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int h = *hint;
  const int stride = E * nthr;
  // new entries below old entry 0 (all of them when the list is empty)
  const int below0 = w > 0 ? count_below(nkey, nid, mnew, skey[0], sid[0] & kIdMask) : mnew;
  for (int i = tid; i < below0 && i < cap; i += nthr) {
    dkey[i] = nkey[i];
    did[i] = nid[i];
    if (!(nid[i] & kExpanded)) atomicMin(hmin, i);
  }
  float ok[E], pk[E];
  uint32_t oi[E], pi[E];
  float nk = 0.0f, qk = 0.0f;
  uint32_t ni = 0u, qi = 0u;
  auto load = [&](int jb, float* k, uint32_t* id, float& ek, uint32_t& ei) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      k[e] = 0.0f;
      id[e] = 0u;
      if (jb + e < w) { k[e] = skey[jb + e]; id[e] = sid[jb + e]; }
    }
    ek = 0.0f;
    ei = 0u;
    if (jb + E < w) { ek = skey[jb + E]; ei = sid[jb + E] & kIdMask; }
  };
  int jb = tid * E;
  if (jb < w) load(jb, ok, oi, nk, ni);
  for (; jb < w; jb += stride) {
    const bool more = jb + stride < w;
    if (more) load(jb + stride, pk, pi, qk, qi);
    int c = count_below(nkey, nid, mnew, ok[0], oi[0] & kIdMask);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = jb + e;
      if (j < w) {
        const int ae = c;
        int be = mnew;                    // new entries below old entry j + 1
        if (j + 1 < w) {
          const float k1 = e + 1 < E ? ok[e + 1] : nk;
          const uint32_t i1 = (e + 1 < E ? oi[e + 1] : ni) & kIdMask;
          be = c;
          while (be < mnew && kid_lt(nkey[be], nid[be] & kIdMask, k1, i1)) ++be;
        }
        if (j + ae < cap) { dkey[j + ae] = ok[e]; did[j + ae] = oi[e]; }
        if (j == h) atomicMin(hmin, j + ae);
        for (int i = ae; i < be; ++i) {
          const int pos = j + 1 + i;
          if (pos < cap) {
            dkey[pos] = nkey[i];
            did[pos] = nid[i];
            if (!(nid[i] & kExpanded)) atomicMin(hmin, pos);
          }
        }
        c = be;
      }
    }
    if (more) {
#pragma unroll
      for (int e = 0; e < E; ++e) { ok[e] = pk[e]; oi[e] = pi[e]; }
      nk = qk;
      ni = qi;
    }
  }
  __syncthreads();
  const int nw = w + mnew < cap ? w + mnew : cap;
  int hm = *hmin;
  if (h >= w) hm = hm < w + mnew ? hm : w + mnew;   // every old entry was expanded
  *hint = hm < nw ? hm : nw;
  return nw;
}

// State of the beam at the start of an expansion.
struct Head {
  int pm, pb;         // first unexpanded entry of the list / of the buffer, or -1
  float mk;           // key and id of list entry pm
  uint32_t mi;
  float tk;           // worst entry of W (meaningful when W holds ef entries)
  uint32_t ti;
};

// What a wave keeps of a beam list in HBM between expansions.  Between buffer
// flushes the list only loses entries at its end (cuts) and gains expanded
// bits before the scan position, so a window of 64 entries from the scan
// position (in registers, lane l holding entry wh + l) and a copy of the last
// kTailCache entries (in the wave's LDS, from entry tw on) stay valid until
// the scan leaves the window or the cuts reach the copy's start.  A flush
// rewrites the list: both are then marked stale.
struct ListCache {
  int wh;          // list position of the window's lane 0, -1 when stale
  int tw;          // list position of the tail copy's entry 0, -1 when stale
  float fk;        // this lane's window entry
  uint32_t fi;
};

// Cuts W to the best ef entries of list [0, w) and buffer [0, wb) (buffered
// beams; at most 64 entries fall out per expansion), and finds the first
// unexpanded entries and the worst entry of W.  Lane x tests the cut "x
// entries from the list, d - x from the buffer", of which exactly one keeps
// every kept entry below every dropped one; it needs list entries w - 1 - x,
// which an LDS list provides directly and an HBM list through the wave's
// caches (refilled in one round trip when they run out).  Every wave computes
// the same result; nothing shared is written.
template <bool GLIST>
__device__ __forceinline__ Head beam_head(const Lds& s, List L, int& w, int& wb, int ef, int hint,
                                          int hint_b, bool buffered, ListCache& lc) {
  const int lane = lane_id();
  const int tj = w - 1 - lane;
  float tk = __builtin_inff();
  uint32_t ti = kIdMask;
  int fj;
  float fk;
  uint32_t fi;
  if constexpr (GLIST) {
    float* ck = s.tck + wave_id() * kTailCache;
    uint32_t* ci = s.tci + wave_id() * kTailCache;
    if (lc.tw < 0 || w - 64 < lc.tw) {
      const int tw = w > kTailCache ? w - kTailCache : 0;
#pragma unroll
      for (int r = 0; r < kTailCache / 64; ++r) {
        const int j = tw + lane + 64 * r;
        if (j < w) { ck[j - tw] = L.key[j]; ci[j - tw] = L.id[j] & kIdMask; }
      }
      lc.tw = tw;
      wave_sync();
    }
    if (tj >= 0) { tk = ck[tj - lc.tw]; ti = ci[tj - lc.tw]; }
    if (lc.wh < 0 || hint < lc.wh || hint >= lc.wh + 64) {
      lc.wh = hint;
      lc.fk = 0.0f;
      lc.fi = kExpanded;
      if (hint + lane < w) { lc.fk = L.key[hint + lane]; lc.fi = L.id[hint + lane]; }
    }
    fj = lc.wh + lane;
    fk = lc.fk;
    fi = lc.fi;
  } else {
    if (tj >= 0) { tk = L.key[tj]; ti = L.id[tj] & kIdMask; }
    fj = hint + lane;
    fk = 0.0f;
    fi = kExpanded;
    if (fj < w) { fk = L.key[fj]; fi = L.id[fj]; }
  }
  int xs = 0;
  if (buffered && w + wb > ef) {
    const int d = w + wb - ef;
    const int x = lane;
    const int y = d - x;
    const float pk = __shfl_up(tk, 1, 64);              // list[w - x] from lane x - 1
    const uint32_t pi = (uint32_t)__shfl_up((int)ti, 1, 64);
    bool ok = x <= d && x <= w && y <= wb;
    if (ok && w - x >= 1 && y >= 1) ok = kid_lt(tk, ti, s.bkey[wb - y], s.bid[wb - y] & kIdMask);
    if (ok && wb - y >= 1 && x >= 1) ok = kid_lt(s.bkey[wb - y - 1], s.bid[wb - y - 1] & kIdMask, pk, pi);
    const uint64_t mk = ballot(ok);
    xs = mk ? __builtin_ctzll(mk) : 64;                  // only d = 64 can need x = 64
    w -= xs;
    wb -= d - xs;
  }
  Head hd;
  hd.tk = __builtin_inff();
  hd.ti = kIdMask;
  if (w > 0) {
    if (xs < 64) {
      hd.tk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tk), xs));
      hd.ti = (uint32_t)__builtin_amdgcn_readlane((int)ti, xs);
    } else {
      hd.tk = L.key[w - 1];
      hd.ti = L.id[w - 1] & kIdMask;
    }
  }
  if (wb > 0) {
    const float bk = s.bkey[wb - 1];
    const uint32_t bi = s.bid[wb - 1] & kIdMask;
    if (w == 0 || kid_lt(hd.tk, hd.ti, bk, bi)) { hd.tk = bk; hd.ti = bi; }
  }
  const uint64_t um = ballot(fj >= hint && fj < w && !(fi & kExpanded));
  hd.pm = -1;
  hd.mk = 0.0f;
  hd.mi = 0u;
  if (um) {
    const int l = __builtin_ctzll(um);
    hd.pm = fj - lane + l;
    hd.mk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fk), l));
    hd.mi = (uint32_t)__builtin_amdgcn_readlane((int)fi, l) & kIdMask;
  } else if (fj - lane + 64 < w) {
    // nothing unexpanded in the window: scan on (the window moves with the scan position)
    hd.pm = next_unexpanded(L.id, fj - lane + 64, w);
    if (hd.pm >= 0) { hd.mk = L.key[hd.pm]; hd.mi = L.id[hd.pm] & kIdMask; }
    if constexpr (GLIST) lc.wh = -1;
  }
  hd.pb = buffered ? next_unexpanded(s.bid, hint_b, wb) : -1;
  return hd;
}

// ----------------------------------------------------------------------------
// the search kernel
// ----------------------------------------------------------------------------

struct QueryState {
  int evals, expansions, visited;
  int vlog_n;
  bool vlog_overflow;
};

__device__ __forceinline__ void log_visited(const SearchParams& p, int slot, int64_t q,
                                            QueryState& st, bool isnew, int id, uint64_t mask) {
  const int idx = mbcnt(mask);
  if (isnew) {
    const int pos = st.vlog_n + idx;
    if (pos < p.vlog_cap) p.vlog[(size_t)slot * p.vlog_cap + pos] = id;
    const int vpos = st.visited + idx;
    if (p.out_visited && vpos < p.visited_cap) p.out_visited[q * p.visited_cap + vpos] = id;
  }
  const int cnt = __builtin_popcountll(mask);
  if (st.vlog_n + cnt > p.vlog_cap) st.vlog_overflow = true;
  st.vlog_n += cnt;
  st.visited += cnt;
}

// ---- invariant checks (builds with ANN_DEBUG_CHECKS only) ------------------
//
// The beam's invariants, checked by the whole workgroup between expansions;
// a violation sets a bit of *p.debug (never a trap):
//   1  |W| = w + wb above ef (after the cut), or a length outside its array
//   2  the list L[0, w) not strictly ascending in (key, id)
//   4  the insert buffer B[0, wb) not strictly ascending in (key, id)
//   8  an id outside [0, n)
//  16  an entry before the scan position (hint, hint_b) not expanded
//  32  an expansion's candidate counts out of range (m > 64 or kept > m)
// Strict order under (key, id) also makes the ids of each array unique.
enum { kDbgSize = 1, kDbgListOrder = 2, kDbgBufOrder = 4, kDbgId = 8, kDbgHint = 16, kDbgCount = 32 };

__device__ __forceinline__ void debug_flag(const SearchParams& p, uint32_t bits) {
#ifdef ANN_DEBUG_CHECKS
  if (bits && p.debug) atomicOr(p.debug, bits);
#else
  (void)p;
  (void)bits;
#endif
}

template <bool GLIST>
__device__ void debug_check_beam(const SearchParams& p, const Lds& s, const List& L, int w, int wb,
                                 int ef, int hint, int hint_b) {
#ifdef ANN_DEBUG_CHECKS
  __syncthreads();
  uint32_t bad = 0;
  const int wcap = p.wbuf > 0 ? p.wbuf : 0;
  if (w < 0 || wb < 0 || w > p.ef_cap || wb > wcap || w + wb > ef) bad |= kDbgSize;
  const int wl = w < p.ef_cap ? w : p.ef_cap;
  const int bl = wb < wcap ? wb : wcap;
  for (int i = threadIdx.x; i < wl; i += blockDim.x) {
    const uint32_t id = L.id[i] & kIdMask;
    if (id >= (uint64_t)p.n) bad |= kDbgId;
    if (i + 1 < wl && !kid_lt(L.key[i], id, L.key[i + 1], L.id[i + 1] & kIdMask)) bad |= kDbgListOrder;
    if (i < hint && !(L.id[i] & kExpanded)) bad |= kDbgHint;
  }
  for (int i = threadIdx.x; i < bl; i += blockDim.x) {
    const uint32_t id = s.bid[i] & kIdMask;
    if (id >= (uint64_t)p.n) bad |= kDbgId;
    if (i + 1 < bl && !kid_lt(s.bkey[i], id, s.bkey[i + 1], s.bid[i + 1] & kIdMask)) bad |= kDbgBufOrder;
    if (i < hint_b && !(s.bid[i] & kExpanded)) bad |= kDbgHint;
  }
  debug_flag(p, bad);
  __syncthreads();
#else
  (void)p; (void)s; (void)L; (void)w; (void)wb; (void)ef; (void)hint; (void)hint_b;
#endif
}

template <class Policy, bool GLIST>
__device__ __forceinline__ void run_query(const SearchParams& p, const Lds& s, Policy& pol, int slot, int64_t q) {
  const int lane = lane_id();
  const int wave = wave_id();
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  int k = p.k_arr ? p.k_arr[q] : p.k_all;
  int ef = p.ef_arr ? p.ef_arr[q] : p.ef_all;
  int status = 0;
  if (k > p.k_max) { k = p.k_max; status = 1; }
  if (k < 1) { k = 1; status = 1; }
  if (ef < k) ef = k;
  if (ef > p.ef_cap) { ef = p.ef_cap; status = 1; }
  k = uniform_int(k);
  ef = uniform_int(ef);

  // FP32 query copy in LDS for the rerank and the PQ tables
  if (p.q_lds_floats > 0 && p.queries) {
    const float* qrow = p.queries + (size_t)q * p.d;
    for (int i = tid; i < p.q_lds_floats; i += nthr) s.q[i] = (i < p.d) ? qrow[i] : 0.0f;
  }
  __syncthreads();
  if (!pol.prep(p, s, q)) status |= 2;

  // Wave 0 owns the visited bits and the log; every wave counts evaluations.
  QueryState st{0, 0, 0, 0, false};
  uint32_t* bits = p.bits + (size_t)slot * p.bits_words;

  // entry point
  int cur = p.entry;
  if (tid == 0) s.cid[0] = cur;
  __syncthreads();
  pol.score(p, s, 1);
  __syncthreads();
  float ckey = s.ckey[0];
  st.evals += 1;

  // greedy descent, layers max_level .. 1 (every wave computes the same
  // neighbour list and minimum; the rows are scored by all waves)
  for (int lc = p.max_level; lc >= 1; --lc) {
    while (true) {
      const int off = p.upper_off[cur];
      int nb = -1;
      if (lane < p.M && off >= 0) nb = p.upper_adj[((size_t)off + lc - 1) * p.M + lane];
      const uint64_t mk = ballot(nb >= 0);
      const int m = __builtin_popcountll(mk);
      if (m == 0) break;
      if (nb >= 0) s.cid[mbcnt(mk)] = nb;
      __syncthreads();
      pol.score(p, s, m);
      __syncthreads();
      st.evals += m;
      float bk = (lane < m) ? s.ckey[lane] : __builtin_inff();
      uint32_t bi = (lane < m) ? (uint32_t)s.cid[lane] : kIdMask;
#pragma unroll
      for (int sft = 32; sft >= 1; sft >>= 1) {
        const float ok = __shfl_xor(bk, sft, 64);
        const uint32_t oi = (uint32_t)__shfl_xor((int)bi, sft, 64);
        if (kid_lt(ok, oi, bk, bi)) { bk = ok; bi = oi; }
      }
      __syncthreads();
      if (kid_lt(bk, bi, ckey, (uint32_t)cur)) {
        cur = uniform_int((int)bi);
        ckey = __builtin_bit_cast(float, uniform_int(__builtin_bit_cast(int, bk)));
      } else {
        break;
      }
    }
  }

  // layer 0
  if (wave == 0) {
    const uint32_t bit = 1u << (cur & 31);
    uint32_t old = 0;
    if (lane == 0) old = atomicOr(&bits[cur >> 5], bit);
    const bool isnew = (lane == 0) && !(old & bit);
    log_visited(p, slot, q, st, isnew, cur, ballot(isnew));
  }
  // the beam list; an HBM list has two arrays per slot and a flush writes
  // the merged list into the other one (L2)
  List L, L2;
  if constexpr (GLIST) {
    L.key = p.glist_key + (size_t)slot * 2 * p.ef_cap;
    L.id = p.glist_id + (size_t)slot * 2 * p.ef_cap;
    L2.key = L.key + p.ef_cap;
    L2.id = L.id + p.ef_cap;
  } else {
    L.key = s.wkey;
    L.id = s.wid;
    L2 = L;
  }
  if (tid == 0) { L.key[0] = ckey; L.id[0] = (uint32_t)cur; }
  __syncthreads();
  // list [0, w) and, for a large beam, insert buffer [0, wb); every entry
  // before hint (list) or hint_b (buffer) is expanded
  const bool buffered = GLIST || (p.wbuf > 0 && ef > p.wbuf_min_ef);
  int w = 1, wb = 0;
  int hint = 0, hint_b = 0;
  ListCache lc{-1, -1, 0.0f, kExpanded};
  while (true) {
    // (the sizes before the cut may exceed ef by one expansion's entries)
    debug_check_beam<GLIST>(p, s, L, w, wb, w + wb > ef ? w + wb : ef, hint, hint_b);
    // cut to ef, best unexpanded entry and worst entry of W (all waves
    // compute them from the same state)
    const Head hd = beam_head<GLIST>(s, L, w, wb, ef, hint, hint_b, buffered, lc);
    debug_check_beam<GLIST>(p, s, L, w, wb, ef, 0, 0);
    const int pm = hd.pm, pb = hd.pb;
    if (pm < 0 && pb < 0) break;
    const bool from_buf = pb >= 0 && (pm < 0 || kid_lt(s.bkey[pb], s.bid[pb] & kIdMask, hd.mk, hd.mi));
    const int c = from_buf ? (int)(s.bid[pb] & kIdMask) : (int)hd.mi;
    hint = pm < 0 ? w : from_buf ? pm : pm + 1;
    hint_b = pb < 0 ? wb : from_buf ? pb + 1 : pb;
    st.expansions += 1;
    const int cm = (st.expansions & 1) ? CTL_M_ODD : CTL_M;
    if (wave == 0) {
      // neighbour list, visited bits (each bit set exactly once), compaction
      // (streaming load, like the rows: +0.3% measured)
      const int nb = (lane < p.M0) ? __builtin_nontemporal_load(&p.adj0[(size_t)c * p.M0 + lane]) : -1;
      bool isnew = false;
      if (nb >= 0) {
        const uint32_t bit = 1u << (nb & 31);
        const uint32_t old = atomicOr(&bits[nb >> 5], bit);
        isnew = !(old & bit);
      }
      const uint64_t mk = ballot(isnew);
      log_visited(p, slot, q, st, isnew, nb, mk);
      if (isnew) s.cid[mbcnt(mk)] = nb;
      if (lane == 0) s.ctl[cm] = __builtin_popcountll(mk);
    }
    __syncthreads();
    // every wave has read the entry: mark it (scans resume after it, and the
    // next merge is several barriers away)
    if (tid == 0) {
      if (from_buf) s.bid[pb] = (uint32_t)c | kExpanded;
      else L.id[pm] = (uint32_t)c | kExpanded;
    }
    const int m = s.ctl[cm];
    if (tid == 0 && m > 64) debug_flag(p, kDbgCount);
    if (m == 0) continue;
    pol.score(p, s, m);
    __syncthreads();
    st.evals += m;
    if (wave == 0) {
      // the worst entry of a full W bounds what is kept
      const bool full = w + wb >= ef;
      const float tk = hd.tk;
      const uint32_t ti = hd.ti;
      // (read for every lane, entry 0 past m, so that both reads are waited
      // for together)
      float kk = s.ckey[lane < m ? lane : 0];
      uint32_t ki = (uint32_t)s.cid[lane < m ? lane : 0];
      if (lane >= m) { kk = __builtin_inff(); ki = kIdMask; }
      const bool keep = lane < m && (!full || kid_lt(kk, ki, tk, ti));
      const uint64_t km = ballot(keep);
      const int mnew = __builtin_popcountll(km);
      // sorted order of the kept entries: each counts the kept entries below
      // it (read from the other lanes' registers) and goes to that place
      int rk = 0;
      for (uint64_t rem = km; rem; rem &= rem - 1) {
        const int i = __builtin_ctzll(rem);
        const float ok = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kk), i));
        const uint32_t oi = (uint32_t)__builtin_amdgcn_readlane((int)ki, i);
        rk += kid_lt(ok, oi, kk, ki) ? 1 : 0;
      }
      wave_sync();
      if (keep) { s.ckey[rk] = kk; s.cid[rk] = (int32_t)ki; }
      if (lane == 0) {
        s.ctl[cm] = mnew;
        s.ctl[CTL_FLUSH] = (buffered && wb + mnew > p.wbuf) ? 1 : 0;
        s.ctl[CTL_HINT] = 0x7FFFFFFF;
      }
    }
    __syncthreads();
    const int mnew = s.ctl[cm];
    if (tid == 0 && mnew > m) debug_flag(p, kDbgCount);
    if (mnew > 0) {
      if (!buffered) {
        w = merge_sorted<4>(L.key, L.id, w, ef, s.ckey, (const uint32_t*)s.cid, mnew, &s.ctl[CTL_R0],
                            nullptr, nullptr);
        const int r0 = s.ctl[CTL_R0];
        if (r0 < hint) hint = r0;
      } else {
        if (s.ctl[CTL_FLUSH]) {
          if constexpr (GLIST) {
            w = merge_copy<4>(L.key, L.id, w, L2.key, L2.id, ef, s.bkey, s.bid, wb, &hint,
                              &s.ctl[CTL_HINT]);
            const List t = L;
            L = L2;
            L2 = t;
          } else {
            w = merge_sorted<8>(L.key, L.id, w, ef, s.bkey, s.bid, wb, &s.ctl[CTL_R0], &hint,
                                &s.ctl[CTL_HINT]);
          }
          wb = 0;
          hint_b = 0;
          lc.wh = -1;
          lc.tw = -1;
        }
        wb = merge_sorted<4>(s.bkey, s.bid, wb, p.wbuf, s.ckey, (const uint32_t*)s.cid, mnew,
                             &s.ctl[CTL_R0], nullptr, nullptr);
        const int r0 = s.ctl[CTL_R0];
        if (r0 < hint_b) hint_b = r0;
      }
    }
  }
  if (buffered && wb > 0) {
    if (tid == 0) s.ctl[CTL_HINT] = 0x7FFFFFFF;
    __syncthreads();
    if constexpr (GLIST) {
      w = merge_copy<4>(L.key, L.id, w, L2.key, L2.id, ef, s.bkey, s.bid, wb, &hint, &s.ctl[CTL_HINT]);
      L = L2;
    } else {
      w = merge_sorted<8>(L.key, L.id, w, ef, s.bkey, s.bid, wb, &s.ctl[CTL_R0], &hint, &s.ctl[CTL_HINT]);
    }
    wb = 0;
  }
  debug_check_beam<GLIST>(p, s, L, w, wb, ef, 0, 0);
  if (wave == 0 && lane == 0) {
    s.ctl[CTL_VISITED] = st.visited;
    s.ctl[CTL_VLOG] = st.vlog_n;
    s.ctl[CTL_VLOG_OVF] = st.vlog_overflow ? 1 : 0;
  }

  // rerank with the FP32 rows (rows split across the waves)
  int nres = w;
  if (p.rerank > 0) {
    int R = p.rerank > k ? p.rerank : k;
    if (R > w) R = w;
    nres = R;
    const int nch = p.d / 4;   // FP32 chunks
    // kRerankRows rows at a time per wave, 64 lanes per row; lane l takes
    // chunks l + 64 t in ascending t (256 chunks, 1,024 floats, per round).
    // Two rows keep the loads in flight without raising the register peak of
    // the kernel (which bounds the waves a compute unit holds).
    constexpr int kRerankRows = 2;
    for (int i0 = kRerankRows * wave; i0 < R; i0 += kRerankRows * num_waves()) {
      int rid[kRerankRows];
      float acc[kRerankRows];
#pragma unroll
      for (int u = 0; u < kRerankRows; ++u) {
        rid[u] = (i0 + u < R) ? (int)(L.id[i0 + u] & kIdMask) : -1;
        acc[u] = 0.0f;
      }
      for (int tb = 0; tb < nch; tb += 256) {
        uint4 raw[kRerankRows][4];
#pragma unroll
        for (int u = 0; u < kRerankRows; ++u) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            // unconditional (row 0, chunk 0 where there is none: the sum is
            // then skipped or not stored), so that the loads stay in flight
            const int g = tb + lane + 64 * t;
            const size_t row = rid[u] >= 0 ? (size_t)rid[u] : 0;
            raw[u][t] = *(const uint4*)(p.x_f32 + row * p.d + (size_t)(g < nch ? g : 0) * 4);
          }
        }
#pragma unroll
        for (int u = 0; u < kRerankRows; ++u) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int g = tb + lane + 64 * t;
            if (g < nch) {
              const float* qc = s.q + g * 4;
              if (p.metric == METRIC_IP) {
                acc[u] = __builtin_fmaf(qc[0], __uint_as_float(raw[u][t].x), acc[u]);
                acc[u] = __builtin_fmaf(qc[1], __uint_as_float(raw[u][t].y), acc[u]);
                acc[u] = __builtin_fmaf(qc[2], __uint_as_float(raw[u][t].z), acc[u]);
                acc[u] = __builtin_fmaf(qc[3], __uint_as_float(raw[u][t].w), acc[u]);
              } else {
                const float t0 = qc[0] - __uint_as_float(raw[u][t].x);
                const float t1 = qc[1] - __uint_as_float(raw[u][t].y);
                const float t2 = qc[2] - __uint_as_float(raw[u][t].z);
                const float t3 = qc[3] - __uint_as_float(raw[u][t].w);
                acc[u] = __builtin_fmaf(t0, t0, acc[u]);
                acc[u] = __builtin_fmaf(t1, t1, acc[u]);
                acc[u] = __builtin_fmaf(t2, t2, acc[u]);
                acc[u] = __builtin_fmaf(t3, t3, acc[u]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kRerankRows; ++u) {
        const float v = fold_lanes<64>(acc[u]);
        if (lane == 0 && rid[u] >= 0) s.rk[i0 + u] = (p.metric == METRIC_IP) ? -v : v;
      }
    }
    __syncthreads();
    // rank by (key, id) and write the first k
    for (int i = tid; i < R; i += nthr) {
      const float ki = s.rk[i];
      const uint32_t ii = L.id[i] & kIdMask;
      int rank = 0;
      for (int jj = 0; jj < R; ++jj) rank += kid_lt(s.rk[jj], L.id[jj] & kIdMask, ki, ii) ? 1 : 0;
      if (rank < k) {
        p.out_ids[q * p.k_max + rank] = (int64_t)ii;
        p.out_dists[q * p.k_max + rank] = ki;
      }
    }
  } else {
    for (int i = tid; i < k && i < w; i += nthr) {
      p.out_ids[q * p.k_max + i] = (int64_t)(L.id[i] & kIdMask);
      p.out_dists[q * p.k_max + i] = L.key[i];
    }
  }
  __syncthreads();
  const int visited = s.ctl[CTL_VISITED];
  const int vlog_n = s.ctl[CTL_VLOG];
  const bool vlog_ovf = s.ctl[CTL_VLOG_OVF] != 0;
  for (int i = tid; i < p.k_max; i += nthr) {
    if (i >= k || i >= nres) {
      p.out_ids[q * p.k_max + i] = -1;
      p.out_dists[q * p.k_max + i] = __builtin_inff();
    }
  }
  if (tid == 0) {
    if (p.out_status) p.out_status[q] = status;
    if (p.out_stats) {
      p.out_stats[q * 4 + 0] = st.evals;
      p.out_stats[q * 4 + 1] = st.expansions;
      p.out_stats[q * 4 + 2] = visited;
      p.out_stats[q * 4 + 3] = w;
    }
  }
  if (p.out_visited) {
    for (int64_t i = visited + tid; i < p.visited_cap; i += nthr) p.out_visited[q * p.visited_cap + i] = -1;
  }

  // leave the slot's visited bits clear for the next query
  if (!vlog_ovf) {
    const int32_t* lg = p.vlog + (size_t)slot * p.vlog_cap;
    for (int i = tid; i < vlog_n; i += nthr) bits[lg[i] >> 5] = 0u;
  } else {
    for (int64_t i = tid; i < p.bits_words; i += nthr) bits[i] = 0u;
  }
  __threadfence();
  __syncthreads();
}

// Waves per SIMD the register allocation must leave room for (4 caps a wave
// at 128 VGPRs); unset, the compiler chooses.
#ifdef ANN_WAVES_PER_EU
#define ANN_OCCUPANCY __attribute__((amdgpu_waves_per_eu(ANN_WAVES_PER_EU)))
#else
#define ANN_OCCUPANCY
#endif

// One step of waiting for a request of a server's ring, by thread 0 of a
// workgroup: straight-line code (no loop: a loop that only thread 0 runs
// would sit in divergent control flow next to the workgroup barriers of the
// caller's loop).  Returns the claimed sequence number, kRingWait to wait and
// try again, kRingRetry to try again at once (the claim word changed under
// this one, or a new request was just seen), or kRingEnd when the kernel is
// draining or the host asked it to end.
constexpr int64_t kRingWait = -2, kRingRetry = -3, kRingEnd = -1;

struct RingWait {
  uint64_t seen;     // the last tail seen
  uint64_t act;      // the last activity clock seen
  int64_t spins;     // waits since either changed
  int backoff;       // pairs of s_sleep 127 before the next look (1 .. 32)
  uint64_t defer_h;  // the request this workgroup left to a lower tier
  uint64_t defer_t;  // since when
};

__device__ __forceinline__ int64_t ring_step(const RingArgs& r, RingWait& w, int tier) {
  uint64_t h = __hip_atomic_load(r.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (h & kRingFlags) return kRingEnd;
  const uint64_t now = (uint64_t)wall_clock64();
  const uint64_t tail = __hip_atomic_load(r.mirror, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // waiting workgroups of lower tiers: they take the traffic first
  uint32_t lower = 0;
#pragma unroll
  for (int t = 0; t < kRingTiers - 1; ++t)
    if (t < tier) lower += __hip_atomic_load(&r.waiting[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (h < tail) {
    // (a lower tier's workgroup may be asleep: after poll_ticks x 10 this
    // one takes the request itself)
    if (lower > 0) {
      if (w.defer_h != h) { w.defer_h = h; w.defer_t = now; }
      if (now - w.defer_t < 10 * r.poll_ticks) {
        w.backoff = 1;
        return kRingWait;
      }
    }
    // counted as in flight before the claim, so that no drain can slip
    // between a successful claim and the count
    __hip_atomic_fetch_add(r.busy, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_compare_exchange_strong(r.head, &h, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
      __hip_atomic_fetch_max(r.activity, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_sub(&r.waiting[tier], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      w.backoff = 1;
      return (int64_t)h;
    }
    __hip_atomic_fetch_sub(r.busy, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return kRingRetry;
  }
  // nothing to claim.  Only the front (the lowest tier with waiting
  // workgroups) stays responsive: it reads the host's tail when it is its
  // turn (one reader per poll_ticks) and looks again soon after the ring
  // moves.  Tiers behind it sleep the longest naps: thousands of workgroups
  // polling the same few words every few microseconds slow every search in
  // flight (measured: 5.6 ms instead of 1.0 ms per request).
  const bool front = lower == 0;
  uint64_t lp = __hip_atomic_load(r.last_poll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (front && now - lp >= r.poll_ticks &&
      __hip_atomic_compare_exchange_strong(r.last_poll, &lp, now, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT)) {
    const uint64_t ht = __hip_atomic_load(r.host_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (__hip_atomic_load(r.host_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
      __hip_atomic_fetch_or(r.head, kRingStop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return kRingEnd;
    }
    if (ht > tail) {
      __hip_atomic_fetch_max(r.mirror, ht, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_max(r.activity, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      w.backoff = 1;
      return kRingRetry;
    }
  }
  if (front && tail != w.seen) { w.seen = tail; w.spins = 0; w.backoff = 1; }
  ++w.spins;
  // the drain test reads two more shared words: every eighth wait only
  if ((w.spins & 7) == 0) {
    const uint64_t act = __hip_atomic_load(r.activity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (act != w.act) { w.act = act; w.spins = 0; }
    if ((now - act > r.idle_ticks || w.spins > r.idle_spins) &&
        __hip_atomic_load(r.busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      // idle with nothing in flight: the whole kernel ends
      if (__hip_atomic_compare_exchange_strong(r.head, &h, h | kRingDrain, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        return kRingEnd;
      return kRingRetry;
    }
  }
  w.backoff = front && w.backoff < 32 ? 2 * w.backoff : 32;
  return kRingWait;
}

// RING: the server's kernel (requests from a ring); otherwise a batch.  Two
// instantiations, so that the ring's state does not add to the registers of
// the batch kernel (they bound how many queries a compute unit holds).
template <class Policy, bool GLIST, bool RING>
__global__ void __launch_bounds__(512) ANN_OCCUPANCY search_kernel(SearchParams p) {
  extern __shared__ __align__(16) char lds_raw[];
  const Lds s = carve(lds_raw, p);
  Policy pol;
  const int slot = blockIdx.x;
  // a device-held batch size (captured launches) is clamped to the buffers' capacity p.nq
  int64_t nq = p.nq;
  if (p.nq_dev) {
    const int64_t nd = (int64_t)uniform_int(*p.nq_dev);
    nq = nd < 0 ? 0 : nd < p.nq ? nd : p.nq;
  }
  if constexpr (RING) {
    // server: one request of the ring at a time.  Every loop here is left by
    // all threads together (the decisions come from LDS after a barrier).
    const RingArgs r = p.ring;
    RingWait w{~0ull, ~0ull, 0, 1, ~0ull, 0};
    const int tier = min((int)blockIdx.x / r.tier_width, kRingTiers - 1);
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&r.waiting[tier], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
      int64_t seq;
      while (true) {
        if (threadIdx.x == 0) {
          const int64_t got = ring_step(r, w, tier);
          // a workgroup that leaves stops counting as waiting
          if (got == kRingEnd)
            __hip_atomic_fetch_sub(&r.waiting[tier], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s.ctl[CTL_SEQ_LO] = (int)(uint32_t)(uint64_t)got;
          s.ctl[CTL_SEQ_HI] = (int)(uint32_t)((uint64_t)got >> 32);
          s.ctl[CTL_BACKOFF] = w.backoff;
        }
        __syncthreads();
        seq = (int64_t)(((uint64_t)(uint32_t)uniform_int(s.ctl[CTL_SEQ_HI]) << 32) |
                        (uint32_t)uniform_int(s.ctl[CTL_SEQ_LO]));
        const int naps = uniform_int(s.ctl[CTL_BACKOFF]);
        __syncthreads();
        if (seq != kRingWait && seq != kRingRetry) break;
        if (seq == kRingWait) {
          // 1 to 32 pairs of the longest sleep (about 6.8 us a pair at
          // 2.4 GHz): the longer nothing arrives, the rarer the looks
          for (int i = 0; i < naps; ++i) {
            __builtin_amdgcn_s_sleep(127);
            __builtin_amdgcn_s_sleep(127);
          }
        }
      }
      if (seq < 0) break;
      const int64_t pos = seq % r.cap;
      // the host's entry into this workgroup's copy: system-scope loads see
      // what the host wrote before it published the entry, without an
      // acquire (which would invalidate this die's L2 once per request)
      if (threadIdx.x == 0) {
        __hip_atomic_store(&r.t_start[pos], (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
        ((int32_t*)p.k_arr)[slot] = __hip_atomic_load(&r.e_k[pos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        ((int32_t*)p.ef_arr)[slot] = __hip_atomic_load(&r.e_ef[pos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      for (int i = threadIdx.x; i < p.d; i += blockDim.x)
        ((float*)p.queries)[(size_t)slot * p.d + i] =
            __hip_atomic_load(&r.e_query[(size_t)pos * p.d + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __syncthreads();
      run_query<Policy, GLIST>(p, s, pol, slot, slot);
      // the results out to the host's entry with system-scope stores, which
      // complete (s_waitcnt) before the completion flag is written
      for (int i = threadIdx.x; i < p.k_max; i += blockDim.x) {
        __hip_atomic_store(&r.e_ids[pos * p.k_max + i], p.out_ids[(int64_t)slot * p.k_max + i],
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r.e_dists[pos * p.k_max + i], p.out_dists[(int64_t)slot * p.k_max + i],
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      if (threadIdx.x == 0) {
        __hip_atomic_store(&r.e_status[pos], p.out_status[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r.t_done[pos], (uint64_t)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r.served_by[pos], slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) {
        __hip_atomic_store(&r.done[pos], (uint64_t)seq + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_fetch_add(&r.waiting[tier], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_sub(r.busy, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // thread 0 has stored the flag before the next round's barrier
      __syncthreads();
    }
    return;
  }
  while (true) {
    if (threadIdx.x == 0) s.ctl[CTL_QUERY] = atomicAdd(p.counter, 1);
    __syncthreads();
    const int qi = uniform_int(s.ctl[CTL_QUERY]);
    __syncthreads();
    if (qi >= nq) break;
    run_query<Policy, GLIST>(p, s, pol, slot, (int64_t)qi);
  }
}

// ----------------------------------------------------------------------------
// kernel selection (instantiated by the per-mode translation units)
// ----------------------------------------------------------------------------

template <class Policy>
inline const void* pick_kernel(const SearchParams& p) {
  if (p.ring.cap > 0)
    return p.glist ? (const void*)search_kernel<Policy, true, true>
                   : (const void*)search_kernel<Policy, false, true>;
  return p.glist ? (const void*)search_kernel<Policy, true, false>
                 : (const void*)search_kernel<Policy, false, false>;
}

// Kernel for a dense mode: L lanes per row, CPL 16-byte chunks per lane.
template <int MODE>
inline const void* dense_symbol(const SearchParams& p) {
  const int L = p.lanes_per_row, cpl = (p.nchunks + L - 1) / L;
  if (L == 64) {
    if (cpl <= 1) return pick_kernel<Dense<MODE, 64, 1>>(p);
    if (cpl <= 2) return pick_kernel<Dense<MODE, 64, 2>>(p);
    if (cpl <= 3) return pick_kernel<Dense<MODE, 64, 3>>(p);
    if (cpl <= 4) return pick_kernel<Dense<MODE, 64, 4>>(p);
  } else if (L == 32) {
    if (cpl <= 1) return pick_kernel<Dense<MODE, 32, 1>>(p);
    if (cpl <= 2) return pick_kernel<Dense<MODE, 32, 2>>(p);
    if constexpr (MODE != MODE_FP8)
      if (cpl <= 3) return pick_kernel<Dense<MODE, 32, 3>>(p);
    if constexpr (MODE == MODE_F32)
      if (cpl <= 4) return pick_kernel<Dense<MODE, 32, 4>>(p);
  } else if (L == 16) {
    if (cpl <= 1) return pick_kernel<Dense<MODE, 16, 1>>(p);
    if (cpl <= 2) return pick_kernel<Dense<MODE, 16, 2>>(p);
    if constexpr (MODE == MODE_F32)
      if (cpl <= 4) return pick_kernel<Dense<MODE, 16, 4>>(p);
  }
  return nullptr;
}

}  // namespace ann
