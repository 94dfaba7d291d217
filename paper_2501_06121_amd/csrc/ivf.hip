// IVF index on the device: inverted lists over a k-means coarse quantizer,
// the index family the paper names beside graphs (Section 1) and plans to add
// (Section 4, Conclusions and Future Work), searched with the same representations and keys as the HNSW
// path (FP32 / FP16 / BF16 / FP8 rows, PQ codes, optional FP32 rerank).
//
// A batch runs two kernels (plus, for the dense modes, a choice of scan):
//  * ivf_probe: one wavefront per query scores the query against every FP32
//    centroid (squared L2 in the fixed FP32 order of a dense FP32 row) and
//    sorts the (key, list id) pairs in LDS; the first nprobe are the probes;
//  * ivf_scan: one wavefront per query walks its probed lists (in ascending
//    list order, so that the queries in flight share rows in the caches) 64
//    rows at a time, scores them with the search kernel's scoring policy and merges the
//    rows that beat the current kk-th best into a sorted list of kk entries
//    in LDS (kk = max(k, rerank depth)).  The list then takes the optional
//    FP32 rerank and is written out;
//  * ivf_scan_shared (dense modes, the default when a query probes more than
//    a quarter of the lists): up to 16 queries (8 by default) per workgroup
//    stage each list of the union of their probes in LDS once and each wave
//    scores the tile for its own query, so that a row is read from device
//    memory once per workgroup instead of once per query.
// The rows of a list are read where they are (no per-list copy), so every
// representation of the index serves the IVF search without extra memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "ann.h"
#include "internal.h"
#include "search_impl.h"

namespace ann {
namespace {

constexpr int kMaxLists = 8192;   // probe sort in LDS: 8 bytes per list
constexpr int kMaxGroup = 16;     // queries per workgroup of the shared scan (1024 threads)
constexpr int kAutoGroup = 8;     // the dense modes' default
constexpr int kCopyBatch = 8;     // 16-byte chunks per thread in flight while staging a tile
constexpr int kIdChunk = 1024;    // list ids (and FP8 scales) staged in LDS at once
// Workgroups of the shared scan one compute unit should hold (the LDS share
// the tile is sized for).
#ifndef ANN_IVF_SHARED_WG_PER_CU
#define ANN_IVF_SHARED_WG_PER_CU 2
#endif

struct IvfArgs {
  int nlist, nprobe, np;          // np = min(nprobe, nlist)
  int k, kk;                      // results; entries kept while scanning
  int sort_n;                     // power of two >= nlist
  const float* cent;              // [nlist][d]
  const int64_t* list_off;        // [nlist + 1]
  const int32_t* list_ids;        // [n]
  int32_t* probes;                // [nq][nprobe]
  int32_t* stats;                 // [nq][2] or NULL
  int group;                      // queries (wavefronts) per workgroup of the shared scan
  int wave_lds;                   // LDS bytes of one wave's region (multiple of 16)
  int tile_rows;                  // rows per LDS tile of the shared scan (<= 64)
  int tile_bytes;                 // tile_rows * row bytes
};

// ---------------------------------------------------------------------------
// probes
// ---------------------------------------------------------------------------

template <int CPL>
__global__ void __launch_bounds__(64) ivf_probe(SearchParams pc, IvfArgs v) {
  extern __shared__ __align__(16) char lds_raw[];
  Lds s{};
  s.cid = (int32_t*)lds_raw;
  s.ckey = (float*)(lds_raw + 256);
  float* pk = (float*)(lds_raw + 512);
  uint32_t* pi = (uint32_t*)(lds_raw + 512 + 4 * (size_t)v.sort_n);
  const int64_t q = blockIdx.x;
  const int lane = lane_id();
  Dense<MODE_F32, 64, CPL> pol;
  pol.prep(pc, s, q);
  for (int base = 0; base < v.nlist; base += 64) {
    const int m = min(64, v.nlist - base);
    if (lane < m) s.cid[lane] = base + lane;
    __syncthreads();
    pol.score(pc, s, m);
    __syncthreads();
    if (lane < m) { pk[base + lane] = s.ckey[lane]; pi[base + lane] = (uint32_t)(base + lane); }
    __syncthreads();
  }
  for (int i = v.nlist + lane; i < v.sort_n; i += 64) { pk[i] = __builtin_inff(); pi[i] = 0xFFFFFFFFu; }
  __syncthreads();
  // bitonic sort of (key, list id), ascending
  for (int kb = 2; kb <= v.sort_n; kb <<= 1) {
    for (int j = kb >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < v.sort_n; i += 64) {
        const int o = i ^ j;
        if (o > i) {
          const float a = pk[i], b = pk[o];
          const uint32_t ai = pi[i], bi = pi[o];
          const bool up = (i & kb) == 0;
          if (up ? kid_lt(b, bi, a, ai) : kid_lt(a, ai, b, bi)) {
            pk[i] = b; pi[i] = bi; pk[o] = a; pi[o] = ai;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = lane; t < v.nprobe; t += 64) v.probes[q * v.nprobe + t] = t < v.np ? (int32_t)pi[t] : -1;
}

// ---------------------------------------------------------------------------
// list scan
// ---------------------------------------------------------------------------

struct ScanLds {
  Lds s;
  float* tk0;                     // two sorted lists (key, id) of kk entries;
  float* tk1;                     // each merge writes the other one
  uint32_t* ti0;
  uint32_t* ti1;
  float* sk;
  uint32_t* si;
  uint32_t* pmask;                // probed lists, one bit per list
};

__device__ ScanLds scan_carve(char* base, const SearchParams& p, const IvfArgs& v) {
  ScanLds L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { char* r = base + off; off += (bytes + 15) & ~size_t(15); return r; };
  L.s.cid = (int32_t*)take(4 * 64);
  L.s.ckey = (float*)take(4 * 64);
  L.sk = (float*)take(4 * 64);
  L.si = (uint32_t*)take(4 * 64);
  L.s.q = (float*)take(sizeof(float) * p.q_lds_floats);
  L.s.lut = (float*)take(sizeof(float) * (p.mode == MODE_PQ ? p.pq_m * 256 : 0));
  L.s.rk = (float*)take(sizeof(float) * (p.rerank > 0 ? v.kk : 0));
  L.pmask = (uint32_t*)take(4 * (size_t)((v.nlist + 31) / 32));
  L.tk0 = (float*)take(sizeof(float) * v.kk);
  L.ti0 = (uint32_t*)take(sizeof(uint32_t) * v.kk);
  L.tk1 = (float*)take(sizeof(float) * v.kk);
  L.ti1 = (uint32_t*)take(sizeof(uint32_t) * v.kk);
  return L;
}

size_t scan_lds_bytes(const SearchParams& p, const IvfArgs& v) {
  auto r16 = [](size_t b) { return (b + 15) & ~size_t(15); };
  size_t b = 4 * r16(256);
  b += r16(sizeof(float) * p.q_lds_floats);
  b += r16(sizeof(float) * (p.mode == MODE_PQ ? p.pq_m * 256 : 0));
  b += r16(sizeof(float) * (p.rerank > 0 ? v.kk : 0));
  b += r16(4 * (size_t)((v.nlist + 31) / 32));
  b += 4 * r16(4 * (size_t)v.kk);
  return b;
}

// Number of entries of the sorted (key, id) array a[0..n) that precede (k, i).
__device__ __forceinline__ int count_less(const float* ak, const uint32_t* ai, int n, float k,
                                          uint32_t i) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kid_lt(ak[mid], ai[mid], k, i)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Merges one batch of scored rows (one per lane; lanes with `pass` enter)
// into the wave's sorted list of kk entries: the new entries are ranked among
// themselves with lane reads, then both sorted runs are merged into the other
// list buffer (merge path), keeping the first kk.  Wave-level ordering only.
__device__ __forceinline__ void merge_batch(const ScanLds& L, int kk, int& cnt, int& cur, float key,
                                            uint32_t id, bool pass) {
  const int lane = lane_id();
  const uint64_t mask = ballot(pass);
  if (mask == 0) return;
  const float* ck = cur ? L.tk1 : L.tk0;
  const uint32_t* ci = cur ? L.ti1 : L.ti0;
  const int ns = __popcll(mask);
  int r = 0;
  for (uint64_t mm = mask; mm; mm &= mm - 1) {
    const int j = __builtin_ctzll(mm);
    const float kj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(key), j));
    const uint32_t ij = (uint32_t)__builtin_amdgcn_readlane((int)id, j);
    r += kid_lt(kj, ij, key, id) ? 1 : 0;
  }
  if (pass) { L.sk[r] = key; L.si[r] = id; }
  wave_sync();
  float* nk = cur ? L.tk0 : L.tk1;
  uint32_t* ni = cur ? L.ti0 : L.ti1;
  for (int i = lane; i < cnt; i += 64) {
    const float a = ck[i];
    const uint32_t ai = ci[i];
    const int pos = i + count_less(L.sk, L.si, ns, a, ai);
    if (pos < kk) { nk[pos] = a; ni[pos] = ai; }
  }
  if (lane < ns) {
    const float a = L.sk[lane];
    const uint32_t ai = L.si[lane];
    const int pos = lane + count_less(ck, ci, cnt, a, ai);
    if (pos < kk) { nk[pos] = a; ni[pos] = ai; }
  }
  wave_sync();
  cnt = min(kk, cnt + ns);
  cur ^= 1;
}

// The end of a query, by its wave: the optional FP32 rerank of the first
// min(max(R, k), cnt) kept entries (4 rows at a time, 64 lanes per row in the
// fixed FP32 order), the ranking by (key, id), the k results with padding, and
// the statistics.
__device__ __forceinline__ void finish_query(const SearchParams& p, const IvfArgs& v,
                                             const ScanLds& L, int64_t q, int cnt, int cur,
                                             int evals) {
  const Lds& s = L.s;
  // the FP32 query: its LDS copy, or (shared scan) device memory
  const float* qv = p.q_lds_floats > 0 ? s.q : p.queries + (size_t)q * p.d;
  const int lane = lane_id();
  const float* fk = cur ? L.tk1 : L.tk0;
  const uint32_t* fi = cur ? L.ti1 : L.ti0;
  const int k = v.k;
  int nres = cnt;
  if (p.rerank > 0) {
    int R = p.rerank > k ? p.rerank : k;
    if (R > cnt) R = cnt;
    nres = R;
    const int nch = p.d / 4;
    for (int i0 = 0; i0 < R; i0 += 4) {
      uint4 raw[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int rid = (i0 + u < R) ? (int)fi[i0 + u] : -1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int g = lane + 64 * t;
          raw[u][t] = (rid >= 0 && g < nch) ? *(const uint4*)(p.x_f32 + (size_t)rid * p.d + (size_t)g * 4)
                                            : make_uint4(0u, 0u, 0u, 0u);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int g = lane + 64 * t;
          if (g < nch) {
            const float* qc = qv + g * 4;
            if (p.metric == METRIC_IP) {
              acc = __builtin_fmaf(qc[0], __uint_as_float(raw[u][t].x), acc);
              acc = __builtin_fmaf(qc[1], __uint_as_float(raw[u][t].y), acc);
              acc = __builtin_fmaf(qc[2], __uint_as_float(raw[u][t].z), acc);
              acc = __builtin_fmaf(qc[3], __uint_as_float(raw[u][t].w), acc);
            } else {
              const float t0 = qc[0] - __uint_as_float(raw[u][t].x);
              const float t1 = qc[1] - __uint_as_float(raw[u][t].y);
              const float t2 = qc[2] - __uint_as_float(raw[u][t].z);
              const float t3 = qc[3] - __uint_as_float(raw[u][t].w);
              acc = __builtin_fmaf(t0, t0, acc);
              acc = __builtin_fmaf(t1, t1, acc);
              acc = __builtin_fmaf(t2, t2, acc);
              acc = __builtin_fmaf(t3, t3, acc);
            }
          }
        }
        acc = fold_lanes<64>(acc);
        if (lane == 0 && i0 + u < R) s.rk[i0 + u] = (p.metric == METRIC_IP) ? -acc : acc;
      }
    }
    wave_sync();
    for (int i = lane; i < R; i += 64) {
      const float ki = s.rk[i];
      const uint32_t ii = fi[i];
      int rank = 0;
      for (int j = 0; j < R; ++j) rank += kid_lt(s.rk[j], fi[j], ki, ii) ? 1 : 0;
      if (rank < k) {
        p.out_ids[q * k + rank] = (int64_t)ii;
        p.out_dists[q * k + rank] = ki;
      }
    }
  } else {
    for (int i = lane; i < k && i < cnt; i += 64) {
      p.out_ids[q * k + i] = (int64_t)fi[i];
      p.out_dists[q * k + i] = fk[i];
    }
  }
  for (int i = lane; i < k; i += 64) {
    if (i >= nres) {
      p.out_ids[q * k + i] = -1;
      p.out_dists[q * k + i] = __builtin_inff();
    }
  }
  if (v.stats && lane == 0) {
    v.stats[q * 2 + 0] = evals;
    v.stats[q * 2 + 1] = v.np;
  }
}

// The probed lists of query q as a bit mask in the wave's LDS region.
__device__ __forceinline__ void probe_mask(const IvfArgs& v, const ScanLds& L, int64_t q) {
  const int lane = lane_id();
  const int words = (v.nlist + 31) / 32;
  for (int w = lane; w < words; w += 64) L.pmask[w] = 0u;
  wave_sync();
  for (int t = lane; t < v.np; t += 64) {
    const int l = v.probes[q * v.nprobe + t];
    if (l >= 0 && l < v.nlist) atomicOr(&L.pmask[l >> 5], 1u << (l & 31));
  }
  wave_sync();
}

// One query per workgroup (one wavefront): the rows are read from device
// memory where they are.  The probed lists are scanned in ascending list
// order, not in probe order: the kept entries do not depend on the order (a
// strict total order on unique ids), and the queries in flight then sweep
// the rows together, so that rows one query brings into the caches serve the
// others.
template <class Policy>
__global__ void __launch_bounds__(64) ivf_scan(SearchParams p, IvfArgs v) {
  extern __shared__ __align__(16) char lds_raw[];
  const ScanLds L = scan_carve(lds_raw, p, v);
  const Lds& s = L.s;
  const int64_t q = blockIdx.x;
  const int lane = lane_id();
  if (p.q_lds_floats > 0) {
    const float* qrow = p.queries + (size_t)q * p.d;
    for (int i = lane; i < p.q_lds_floats; i += 64) s.q[i] = (i < p.d) ? qrow[i] : 0.0f;
  }
  __syncthreads();
  Policy pol;
  pol.prep(p, s, q);
  probe_mask(v, L, q);
  const int words = (v.nlist + 31) / 32;
  int cnt = 0, cur = 0, evals = 0;
  for (int w = 0; w < words; ++w) {
    for (uint32_t bits = (uint32_t)uniform_int((int)L.pmask[w]); bits; bits &= bits - 1u) {
      const int l = w * 32 + __builtin_ctz(bits);
      const int64_t b = v.list_off[l], e = v.list_off[l + 1];
      for (int64_t base = b; base < e; base += 64) {
        const int m = (int)min<int64_t>(64, e - base);
        if (lane < m) s.cid[lane] = v.list_ids[base + lane];
        __syncthreads();
        pol.score(p, s, m);
        __syncthreads();
        evals += m;
        const float key = lane < m ? s.ckey[lane] : __builtin_inff();
        const uint32_t id = lane < m ? (uint32_t)s.cid[lane] : 0xFFFFFFFFu;
        const float* ck = cur ? L.tk1 : L.tk0;
        const uint32_t* ci = cur ? L.ti1 : L.ti0;
        bool pass = lane < m;
        if (cnt == v.kk) pass = pass && kid_lt(key, id, ck[v.kk - 1], ci[v.kk - 1]);
        merge_batch(L, v.kk, cnt, cur, key, id, pass);
      }
    }
  }
  finish_query(p, v, L, q, cnt, cur, evals);
}

// v.group queries per workgroup (one wavefront each), dense modes.  The
// workgroup walks the union of its queries' probed lists in ascending order,
// stages the list's ids (up to kIdChunk at a time) and then its rows,
// v.tile_rows at a time, in LDS once; every wave
// whose query probes that list then scores the tile from LDS with the same
// scoring policy (same keys as from device memory) and merges it into its own
// list.  A row is read from device memory once per workgroup instead of once
// per query.
template <class Policy>
__global__ void __launch_bounds__(1024) ivf_scan_shared(SearchParams p, IvfArgs v) {
  extern __shared__ __align__(16) char lds_raw[];
  const size_t row_bytes = (size_t)p.nchunks * 16;
  const int words = (v.nlist + 31) / 32;
  char* tile = lds_raw;                                              // [tile_rows][row_bytes]
  uint32_t* list_ids = (uint32_t*)(lds_raw + v.tile_bytes);          // [kIdChunk] of the list
  float* list_scale = (float*)(lds_raw + v.tile_bytes + 4 * kIdChunk);   // [kIdChunk] (FP8)
  uint32_t* umask = (uint32_t*)(lds_raw + v.tile_bytes + 8 * kIdChunk);  // [words]
  char* regions = lds_raw + v.tile_bytes + 8 * kIdChunk + ((4 * (size_t)words + 15) & ~size_t(15));
  const int wave = wave_id();
  const int lane = lane_id();
  const ScanLds L = scan_carve(regions + (size_t)wave * v.wave_lds, p, v);
  const Lds& s = L.s;
  const int64_t q = (int64_t)blockIdx.x * v.group + wave;
  const bool active = q < p.nq;
  Policy pol;
  if (active) {
    if (p.q_lds_floats > 0) {
      const float* qrow = p.queries + (size_t)q * p.d;
      for (int i = lane; i < p.q_lds_floats; i += 64) s.q[i] = (i < p.d) ? qrow[i] : 0.0f;
    }
    pol.prep(p, s, q);
    probe_mask(v, L, q);
  } else {
    for (int w = lane; w < words; w += 64) L.pmask[w] = 0u;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < words; w += blockDim.x) {
    uint32_t u = 0u;
    for (int g = 0; g < num_waves(); ++g) u |= scan_carve(regions + (size_t)g * v.wave_lds, p, v).pmask[w];
    umask[w] = u;
  }
  __syncthreads();
  const int nch = p.nchunks;
  const char* rows = (const char*)p.rows;
  int cnt = 0, cur = 0, evals = 0;
  for (int w = 0; w < words; ++w) {
    for (uint32_t bits = (uint32_t)uniform_int((int)umask[w]); bits; bits &= bits - 1u) {
      const int bit = __builtin_ctz(bits);
      const int l = w * 32 + bit;
      const bool mine = active && ((L.pmask[w] >> bit) & 1u);
      const int64_t b = v.list_off[l], e = v.list_off[l + 1];
      for (int64_t c0 = b; c0 < e; c0 += kIdChunk) {
        // the ids (and FP8 scales) of up to kIdChunk rows of the list, once
        const int nc = (int)min<int64_t>(kIdChunk, e - c0);
        __syncthreads();                  // every wave is done with the previous tile
        for (int r = threadIdx.x; r < nc; r += blockDim.x) {
          const int32_t id = v.list_ids[c0 + r];
          list_ids[r] = (uint32_t)id;
          if (p.mode == MODE_FP8) list_scale[r] = p.fp8_scale[id];
        }
        for (int t0 = 0; t0 < nc; t0 += v.tile_rows) {
          const int m = min(v.tile_rows, nc - t0);
          __syncthreads();                // ids staged / the previous tile scored
          // the rows, kCopyBatch 16-byte chunks per thread in flight at once
          const int total = m * nch;
          for (int cb = threadIdx.x; cb < total; cb += kCopyBatch * blockDim.x) {
            uint4 x[kCopyBatch];
#pragma unroll
            for (int u = 0; u < kCopyBatch; ++u) {
              const int c = cb + u * (int)blockDim.x;
              x[u] = make_uint4(0u, 0u, 0u, 0u);
              if (c < total) {
                const int r = c / nch, g = c - r * nch;
                x[u] = *(const uint4*)(rows + (size_t)list_ids[t0 + r] * row_bytes + (size_t)g * 16);
              }
            }
#pragma unroll
            for (int u = 0; u < kCopyBatch; ++u) {
              const int c = cb + u * (int)blockDim.x;
              if (c < total) {
                const int r = c / nch, g = c - r * nch;
                *(uint4*)(tile + (size_t)r * row_bytes + (size_t)g * 16) = x[u];
              }
            }
          }
          __syncthreads();
          if (!mine) continue;
          if (lane < m) s.cid[lane] = lane;
          wave_sync();
          pol.score_rows(p, s, 0, m, tile, list_scale + t0);
          wave_sync();
          evals += m;
          const float key = lane < m ? s.ckey[lane] : __builtin_inff();
          const uint32_t id = lane < m ? list_ids[t0 + lane] : 0xFFFFFFFFu;
          const float* ck = cur ? L.tk1 : L.tk0;
          const uint32_t* ci = cur ? L.ti1 : L.ti0;
          bool pass = lane < m;
          if (cnt == v.kk) pass = pass && kid_lt(key, id, ck[v.kk - 1], ci[v.kk - 1]);
          merge_batch(L, v.kk, cnt, cur, key, id, pass);
        }
      }
    }
  }
  if (active) finish_query(p, v, L, q, cnt, cur, evals);
}

// ---------------------------------------------------------------------------
// kernel selection
// ---------------------------------------------------------------------------

template <class Policy, bool SHARED>
const void* scan_sym() {
  if constexpr (SHARED) return (const void*)ivf_scan_shared<Policy>;
  else return (const void*)ivf_scan<Policy>;
}

template <int MODE, bool SH>
const void* scan_dense(int L, int cpl) {
  if (L == 64) {
    if (cpl <= 1) return scan_sym<Dense<MODE, 64, 1>, SH>();
    if (cpl <= 2) return scan_sym<Dense<MODE, 64, 2>, SH>();
    if (cpl <= 3) return scan_sym<Dense<MODE, 64, 3>, SH>();
    if (cpl <= 4) return scan_sym<Dense<MODE, 64, 4>, SH>();
  } else if (L == 32) {
    if (cpl <= 1) return scan_sym<Dense<MODE, 32, 1>, SH>();
    if (cpl <= 2) return scan_sym<Dense<MODE, 32, 2>, SH>();
    if constexpr (MODE != MODE_FP8)
      if (cpl <= 3) return scan_sym<Dense<MODE, 32, 3>, SH>();
    if constexpr (MODE == MODE_F32)
      if (cpl <= 4) return scan_sym<Dense<MODE, 32, 4>, SH>();
  } else if (L == 16) {
    if (cpl <= 1) return scan_sym<Dense<MODE, 16, 1>, SH>();
    if (cpl <= 2) return scan_sym<Dense<MODE, 16, 2>, SH>();
    if constexpr (MODE == MODE_F32)
      if (cpl <= 4) return scan_sym<Dense<MODE, 16, 4>, SH>();
  }
  return nullptr;
}

template <bool SH>
const void* scan_symbol(const SearchParams& p) {
  const int L = p.lanes_per_row, cpl = (p.nchunks + L - 1) / L;
  switch (p.mode) {
    case MODE_F32: return scan_dense<MODE_F32, SH>(L, cpl);
    case MODE_F16: return scan_dense<MODE_F16, SH>(L, cpl);
    case MODE_BF16: return scan_dense<MODE_BF16, SH>(L, cpl);
    case MODE_FP8: return scan_dense<MODE_FP8, SH>(L, cpl);
    case MODE_PQ: return SH ? nullptr : scan_sym<PQ<16>, false>();
  }
  return nullptr;
}

const void* probe_symbol(int cpl) {
  switch (cpl) {
    case 1: return (const void*)ivf_probe<1>;
    case 2: return (const void*)ivf_probe<2>;
    case 3: return (const void*)ivf_probe<3>;
    case 4: return (const void*)ivf_probe<4>;
  }
  return nullptr;
}

hipError_t launch(const void* fn, int64_t blocks, int threads, size_t lds, hipStream_t st,
                  SearchParams& p, IvfArgs& v) {
  void* args[] = {&p, &v};
  if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(threads), args, lds, st);
}

}  // namespace
}  // namespace ann

using namespace ann;

struct ann_ivf {
  ann_index* ix = nullptr;
  int nlist = 0;
  float* cent = nullptr;
  int64_t* list_off = nullptr;
  int32_t* list_ids = nullptr;
  int32_t* probes = nullptr;      // scratch for batches without out_probes
  int64_t probes_cap = 0;         // entries
  hipEvent_t done = nullptr;      // recorded after the last batch that used `probes`
  std::mutex mu;
};

extern "C" int ann_ivf_create(ann_index* ix, int32_t nlist, const float* centroids,
                              const int64_t* list_off, const int32_t* list_ids, ann_ivf** out) {
  if (!ix || !centroids || !list_off || !list_ids || !out) return fail(ANN_EINVAL, "NULL argument");
  *out = nullptr;
  if (!ix->x_f32 && !ix->x_f16 && !ix->x_bf16 && !ix->x_fp8 && !ix->pq_codes)
    return fail(ANN_EUNSUP, "an IVF index needs dense rows or PQ codes");
  if (nlist < 1 || nlist > kMaxLists) return fail(ANN_EINVAL, "nlist %d outside [1, %d]", nlist, kMaxLists);
  if (ix->d % 4 != 0 || ix->d > 1024) return fail(ANN_EUNSUP, "centroids of %d dimensions (a multiple of 4, at most 1024)", ix->d);
  const int64_t n = ix->n;
  if (list_off[0] != 0 || list_off[nlist] != n)
    return fail(ANN_EFORMAT, "list offsets must run from 0 to n = %lld", (long long)n);
  std::vector<uint8_t> seen((size_t)n, 0);
  for (int l = 0; l < nlist; ++l) {
    if (list_off[l + 1] < list_off[l]) return fail(ANN_EFORMAT, "list offsets decrease at list %d", l);
    for (int64_t t = list_off[l]; t < list_off[l + 1]; ++t) {
      const int32_t r = list_ids[t];
      if (r < 0 || r >= n) return fail(ANN_EFORMAT, "row %d in list %d outside [0, %lld)", r, l, (long long)n);
      if (seen[r]) return fail(ANN_EFORMAT, "row %d appears in two lists", r);
      seen[r] = 1;
    }
  }
  for (int c = 0; c < nlist * ix->d; ++c)
    if (!std::isfinite(centroids[c])) return fail(ANN_EFORMAT, "centroid value %d is not finite", c);
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  ann_ivf* v = new ann_ivf;
  v->ix = ix;
  v->nlist = nlist;
  const size_t cb = sizeof(float) * (size_t)nlist * ix->d;
  hipError_t e = hipMalloc((void**)&v->cent, cb);
  if (e == hipSuccess) e = hipMalloc((void**)&v->list_off, sizeof(int64_t) * (nlist + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&v->list_ids, sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
  if (e == hipSuccess) e = hipMemcpy(v->cent, centroids, cb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(v->list_off, list_off, sizeof(int64_t) * (nlist + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && n > 0) e = hipMemcpy(v->list_ids, list_ids, sizeof(int32_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&v->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    hipFree(v->cent); hipFree(v->list_off); hipFree(v->list_ids);
    if (v->done) hipEventDestroy(v->done);
    delete v;
    return e == hipErrorOutOfMemory ? fail(ANN_ENOMEM, "device memory for the IVF lists")
                                    : hip_fail(e, "IVF upload");
  }
  *out = v;
  return ANN_OK;
}

extern "C" int ann_ivf_free(ann_ivf* v) {
  if (!v) return ANN_OK;
  hipSetDevice(v->ix->device);
  hipDeviceSynchronize();
  hipFree(v->cent);
  hipFree(v->list_off);
  hipFree(v->list_ids);
  hipFree(v->probes);
  hipEventDestroy(v->done);
  delete v;
  return ANN_OK;
}

extern "C" int ann_ivf_search(ann_ivf* v, const ann_ivf_batch* b, void* stream) {
  if (!v || !b) return fail(ANN_EINVAL, "NULL argument");
  ann_index* ix = v->ix;
  if (b->mode == ANN_MODE_SPARSE) return fail(ANN_EUNSUP, "the IVF index serves dense and PQ modes");
  if (b->k < 1 || b->k > ANN_K_MAX) return fail(ANN_EINVAL, "k %d outside [1, %d]", b->k, ANN_K_MAX);
  if (b->nprobe < 1) return fail(ANN_EINVAL, "nprobe < 1");
  if (b->rerank < 0 || b->rerank > ANN_K_MAX) return fail(ANN_EINVAL, "rerank %d outside [0, %d]", b->rerank, ANN_K_MAX);
  ann_batch hb{};
  hb.mode = b->mode;
  hb.rerank = b->rerank;
  hb.nq = b->nq;
  hb.queries = b->queries;
  hb.k_all = hb.ef_all = hb.k_max = hb.ef_max = b->k;
  hb.out_ids = b->out_ids;
  hb.out_dists = b->out_dists;
  SearchParams P;
  int rc = make_params(ix, &hb, &P);
  if (rc) return rc;
  if (b->nq == 0) return ANN_OK;
  IvfArgs A{};
  A.nlist = v->nlist;
  A.nprobe = b->nprobe;
  A.np = std::min(b->nprobe, v->nlist);
  A.k = b->k;
  A.kk = std::max(b->k, b->rerank);
  A.sort_n = 1;
  while (A.sort_n < v->nlist) A.sort_n <<= 1;
  A.cent = v->cent;
  A.list_off = v->list_off;
  A.list_ids = v->list_ids;
  A.stats = b->out_stats;
  if (b->group < 0 || b->group > kMaxGroup)
    return fail(ANN_EINVAL, "group %d outside [0, %d]", b->group, kMaxGroup);
  if (P.mode == MODE_PQ && b->group > 1)
    return fail(ANN_EINVAL, "the PQ scan takes one query per workgroup (group 0 or 1)");
  // default: share the tiles when a query probes more than a quarter of the
  // lists (8 such queries overlap enough to pay for the shared staging;
  // measured on 1M x 768 with 1,024 lists: equal at nprobe 256, 2.6x faster
  // at nprobe 896, 2x slower at nprobe 64)
  A.group = b->group ? b->group : (P.mode != MODE_PQ && 4 * A.np > A.nlist ? kAutoGroup : 1);
  if (b->nq < A.group) A.group = (int)b->nq;
  auto r16 = [](size_t x) { return (x + 15) & ~size_t(15); };
  const int q_lds = P.q_lds_floats;
  size_t scan_lds = 0;
  if (A.group > 1) {
    P.q_lds_floats = 0;   // the shared scan reranks from the query in device memory
    A.wave_lds = (int)r16(scan_lds_bytes(P, A));
    // the tile takes what the waves leave of half the LDS (two workgroups per
    // compute unit), at most 64 rows; with less room, the whole LDS
    const size_t row_bytes = (size_t)P.nchunks * 16;
    const size_t fixed = 8 * (size_t)kIdChunk + r16(4 * (size_t)((A.nlist + 31) / 32)) + (size_t)A.group * A.wave_lds;
    auto fit = [&](size_t budget) {
      const size_t r = budget > fixed ? std::min<size_t>(64, (budget - fixed) / row_bytes) : 0;
      return (int)(r >= 8 ? r & ~size_t(7) : r);
    };
    A.tile_rows = fit(ix->lds_limit / ANN_IVF_SHARED_WG_PER_CU);
    if (A.tile_rows < 8) A.tile_rows = std::max(A.tile_rows, fit(ix->lds_limit));
    if (A.tile_rows >= 1) {
      A.tile_bytes = (int)(A.tile_rows * row_bytes);
      scan_lds = A.tile_bytes + fixed;
    } else if (b->group) {
      return fail(ANN_EBUDGET, "on-chip memory of the shared IVF scan: %d queries of %d bytes and rows of %zu bytes",
                  A.group, A.wave_lds, row_bytes);
    } else {
      A.group = 1;                       // the default falls back to one query per workgroup
      P.q_lds_floats = q_lds;
    }
  }
  if (A.group == 1) {
    A.wave_lds = (int)r16(scan_lds_bytes(P, A));
    scan_lds = A.wave_lds;
  }
  const void* scan = A.group > 1 ? scan_symbol<true>(P) : scan_symbol<false>(P);
  if (!scan) return fail(ANN_EBUDGET, "no IVF scan kernel for mode %d with %d lanes per row", P.mode, P.lanes_per_row);
  if (scan_lds > ix->lds_limit)
    return fail(ANN_EBUDGET, "on-chip memory of the IVF scan: %zu bytes > %zu", scan_lds, ix->lds_limit);
  // the probe kernel scores FP32 centroids with L2 keys, 64 lanes per centroid
  SearchParams C = P;
  C.mode = MODE_F32;
  C.metric = METRIC_L2;
  C.rows = v->cent;
  C.nchunks = ix->d / 4;
  C.lanes_per_row = 64;
  C.fp8_scale = nullptr;
  const void* probe = probe_symbol((C.nchunks + 63) / 64);
  const size_t probe_lds = 512 + 8 * (size_t)A.sort_n;
  if (!probe) return fail(ANN_EUNSUP, "centroids of %d dimensions", ix->d);

  std::lock_guard<std::mutex> g(v->mu);
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  hipStream_t st = stream ? (hipStream_t)stream : ix->stream;
  const int64_t need = b->nq * (int64_t)b->nprobe;
  if (b->out_probes) {
    A.probes = b->out_probes;
  } else {
    if (v->probes_cap < need) {
      HIP_OR_RETURN(hipEventSynchronize(v->done), "hipEventSynchronize");
      hipFree(v->probes);
      v->probes = nullptr;
      v->probes_cap = 0;
      hipError_t e = hipMalloc((void**)&v->probes, sizeof(int32_t) * (size_t)need);
      if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(ANN_ENOMEM, "probe scratch") : hip_fail(e, "hipMalloc (probes)");
      v->probes_cap = need;
    }
    // a batch on another stream may still read the scratch
    HIP_OR_RETURN(hipStreamWaitEvent(st, v->done, 0), "hipStreamWaitEvent");
    A.probes = v->probes;
  }
  HIP_OR_RETURN(launch(probe, b->nq, 64, probe_lds, st, C, A), "ivf_probe launch");
  HIP_OR_RETURN(launch(scan, (b->nq + A.group - 1) / A.group, 64 * A.group, scan_lds, st, P, A),
                "ivf_scan launch");
  if (!b->out_probes) HIP_OR_RETURN(hipEventRecord(v->done, st), "hipEventRecord");
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "IVF search");
  return ANN_OK;
}
