// Exact k-nearest neighbours on matrix cores (MFMA), used as ground truth.
//
// The k-NN problem of the paper (Section 1: the k nearest neighbours of a
// query among a dataset X of d-dimensional vectors) solved by a full scan:
//
// Stage 1 (bf_tiles): a workgroup of 4 wavefronts owns 128 queries and a
//   contiguous range of base rows.  For each tile of 64 base rows it forms the
//   128 x 64 block of dot products with v_mfma_f32_16x16x4_f32 (operands
//   staged through LDS in slices of 16 dimensions), turns them into
//   approximate keys (-dot, or |x|^2 - 2 dot for L2: |q|^2 is the same for
//   every row of a query), and merges the survivors of a per-query threshold
//   into a sorted top-64 list per query held in LDS.  At the end the lists go
//   to scratch memory: 64 candidates per (query, range).
// Stage 2 (bf_finish): one wavefront per query merges the candidate lists of
//   all ranges into the approximate top-64, re-scores the best k + 16 with the
//   FP32 rows in the same fixed order as the search kernel, sorts them by
//   (key, id) and writes the first k.  The result is certified exact when the
//   k-th exact key plus the worst-case difference between the MFMA and the
//   fixed-order evaluations stays below the approximate key of every
//   candidate that was not re-scored.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ann.h"
#include "internal.h"
#include "search_kernels.h"

namespace ann {
namespace {

constexpr int BM = 128;     // queries per workgroup
constexpr int BN = 64;      // base rows per tile
constexpr int BK = 16;      // dimensions per LDS slice
constexpr int KC = 64;      // candidates kept per query and range
constexpr int kRescore = 16;

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
  int d;
  int metric;
  const float* Q;
  int64_t nq;
  int64_t rows_per_range;
  int nranges;
  float* cand_key;       // [nq][nranges][KC]
  int32_t* cand_id;
};

__global__ void __launch_bounds__(256) bf_tiles(BfParams p) {
  __shared__ float sq[2][BM][BK + 1];
  __shared__ float sx[2][BN][BK + 1];
  __shared__ float tile[BM][BN + 1];
  __shared__ float lk[BM][KC];
  __shared__ int li[BM][KC];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int64_t q0 = (int64_t)blockIdx.x * BM;
  const int range = blockIdx.y;
  const int64_t r_begin = (int64_t)range * p.rows_per_range;
  const int64_t r_end = r_begin + p.rows_per_range < p.n ? r_begin + p.rows_per_range : p.n;

  for (int i = tid; i < BM * KC; i += 256) {
    lk[i / KC][i % KC] = __builtin_inff();
    li[i / KC][i % KC] = 0x7FFFFFFF;
  }
  __syncthreads();

  for (int64_t t0 = r_begin; t0 < r_end; t0 += BN) {
    floatx4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    // slice loader: 128 x 16 query floats and 64 x 16 base floats
    auto load_slice = [&](int buf, int k0) {
      for (int i = tid; i < BM * BK; i += 256) {
        const int r = i / BK, c = i % BK;
        const int64_t qi = q0 + r;
        sq[buf][r][c] = (qi < p.nq && k0 + c < p.d) ? p.Q[qi * p.d + k0 + c] : 0.0f;
      }
      for (int i = tid; i < BN * BK; i += 256) {
        const int r = i / BK, c = i % BK;
        const int64_t xi = t0 + r;
        sx[buf][r][c] = (xi < r_end && k0 + c < p.d) ? p.X[xi * p.d + k0 + c] : 0.0f;
      }
    };
    load_slice(0, 0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < p.d; k0 += BK) {
      if (k0 + BK < p.d) load_slice(buf ^ 1, k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float a[2], b[4];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) a[rb] = sq[buf][wave * 32 + rb * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) b[cb] = sx[buf][cb * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
      }
      __syncthreads();
      buf ^= 1;
    }
    // approximate keys into the tile: row 16*rb + 4*(lane/16) + r, col 16*cb + lane%16
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wave * 32 + rb * 16 + 4 * (lane >> 4) + r;
          const int col = cb * 16 + (lane & 15);
          const int64_t xi = t0 + col;
          float key = __builtin_inff();
          if (xi < r_end) {
            const float dot = acc[rb][cb][r];
            key = (p.metric == METRIC_IP) ? -dot : p.x2[xi] - 2.0f * dot;
          }
          tile[row][col] = key;
        }
    __syncthreads();
    // each wave merges its 32 rows
    for (int rr = 0; rr < 32; ++rr) {
      const int row = wave * 32 + rr;
      if (q0 + row >= p.nq) break;
      const float thr_k = lk[row][KC - 1];
      const int thr_i = li[row][KC - 1];
      float k = tile[row][lane];
      // columns past the range are empty entries (+inf, largest id)
      int id = (t0 + lane < r_end) ? (int)(t0 + lane) : 0x7FFFFFFF;
      const bool keep = kid_less(k, id, thr_k, thr_i);
      if (!__ballot(keep)) continue;
      if (!keep) { k = __builtin_inff(); id = 0x7FFFFFFF; }
      merge_list(lk[row], li[row], k, id);
    }
    __syncthreads();
  }
  for (int i = tid; i < BM * KC; i += 256) {
    const int r = i / KC, c = i % KC;
    const int64_t qi = q0 + r;
    if (qi < p.nq) {
      const size_t o = ((size_t)qi * p.nranges + range) * KC + c;
      p.cand_key[o] = lk[r][c];
      p.cand_id[o] = li[r][c];
    }
  }
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
  lk[lane] = __builtin_inff();
  li[lane] = 0x7FFFFFFF;
  __syncthreads();
  for (int r = 0; r < p.nranges; ++r) {
    const size_t o = ((size_t)q * p.nranges + r) * KC + lane;
    merge_list(lk, li, p.cand_key[o], p.cand_id[o]);
  }
  const float* qr = p.Q + q * p.d;
  // |q|_1 and |q|^2 for the error bound and the L2 offset
  float a1 = 0.f, q2 = 0.f;
  for (int i = lane; i < p.d; i += 64) { a1 += fabsf(qr[i]); q2 = __builtin_fmaf(qr[i], qr[i], q2); }
  for (int s = 32; s >= 1; s >>= 1) { a1 += __shfl_xor(a1, s, 64); q2 += __shfl_xor(q2, s, 64); }
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
  E *= (p.metric == METRIC_IP) ? a1 * p.xmax : 2.0f * a1 * p.xmax + p.x2max + q2;
  float kth = __shfl(kx, 0, 64);
  for (int j = 0; j < 64; ++j) {
    const int rj = __shfl(rank, j, 64);
    if (rj == p.k - 1) kth = __shfl(kx, j, 64);
  }
  float thr = (R < KC) ? lk[R] : __builtin_inff();
  if (p.metric != METRIC_IP) thr += q2;
  if (lane == 0 && p.out_certified) p.out_certified[q] = (R >= KC) || (kth + E < thr) ? 1 : 0;
}

}  // namespace

size_t bruteforce_scratch_bytes(int64_t n, int64_t nq, int k) {
  (void)k;
  const int nranges = n < 65536 ? 1 : 8;
  return (size_t)nq * nranges * KC * 8 + (size_t)n * 4 + 256;
}

}  // namespace ann

using namespace ann;

extern "C" int ann_bruteforce(const ann_index* cix, const float* queries, int64_t nq, int32_t k,
                              int64_t* out_ids, float* out_dists, int32_t* out_certified,
                              void* stream) {
  if (!cix) return fail(ANN_EINVAL, "index is NULL");
  ann_index* ix = const_cast<ann_index*>(cix);
  if (!ix->x_f32) return fail(ANN_EUNSUP, "brute force needs the FP32 rows");
  if (k < 1 || k > KC - kRescore) return fail(ANN_EINVAL, "k %d outside [1, %d]", k, KC - kRescore);
  if (nq < 0) return fail(ANN_EINVAL, "nq < 0");
  if (nq == 0) return ANN_OK;
  if (!queries || !out_ids || !out_dists) return fail(ANN_EINVAL, "NULL pointer");
  std::lock_guard<std::mutex> lock(ix->mu);
  HIP_OR_RETURN(hipSetDevice(ix->device), "hipSetDevice");
  hipStream_t st = stream ? (hipStream_t)stream : ix->stream;
  const int nranges = ix->n < 65536 ? 1 : 8;
  const size_t need = bruteforce_scratch_bytes(ix->n, nq, k);
  if (ix->bf_scratch_bytes < need) {
    if (ix->bf_scratch) {
      HIP_OR_RETURN(hipStreamSynchronize(st), "hipStreamSynchronize");
      (void)hipFree(ix->bf_scratch);
      ix->bf_scratch = nullptr;
      ix->bf_scratch_bytes = 0;
    }
    HIP_OR_RETURN(hipMalloc(&ix->bf_scratch, need), "hipMalloc (brute-force scratch)");
    ix->bf_scratch_bytes = need;
    ix->bf_norms_ready = false;
  }
  char* base = (char*)ix->bf_scratch;
  float* x2 = (float*)base;
  float* ckey = (float*)(base + (((size_t)ix->n * 4 + 255) & ~size_t(255)));
  int32_t* cid = (int32_t*)(ckey + (size_t)nq * nranges * KC);
  if (!ix->bf_norms_ready) {
    hipLaunchKernelGGL(bf_norms, dim3((unsigned)ix->n), dim3(64), 0, st, ix->x_f32, ix->n, ix->d, x2);
    HIP_OR_RETURN(hipGetLastError(), "bf_norms launch");
    ix->bf_norms_ready = true;
  }
  BfParams p;
  p.X = ix->x_f32; p.x2 = x2; p.n = ix->n; p.d = ix->d; p.metric = ix->metric;
  p.Q = queries; p.nq = nq; p.nranges = nranges;
  p.rows_per_range = (ix->n + nranges - 1) / nranges;
  p.cand_key = ckey; p.cand_id = cid;
  const dim3 grid((unsigned)((nq + BM - 1) / BM), (unsigned)nranges);
  hipLaunchKernelGGL(bf_tiles, grid, dim3(256), 0, st, p);
  HIP_OR_RETURN(hipGetLastError(), "bf_tiles launch");
  BfFinish f;
  f.X = ix->x_f32; f.n = ix->n; f.d = ix->d; f.metric = ix->metric; f.Q = queries; f.nq = nq;
  f.nranges = nranges; f.cand_key = ckey; f.cand_id = cid; f.k = k;
  f.xmax = ix->xmax; f.x2max = ix->x2max;
  f.out_ids = out_ids; f.out_dists = out_dists; f.out_certified = out_certified;
  hipLaunchKernelGGL(bf_finish, dim3((unsigned)nq), dim3(64), 0, st, f);
  HIP_OR_RETURN(hipGetLastError(), "bf_finish launch");
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "brute force");
  return ANN_OK;
}
