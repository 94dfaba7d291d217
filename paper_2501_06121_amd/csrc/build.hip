// HNSW construction on the device (dense FP32 rows), the index of the paper's
// Section 2 built as its citation's Algorithms 1 and 4 describe, in batches:
// every node of a batch searches the graph as it was before the batch, then
// the batch's links are applied.  This is the same schedule as the oracle's
// batched build, and every key uses the fixed FP32 order of the search, so
// the device graph equals the oracle's bit for bit.
//
// Per batch:
//  * build_choose: one wavefront per new node i (the query is row i).  From
//    the entry point, greedy descent through the layers above l_i (ef = 1);
//    then on each layer lc = min(L, l_i) .. 0 a beam search of width efC
//    whose entry set is the previous layer's result, and the neighbour
//    heuristic on its result: walk the candidates by increasing (key, id)
//    and keep one iff it is strictly closer to i than to every kept one,
//    until M are kept.  Node i's own lists are written directly (nothing in
//    the frozen graph links to i yet).
//  * the host groups the reverse links by (target, layer), sources in node
//    order;
//  * build_link: one wavefront per group appends the sources to the
//    target's list in order; whenever the list would exceed its capacity
//    (2M on layer 0, M above) the list plus the new source are sorted by
//    their keys to the target and cut back by the same heuristic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "ann.h"
#include "internal.h"
#include "search_impl.h"

namespace ann {
namespace {

struct BuildParams {
  int64_t first;             // batch nodes first .. first + count - 1
  int M, M0, efc, max_level, entry, nlev;   // nlev: layers kept per node in out_n
  const uint8_t* levels;
  int32_t* adj0;             // n x M0, -1 padded
  const int32_t* upper_off;  // per node, -1 for layer-0 nodes
  int32_t* upper_adj;        // lists x M, -1 padded
  int32_t* out_n;            // [count][nlev][M] chosen neighbours, -1 padded
  // build_link
  const int32_t* g_tgt;      // per group: target node, layer, first source
  const int32_t* g_lay;
  const int32_t* g_off;      // [groups + 1]
  const int32_t* g_src;
};

__device__ __forceinline__ int32_t* list_of(const BuildParams& b, int64_t v, int lc) {
  return lc == 0 ? b.adj0 + (size_t)v * b.M0 : b.upper_adj + ((size_t)b.upper_off[v] + lc - 1) * b.M;
}

// LDS of one build wavefront
struct BuildLds {
  float* wkey;      // [efc] beam
  uint32_t* wid;
  int32_t* rid;     // [64] kept neighbours of the heuristic
  float* ck2;       // [128] keys of a list being pruned
  int32_t* ci2;     // [128] its ids
};

// The neighbour heuristic over the sorted candidates (keys to the base in
// ckeys[0, nc), ids in cids): keep a candidate iff its key is strictly below
// its key to every kept one, until `cap` are kept.  `pe` scores rows against
// the candidate (its row as the query).  Returns the count kept (ids in
// bl.rid).  Whole wavefront.
template <class Policy>
__device__ int heuristic(const SearchParams& p, const Lds& s, const BuildLds& bl, Policy& pe,
                         const float* ckeys, const uint32_t* cids, int nc, int cap) {
  const int lane = lane_id();
  int kept = 0;
  for (int j = 0; j < nc && kept < cap; ++j) {
    const float ek = ckeys[j];
    const int e = (int)(cids[j] & kIdMask);
    bool keep = true;
    if (kept > 0) {
      // keys of candidate e to the kept ones: row e is the query
      pe.prep(p, s, e);
      if (lane < kept) s.cid[lane] = bl.rid[lane];
      wave_sync();
      pe.score(p, s, kept);
      wave_sync();
      const bool bad = lane < kept && !(ek < s.ckey[lane]);
      keep = !ballot(bad);
      wave_sync();
    }
    if (keep) {
      if (lane == 0) bl.rid[kept] = e;
      wave_sync();
      ++kept;
    }
  }
  return kept;
}

template <class Policy>
__global__ void __launch_bounds__(64) build_choose(SearchParams p, BuildParams b) {
  extern __shared__ __align__(16) char lds_raw[];
  // carve: search Lds (cid, ckey, rnk, ctl) + the build's own arrays
  Lds s = {};
  size_t off = 0;
  auto take = [&](size_t bytes) { char* r = lds_raw + off; off += (bytes + 15) & ~size_t(15); return r; };
  BuildLds bl;
  bl.wkey = (float*)take(4 * (size_t)b.efc);
  bl.wid = (uint32_t*)take(4 * (size_t)b.efc);
  bl.rid = (int32_t*)take(4 * 64);
  bl.ck2 = (float*)take(4 * 128);
  bl.ci2 = (int32_t*)take(4 * 128);
  s.cid = (int32_t*)take(4 * 64);
  s.ckey = (float*)take(4 * 64);
  s.rnk = (int32_t*)take(4 * 64);
  s.ctl = (int32_t*)take(4 * 16);
  s.wkey = bl.wkey;
  s.wid = bl.wid;

  const int lane = lane_id();
  const int slot = blockIdx.x;
  const int64_t t = blockIdx.x;
  const int64_t i = b.first + t;
  const int li = b.levels[i];
  int32_t* on = b.out_n + (size_t)t * b.nlev * b.M;
  for (int j = lane; j < b.nlev * b.M; j += 64) on[j] = -1;
  if (b.entry < 0) return;                // the first node: no neighbours
  Policy pol, pe;
  pol.prep(p, s, i);
  QueryState st{0, 0, 0, 0, false};
  uint32_t* bits = p.bits + (size_t)slot * p.bits_words;

  int cur = b.entry;
  if (lane == 0) s.cid[0] = cur;
  wave_sync();
  pol.score(p, s, 1);
  wave_sync();
  float ckey = s.ckey[0];
  // greedy descent on the layers above l_i
  for (int lc = b.max_level; lc > li; --lc) {
    while (true) {
      const int uo = b.upper_off[cur];
      int nb = -1;
      if (lane < b.M && uo >= 0) nb = b.upper_adj[((size_t)uo + lc - 1) * b.M + lane];
      const uint64_t mk = ballot(nb >= 0);
      const int m = __builtin_popcountll(mk);
      if (m == 0) break;
      wave_sync();
      if (nb >= 0) s.cid[mbcnt(mk)] = nb;
      wave_sync();
      pol.score(p, s, m);
      wave_sync();
      float bk = (lane < m) ? s.ckey[lane] : __builtin_inff();
      uint32_t bi = (lane < m) ? (uint32_t)s.cid[lane] : kIdMask;
#pragma unroll
      for (int sft = 32; sft >= 1; sft >>= 1) {
        const float ok = __shfl_xor(bk, sft, 64);
        const uint32_t oi = (uint32_t)__shfl_xor((int)bi, sft, 64);
        if (kid_lt(ok, oi, bk, bi)) { bk = ok; bi = oi; }
      }
      if (kid_lt(bk, bi, ckey, (uint32_t)cur)) {
        cur = uniform_int((int)bi);
        ckey = __builtin_bit_cast(float, uniform_int(__builtin_bit_cast(int, bk)));
      } else {
        break;
      }
    }
  }
  // beam searches of width efC, layers min(L, l_i) .. 0; W carries over as
  // the next layer's entry set (all entries unexpanded again)
  int w = 1;
  if (lane == 0) { bl.wkey[0] = ckey; bl.wid[0] = (uint32_t)cur; }
  wave_sync();
  const int top = b.max_level < li ? b.max_level : li;
  for (int lc = top; lc >= 0; --lc) {
    const int cap = lc == 0 ? b.M0 : b.M;
    // entry set: unexpanded, visited
    for (int j = lane; j < w; j += 64) bl.wid[j] &= kIdMask;
    wave_sync();
    for (int j0 = 0; j0 < w; j0 += 64) {
      const int j = j0 + lane;
      bool isnew = false;
      int id = -1;
      if (j < w) {
        id = (int)bl.wid[j];
        const uint32_t bit = 1u << (id & 31);
        isnew = !(atomicOr(&bits[id >> 5], bit) & bit);
      }
      log_visited(p, slot, i, st, isnew, id, ballot(isnew));
    }
    int hint = 0;
    ListCache lc_unused{-1, -1, 0.0f, kExpanded};
    int wb_unused = 0;
    while (true) {
      const Head hd = beam_head<false>(s, List{bl.wkey, bl.wid}, w, wb_unused, b.efc, hint, 0, false,
                                       lc_unused);
      if (hd.pm < 0) break;
      const int c = (int)hd.mi;
      hint = hd.pm + 1;
      int nb = -1;
      if (lane < cap) {
        if (lc == 0) nb = b.adj0[(size_t)c * b.M0 + lane];
        else nb = b.upper_adj[((size_t)b.upper_off[c] + lc - 1) * b.M + lane];
      }
      bool isnew = false;
      if (nb >= 0) {
        const uint32_t bit = 1u << (nb & 31);
        isnew = !(atomicOr(&bits[nb >> 5], bit) & bit);
      }
      const uint64_t mk = ballot(isnew);
      log_visited(p, slot, i, st, isnew, nb, mk);
      wave_sync();
      if (lane == 0) bl.wid[hd.pm] = (uint32_t)c | kExpanded;
      if (isnew) s.cid[mbcnt(mk)] = nb;
      wave_sync();
      const int m = __builtin_popcountll(mk);
      if (m == 0) continue;
      pol.score(p, s, m);
      wave_sync();
      const bool full = w >= b.efc;
      float kk = __builtin_inff();
      uint32_t ki = kIdMask;
      bool keep = false;
      if (lane < m) {
        kk = s.ckey[lane];
        ki = (uint32_t)s.cid[lane];
        keep = !full || kid_lt(kk, ki, hd.tk, hd.ti);
      }
      const uint64_t km = ballot(keep);
      const int mnew = __builtin_popcountll(km);
      if (mnew == 0) continue;
      int rk = 0;
      for (uint64_t rem = km; rem; rem &= rem - 1) {
        const int l = __builtin_ctzll(rem);
        const float ok = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kk), l));
        const uint32_t oi = (uint32_t)__builtin_amdgcn_readlane((int)ki, l);
        rk += kid_lt(ok, oi, kk, ki) ? 1 : 0;
      }
      wave_sync();
      if (keep) { s.ckey[rk] = kk; s.cid[rk] = (int32_t)ki; }
      wave_sync();
      w = merge_sorted<4>(bl.wkey, bl.wid, w, b.efc, s.ckey, (const uint32_t*)s.cid, mnew,
                          &s.ctl[CTL_R0], nullptr, nullptr);
      const int r0 = s.ctl[CTL_R0];
      if (r0 < hint) hint = r0;
    }
    // a fresh visited set for the next layer
    if (!st.vlog_overflow) {
      const int32_t* lg = p.vlog + (size_t)slot * p.vlog_cap;
      for (int j = lane; j < st.vlog_n; j += 64) bits[lg[j] >> 5] = 0u;
    } else {
      for (int64_t j = lane; j < p.bits_words; j += 64) bits[j] = 0u;
    }
    st.vlog_n = 0;
    st.vlog_overflow = false;
    __threadfence_block();
    wave_sync();
    // node i's neighbours on this layer
    const int kept = heuristic(p, s, bl, pe, bl.wkey, bl.wid, w, b.M);
    if (lane < kept) {
      on[lc * b.M + lane] = bl.rid[lane];
      list_of(b, i, lc)[lane] = bl.rid[lane];
    }
    wave_sync();
  }
}

// One group of reverse links: sources g_src[g_off[g] ..] appended in order to
// the list of (g_tgt[g], g_lay[g]); an overflowing list is cut back to its
// capacity by the heuristic over its entries sorted by key to the target.
template <class Policy>
__global__ void __launch_bounds__(64) build_link(SearchParams p, BuildParams b) {
  extern __shared__ __align__(16) char lds_raw[];
  Lds s = {};
  size_t off = 0;
  auto take = [&](size_t bytes) { char* r = lds_raw + off; off += (bytes + 15) & ~size_t(15); return r; };
  BuildLds bl;
  bl.rid = (int32_t*)take(4 * 64);
  bl.ck2 = (float*)take(4 * 128);
  bl.ci2 = (int32_t*)take(4 * 128);
  s.cid = (int32_t*)take(4 * 128);
  s.ckey = (float*)take(4 * 128);
  s.ctl = (int32_t*)take(4 * 16);
  const int lane = lane_id();
  const int g = blockIdx.x;
  const int e = b.g_tgt[g];
  const int lc = b.g_lay[g];
  const int cap = lc == 0 ? b.M0 : b.M;
  int32_t* L = list_of(b, e, lc);
  // current length: valid ids first, -1 padded
  const int v0 = lane < cap ? L[lane] : -1;
  int cnt = __builtin_popcountll(ballot(v0 >= 0));
  Policy pt, pe;
  bool pt_ready = false;
  for (int si = b.g_off[g]; si < b.g_off[g + 1]; ++si) {
    const int src = b.g_src[si];
    if (cnt < cap) {
      if (lane == 0) L[cnt] = src;
      ++cnt;
      continue;
    }
    // prune: the list and the new source, sorted by key to e, heuristic to cap
    if (!pt_ready) { pt.prep(p, s, e); pt_ready = true; }
    const int nc = cnt + 1;
    __threadfence_block();
    wave_sync();
    for (int j = lane; j < nc; j += 64) s.cid[j] = j < cnt ? L[j] : src;
    wave_sync();
    pt.score(p, s, nc);
    wave_sync();
    // rank sort by (key, id)
    for (int j = lane; j < nc; j += 64) {
      const float kj = s.ckey[j];
      const uint32_t ij = (uint32_t)s.cid[j];
      int r = 0;
      for (int u = 0; u < nc; ++u) r += kid_lt(s.ckey[u], (uint32_t)s.cid[u], kj, ij) ? 1 : 0;
      bl.ck2[r] = kj;
      bl.ci2[r] = (int32_t)ij;
    }
    wave_sync();
    const int kept = heuristic(p, s, bl, pe, bl.ck2, (const uint32_t*)bl.ci2, nc, cap);
    for (int j = lane; j < cap; j += 64) L[j] = j < kept ? bl.rid[j] : -1;
    __threadfence_block();
    wave_sync();
    cnt = kept;
  }
}

template <class Policy>
hipError_t run_choose(const SearchParams& p, const BuildParams& b, int64_t count, hipStream_t st) {
  const size_t lds = 2 * (size_t)((4 * b.efc + 15) & ~15) + 256 + 512 + 512 + 256 * 3 + 64 + 64;
  if (lds > 65536) hipFuncSetAttribute((const void*)build_choose<Policy>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(build_choose<Policy>, dim3((unsigned)count), dim3(64), lds, st, p, b);
  return hipGetLastError();
}

template <class Policy>
hipError_t run_link(const SearchParams& p, const BuildParams& b, int64_t groups, hipStream_t st) {
  const size_t lds = 256 + 512 + 512 + 512 + 512 + 64 + 64;
  hipLaunchKernelGGL(build_link<Policy>, dim3((unsigned)groups), dim3(64), lds, st, p, b);
  return hipGetLastError();
}

typedef hipError_t (*ChooseFn)(const SearchParams&, const BuildParams&, int64_t, hipStream_t);
typedef hipError_t (*LinkFn)(const SearchParams&, const BuildParams&, int64_t, hipStream_t);

// FP32 rows, one row per wavefront group of L lanes with CPL chunks each
bool pick_build_kernels(int nchunks, int* lanes, ChooseFn* cf, LinkFn* lf) {
#define ANN_BUILD_SHAPE(L, C)                                  \
  if (nchunks <= (L) * (C)) {                                  \
    *lanes = L;                                                \
    *cf = run_choose<Dense<MODE_F32, L, C>>;                   \
    *lf = run_link<Dense<MODE_F32, L, C>>;                     \
    return true;                                               \
  }
  ANN_BUILD_SHAPE(16, 1)
  ANN_BUILD_SHAPE(32, 1)
  ANN_BUILD_SHAPE(64, 1)
  ANN_BUILD_SHAPE(64, 2)
  ANN_BUILD_SHAPE(64, 3)
  ANN_BUILD_SHAPE(64, 4)
#undef ANN_BUILD_SHAPE
  return false;
}

}  // namespace
}  // namespace ann

// A graph built on the device, exported to host arrays in the index layout.
struct ann_graph {
  int64_t n = 0;
  int M = 0, M0 = 0, max_level = -1, entry = -1;
  int64_t nlists = 0;
  std::vector<uint8_t> levels;
  std::vector<int32_t> adj0, upper_off, upper_adj;
};

using namespace ann;

namespace {

struct DeviceArrays {
  std::vector<void*> ptrs;
  ~DeviceArrays() { for (void* q : ptrs) if (q) (void)hipFree(q); }
  template <class T>
  hipError_t alloc(T** out, size_t count) {
    *out = nullptr;
    hipError_t e = hipMalloc((void**)out, std::max<size_t>(1, count) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(*out);
    return e;
  }
};

}  // namespace

extern "C" int ann_hnsw_build(const float* X, int64_t n, int32_t d, int32_t metric, int32_t M,
                              int32_t efc, const double* u, int64_t seq_prefix, double batch_frac,
                              int64_t batch_cap, ann_graph** out, void* stream) {
  if (!out) return fail(ANN_EINVAL, "NULL output");
  *out = nullptr;
  if (!X || !u) return fail(ANN_EINVAL, "NULL pointer");
  if (n < 1 || n > INT32_MAX - 1) return fail(ANN_EINVAL, "n %lld outside [1, 2^31 - 2]", (long long)n);
  if (d < 4 || d % 4 != 0 || d > 1024) return fail(ANN_EUNSUP, "d %d: needs a multiple of 4, at most 1024", d);
  if (metric != ANN_METRIC_L2 && metric != ANN_METRIC_IP) return fail(ANN_EINVAL, "unknown metric %d", metric);
  if (M < 2 || M > 32) return fail(ANN_EINVAL, "M %d outside [2, 32]", M);
  if (efc < 1 || efc > 4096) return fail(ANN_EINVAL, "efConstruction %d outside [1, 4096]", efc);
  if (seq_prefix < 0 || batch_frac < 0 || batch_cap < 1) return fail(ANN_EINVAL, "bad batch schedule");
  int lanes = 0;
  ChooseFn choose = nullptr;
  LinkFn link = nullptr;
  if (!pick_build_kernels(d / 4, &lanes, &choose, &link)) return fail(ANN_EUNSUP, "d %d", d);
  hipStream_t st = (hipStream_t)stream;
  const int M0 = 2 * M;
  // levels: floor(-ln(1 - u) / ln M), at most 30
  std::vector<uint8_t> levels((size_t)n);
  const double mL = 1.0 / std::log((double)M);
  int top = 0;
  for (int64_t i = 0; i < n; ++i) {
    const double l = std::floor(-std::log(1.0 - u[i]) * mL);
    levels[i] = (uint8_t)std::min(l, 30.0);
    top = std::max<int>(top, levels[i]);
  }
  std::vector<int32_t> upper_off((size_t)n, -1);
  int64_t nlists = 0;
  for (int64_t i = 0; i < n; ++i)
    if (levels[i] > 0) { upper_off[i] = (int32_t)nlists; nlists += levels[i]; }
  const int nlev = top + 1;
  const int64_t bmax = batch_frac > 0 ? std::max<int64_t>(1, batch_cap) : 1;
  const int64_t words = (n + 31) / 32;
  const int vlog_cap = (int)std::max<int64_t>(256, std::min<int64_t>(n / 64, 1 << 20));
  DeviceArrays dev;
  uint8_t* d_levels;
  int32_t *d_adj0, *d_uoff, *d_uadj, *d_outn, *d_vlog, *d_gt, *d_gl, *d_go, *d_gs;
  uint32_t* d_bits;
  const int64_t max_pairs = bmax * nlev * M;
  HIP_OR_RETURN(dev.alloc(&d_levels, (size_t)n), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_adj0, (size_t)n * M0), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_uoff, (size_t)n), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_uadj, (size_t)nlists * M), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_outn, (size_t)max_pairs), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_bits, (size_t)bmax * words), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_vlog, (size_t)bmax * vlog_cap), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_gt, (size_t)max_pairs), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_gl, (size_t)max_pairs), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_go, (size_t)max_pairs + 1), "hipMalloc (build)");
  HIP_OR_RETURN(dev.alloc(&d_gs, (size_t)max_pairs), "hipMalloc (build)");
  HIP_OR_RETURN(hipMemcpyAsync(d_levels, levels.data(), (size_t)n, hipMemcpyHostToDevice, st), "upload");
  HIP_OR_RETURN(hipMemcpyAsync(d_uoff, upper_off.data(), (size_t)n * 4, hipMemcpyHostToDevice, st), "upload");
  HIP_OR_RETURN(hipMemsetAsync(d_adj0, 0xFF, (size_t)n * M0 * 4, st), "memset");
  if (nlists) HIP_OR_RETURN(hipMemsetAsync(d_uadj, 0xFF, (size_t)nlists * M * 4, st), "memset");
  HIP_OR_RETURN(hipMemsetAsync(d_bits, 0, (size_t)bmax * words * 4, st), "memset");

  SearchParams p;
  std::memset(&p, 0, sizeof p);
  p.mode = MODE_F32;
  p.metric = metric == ANN_METRIC_IP ? METRIC_IP : METRIC_L2;
  p.d = d;
  p.nchunks = d / 4;
  p.lanes_per_row = lanes;
  p.waves_per_query = 1;
  p.rows = X;
  p.queries = X;
  p.x_f32 = X;
  p.n = n;
  p.M = M;
  p.M0 = M0;
  p.bits = d_bits;
  p.bits_words = words;
  p.vlog = d_vlog;
  p.vlog_cap = vlog_cap;
  BuildParams b;
  std::memset(&b, 0, sizeof b);
  b.M = M; b.M0 = M0; b.efc = efc; b.nlev = nlev;
  b.levels = d_levels; b.adj0 = d_adj0; b.upper_off = d_uoff; b.upper_adj = d_uadj; b.out_n = d_outn;
  b.g_tgt = d_gt; b.g_lay = d_gl; b.g_off = d_go; b.g_src = d_gs;

  int max_level = -1, entry = -1;
  std::vector<int32_t> hn((size_t)max_pairs);
  std::vector<std::pair<int64_t, int32_t>> rev;
  std::vector<int32_t> gt, gl, go, gs;
  int64_t done = 0;
  while (done < n) {
    int64_t bsz = 1;
    if (done >= seq_prefix && batch_frac > 0)
      bsz = std::max<int64_t>(1, std::min<int64_t>(batch_cap, (int64_t)(done * batch_frac)));
    bsz = std::min(bsz, n - done);
    b.first = done;
    b.max_level = max_level;
    b.entry = entry;
    HIP_OR_RETURN(choose(p, b, bsz, st), "build_choose launch");
    const size_t nn = (size_t)bsz * nlev * M;
    HIP_OR_RETURN(hipMemcpyAsync(hn.data(), d_outn, nn * 4, hipMemcpyDeviceToHost, st), "download");
    HIP_OR_RETURN(hipStreamSynchronize(st), "build_choose");
    // reverse links grouped by (target, layer), sources in node order
    rev.clear();
    for (int64_t t = 0; t < bsz; ++t)
      for (int lc = 0; lc < nlev; ++lc)
        for (int j = 0; j < M; ++j) {
          const int32_t e = hn[((size_t)t * nlev + lc) * M + j];
          if (e >= 0) rev.emplace_back((int64_t)e * 32 + lc, (int32_t)(done + t));
        }
    std::stable_sort(rev.begin(), rev.end(),
                     [](const std::pair<int64_t, int32_t>& a, const std::pair<int64_t, int32_t>& c) {
                       return a.first < c.first;
                     });
    gt.clear(); gl.clear(); go.clear(); gs.clear();
    for (size_t j = 0; j < rev.size(); ++j) {
      if (j == 0 || rev[j].first != rev[j - 1].first) {
        gt.push_back((int32_t)(rev[j].first / 32));
        gl.push_back((int32_t)(rev[j].first % 32));
        go.push_back((int32_t)j);
      }
      gs.push_back(rev[j].second);
    }
    go.push_back((int32_t)rev.size());
    const int64_t groups = (int64_t)gt.size();
    if (groups > 0) {
      HIP_OR_RETURN(hipMemcpyAsync(d_gt, gt.data(), gt.size() * 4, hipMemcpyHostToDevice, st), "upload");
      HIP_OR_RETURN(hipMemcpyAsync(d_gl, gl.data(), gl.size() * 4, hipMemcpyHostToDevice, st), "upload");
      HIP_OR_RETURN(hipMemcpyAsync(d_go, go.data(), go.size() * 4, hipMemcpyHostToDevice, st), "upload");
      HIP_OR_RETURN(hipMemcpyAsync(d_gs, gs.data(), gs.size() * 4, hipMemcpyHostToDevice, st), "upload");
      HIP_OR_RETURN(link(p, b, groups, st), "build_link launch");
      // the host vectors are reused by the next batch only after it synchronizes
    }
    for (int64_t t = 0; t < bsz; ++t)
      if ((int)levels[done + t] > max_level) { max_level = levels[done + t]; entry = (int32_t)(done + t); }
    done += bsz;
  }
  auto* g = new ann_graph;
  g->n = n; g->M = M; g->M0 = M0; g->max_level = max_level; g->entry = entry; g->nlists = nlists;
  g->levels = levels;
  g->upper_off = upper_off;
  g->adj0.resize((size_t)n * M0);
  g->upper_adj.resize((size_t)nlists * M);
  hipError_t e = hipMemcpyAsync(g->adj0.data(), d_adj0, (size_t)n * M0 * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && nlists)
    e = hipMemcpyAsync(g->upper_adj.data(), d_uadj, (size_t)nlists * M * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { delete g; return hip_fail(e, "build download"); }
  *out = g;
  return ANN_OK;
}

extern "C" int ann_graph_info(const ann_graph* g, int64_t* info) {
  if (!g || !info) return fail(ANN_EINVAL, "NULL argument");
  info[0] = g->n; info[1] = g->M; info[2] = g->M0; info[3] = g->max_level; info[4] = g->entry;
  info[5] = g->nlists;
  return ANN_OK;
}

extern "C" int ann_graph_export(const ann_graph* g, uint8_t* levels, int32_t* adj0, int32_t* upper_off,
                                int32_t* upper_adj) {
  if (!g || !levels || !adj0 || !upper_off || (g->nlists && !upper_adj)) return fail(ANN_EINVAL, "NULL argument");
  std::memcpy(levels, g->levels.data(), g->levels.size());
  std::memcpy(adj0, g->adj0.data(), g->adj0.size() * 4);
  std::memcpy(upper_off, g->upper_off.data(), g->upper_off.size() * 4);
  if (g->nlists) std::memcpy(upper_adj, g->upper_adj.data(), g->upper_adj.size() * 4);
  return ANN_OK;
}

extern "C" int ann_graph_free(ann_graph* g) {
  delete g;
  return ANN_OK;
}
