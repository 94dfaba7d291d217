// CPU oracle for batched HNSW search -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct reference for what the GPU library
// computes.  Only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark may load it; the product path never does.  It shares no code,
// header, table or constant with the GPU library.
//
// What it follows (arXiv 2501.06121, "kANNolo"):
//  * the k-nearest-neighbour problem over a dataset of d-dimensional vectors
//    (Section 1);
//  * dense vectors with L2 or inner product, sparse vectors with inner
//    product (Section 3, Table 1);
//  * the HNSW index (Section 2, "The indexing method ... HNSW" and its
//    citation: Malkov & Yashunin, Algorithms 1, 2, 4 and 5), built on the
//    original vectors even when a quantized representation is searched
//    (Section 3.1, "Performance");
//  * Product Quantization (Section 2 and its citation: Jegou et al.), with
//    asymmetric distances from per-query lookup tables;
//  * the Identity quantizer (Section 2), plus reduced-precision storage
//    copies (FP16, BF16, FP8-E4M3 with a per-vector scale);
//  * an inverted-file (IVF) index over a k-means coarse quantizer, the index
//    family Section 1 names beside graphs and Section 4 (Conclusions and Future Work) plans to add.
//
// Distances are "keys", smaller is better: squared L2, or the negated inner
// product.  Two evaluation modes exist:
//  * EXACT: products and sums in FP64 from the FP32 (or exactly up-converted)
//    inputs, rounded once to FP32.
//  * CANON: a fixed FP32 evaluation order that the GPU reproduces bit for bit.
//    64 partial sums start at +0.  Element i belongs to chunk g = i / c, where
//    c = 16 bytes / element size (FP32 4, FP16/BF16 8, FP8 16, sparse 1), and
//    chunk g feeds partial g mod 64.  Each partial takes fmaf() over its
//    elements in ascending i.  The 64 partials are then folded by the xor
//    tree p[l] = p[l] + p[l ^ s] for s = 32, 16, 8, 4, 2, 1, and the result is
//    p[0].  This order is this project's reading: the paper fixes no order.
//
// Ties are broken by the total order on (key, id) everywhere.
//
// Build: g++ -O2 -fopenmp -mavx2 -mfma -ffp-contract=off -fPIC -shared.
// -ffp-contract=off keeps every multiply and add as written; fmaf() is the
// only fused operation.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <cstdio>
#include <vector>
#include <queue>
#include <algorithm>
#include <utility>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// Number formats (storage copies of the Identity quantizer)
// ---------------------------------------------------------------------------

// IEEE half: 1 sign, 5 exponent (bias 15), 10 mantissa bits.  Round to
// nearest even, overflow to infinity.
uint16_t f32_to_f16(float x) {
  uint32_t bits; std::memcpy(&bits, &x, 4);
  uint16_t sign = (uint16_t)((bits >> 16) & 0x8000u);
  if (std::isnan(x)) return (uint16_t)(sign | 0x7E00u);
  double a = std::fabs((double)x);
  if (a >= 65520.0) return (uint16_t)(sign | 0x7C00u);     // rounds to inf
  if (a < std::ldexp(1.0, -14)) {                           // subnormal range
    double q = std::nearbyint(a * std::ldexp(1.0, 24));     // units of 2^-24
    return (uint16_t)(sign | (uint16_t)q);                  // q = 1024 -> min normal
  }
  int e; std::frexp(a, &e); e -= 1;                          // a in [2^e, 2^(e+1))
  double m = std::nearbyint(a * std::ldexp(1.0, 10 - e));    // in [1024, 2048]
  if (m >= 2048.0) { m = 1024.0; e += 1; }
  if (e > 15) return (uint16_t)(sign | 0x7C00u);
  return (uint16_t)(sign | (uint16_t)((e + 15) << 10) | (uint16_t)((int)m - 1024));
}

float f16_to_f32(uint16_t h) {
  int s = (h >> 15) & 1, e = (h >> 10) & 31, m = h & 1023;
  double v;
  if (e == 0) v = std::ldexp((double)m, -24);
  else if (e == 31) v = m ? NAN : INFINITY;
  else v = std::ldexp((double)(1024 + m), e - 25);
  return (float)(s ? -v : v);
}

// bfloat16: the upper half of an FP32, round to nearest even.
uint16_t f32_to_bf16(float x) {
  uint32_t u; std::memcpy(&u, &x, 4);
  if (std::isnan(x)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_to_f32(uint16_t b) {
  uint32_t u = (uint32_t)b << 16; float f; std::memcpy(&f, &u, 4); return f;
}

// OCP FP8 E4M3 ("fn"): 1 sign, 4 exponent (bias 7), 3 mantissa bits, no
// infinities, 0x7F/0xFF = NaN, largest finite 448.  Round to nearest even,
// saturating at +-448.
uint8_t f32_to_e4m3(float x) {
  uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
  if (std::isnan(x)) return (uint8_t)(sign | 0x7F);
  double a = std::fabs((double)x);
  if (a >= 448.0) return (uint8_t)(sign | 0x7E);
  if (a < std::ldexp(1.0, -6)) {                            // subnormal range
    double q = std::nearbyint(a * std::ldexp(1.0, 9));       // units of 2^-9
    return (uint8_t)(sign | (uint8_t)q);                     // q = 8 -> min normal
  }
  int e; std::frexp(a, &e); e -= 1;
  double m = std::nearbyint(a * std::ldexp(1.0, 3 - e));     // in [8, 16]
  if (m >= 16.0) { m = 8.0; e += 1; }
  int code = ((e + 7) << 3) | ((int)m - 8);
  if (code > 0x7E) code = 0x7E;
  return (uint8_t)(sign | code);
}

float e4m3_to_f32(uint8_t b) {
  int s = b >> 7, e = (b >> 3) & 15, m = b & 7;
  if (e == 15 && m == 7) return NAN;
  double v = (e == 0) ? std::ldexp((double)m, -9) : std::ldexp((double)(8 + m), e - 10);
  return (float)(s ? -v : v);
}

// ---------------------------------------------------------------------------
// Representations searched
// ---------------------------------------------------------------------------

enum { MODE_F32 = 0, MODE_F16 = 1, MODE_BF16 = 2, MODE_FP8 = 3, MODE_PQ = 4, MODE_SPARSE = 5 };
enum { MET_L2 = 0, MET_IP = 1 };
enum { KEY_CANON = 0, KEY_EXACT = 1 };

struct Store {
  int mode = MODE_F32, metric = MET_L2, d = 0;
  const float* f32 = nullptr;
  const uint16_t* f16 = nullptr;   // also bf16
  const uint8_t* fp8 = nullptr;
  const float* fp8_scale = nullptr;
  // PQ
  int pq_m = 0, pq_ksub = 0, pq_dsub = 0;
  const float* pq_cb = nullptr;    // [m][ksub][dsub]
  const uint8_t* pq_codes = nullptr;  // [n][m]
  // sparse CSR
  const int64_t* sp_ptr = nullptr;
  const uint16_t* sp_ids = nullptr;
  const float* sp_vals = nullptr;
};

int chunk_elems(int mode) {
  switch (mode) {
    case MODE_F32: return 4;
    case MODE_F16: case MODE_BF16: return 8;
    case MODE_FP8: return 16;
    default: return 1;
  }
}

// Element i of row r, exactly up-converted to FP32 (no scale applied).
inline float elem(const Store& s, int64_t r, int i) {
  size_t o = (size_t)r * s.d + i;
  switch (s.mode) {
    case MODE_F32: return s.f32[o];
    case MODE_F16: return f16_to_f32(s.f16[o]);
    case MODE_BF16: return bf16_to_f32(s.f16[o]);
    case MODE_FP8: return e4m3_to_f32(s.fp8[o]);
  }
  return 0.f;
}

void xor_tree(float* p) {
  for (int s = 32; s >= 1; s >>= 1) {
    float t[64];
    for (int l = 0; l < 64; ++l) t[l] = p[l] + p[l ^ s];
    std::memcpy(p, t, sizeof t);
  }
}

// CANON key of FP32 q against an FP32 row, d a multiple of 4: the same
// order as the generic loop below, written chunk by chunk so that the
// compiler can vectorise across the 64 independent partials.
float canon_f32(const float* q, const float* x, int d, int metric) {
  float p[64];
  for (int l = 0; l < 64; ++l) p[l] = 0.0f;
  const int nchunk = d / 4;
  for (int g0 = 0; g0 < nchunk; g0 += 64) {
    const int cnt = std::min(64, nchunk - g0);
    const float* qb = q + 4 * g0;
    const float* xb = x + 4 * g0;
    if (metric == MET_IP) {
      for (int l = 0; l < cnt; ++l) {
        float a = p[l];
        a = std::fmaf(qb[4 * l + 0], xb[4 * l + 0], a);
        a = std::fmaf(qb[4 * l + 1], xb[4 * l + 1], a);
        a = std::fmaf(qb[4 * l + 2], xb[4 * l + 2], a);
        a = std::fmaf(qb[4 * l + 3], xb[4 * l + 3], a);
        p[l] = a;
      }
    } else {
      for (int l = 0; l < cnt; ++l) {
        float a = p[l];
        float t0 = qb[4 * l + 0] - xb[4 * l + 0];
        float t1 = qb[4 * l + 1] - xb[4 * l + 1];
        float t2 = qb[4 * l + 2] - xb[4 * l + 2];
        float t3 = qb[4 * l + 3] - xb[4 * l + 3];
        a = std::fmaf(t0, t0, a);
        a = std::fmaf(t1, t1, a);
        a = std::fmaf(t2, t2, a);
        a = std::fmaf(t3, t3, a);
        p[l] = a;
      }
    }
  }
  xor_tree(p);
  return metric == MET_IP ? -p[0] : p[0];
}

// Dense key of FP32 query q against row r of a dense store.
float dense_key(const Store& s, const float* q, int64_t r, int kmode) {
  const int d = s.d;
  if (kmode == KEY_CANON && s.mode == MODE_F32 && d % 4 == 0)
    return canon_f32(q, s.f32 + (size_t)r * d, d, s.metric);
  const float scale = (s.mode == MODE_FP8) ? s.fp8_scale[r] : 1.0f;
  if (kmode == KEY_EXACT) {
    double acc = 0.0;
    for (int i = 0; i < d; ++i) {
      double x = (double)elem(s, r, i) * (double)scale;
      if (s.metric == MET_IP) acc += (double)q[i] * x;
      else { double t = (double)q[i] - x; acc += t * t; }
    }
    return (float)(s.metric == MET_IP ? -acc : acc);
  }
  float p[64];
  for (int l = 0; l < 64; ++l) p[l] = 0.0f;
  const int c = chunk_elems(s.mode);
  for (int i = 0; i < d; ++i) {
    const int l = (i / c) % 64;
    float x = elem(s, r, i);
    if (s.metric == MET_IP) {
      p[l] = std::fmaf(q[i], x, p[l]);
    } else {
      if (s.mode == MODE_FP8) x = scale * x;
      float t = q[i] - x;
      p[l] = std::fmaf(t, t, p[l]);
    }
  }
  xor_tree(p);
  float S = p[0];
  if (s.metric == MET_IP) {
    if (s.mode == MODE_FP8) S = scale * S;
    return -S;
  }
  return S;
}

// Sparse query (sorted ids) against doc r: -sum over shared term ids.
float sparse_key(const Store& s, const uint16_t* qid, const float* qv, int qn, int64_t r,
                 int kmode) {
  const int64_t b = s.sp_ptr[r], e = s.sp_ptr[r + 1];
  if (kmode == KEY_EXACT) {
    double acc = 0.0;
    int64_t j = b; int t = 0;
    while (j < e && t < qn) {
      if (s.sp_ids[j] < qid[t]) ++j;
      else if (s.sp_ids[j] > qid[t]) ++t;
      else { acc += (double)qv[t] * (double)s.sp_vals[j]; ++j; ++t; }
    }
    return (float)(-acc);
  }
  float p[64];
  for (int l = 0; l < 64; ++l) p[l] = 0.0f;
  for (int64_t j = b; j < e; ++j) {
    // query weight of this doc term, or 0 if the query lacks it
    const uint16_t* it = std::lower_bound(qid, qid + qn, s.sp_ids[j]);
    float w = (it != qid + qn && *it == s.sp_ids[j]) ? qv[it - qid] : 0.0f;
    const int l = (int)((j - b) % 64);
    p[l] = std::fmaf(w, s.sp_vals[j], p[l]);
  }
  xor_tree(p);
  return -p[0];
}

// Per-query PQ lookup table: lut[m][j] = partial key of subvector m of q
// against centroid j of subspace m (IP: positive dot product, negated at the
// end; L2: squared distance).  CANON: one sequential fmaf chain per entry,
// stored in FP32.  EXACT: FP64 sums kept in FP64 (lut64), so that the ADC key
// is rounded once.
template <class T>
void pq_lut(const Store& s, const float* q, T* lut, int kmode) {
  for (int m = 0; m < s.pq_m; ++m)
    for (int j = 0; j < s.pq_ksub; ++j) {
      const float* c = s.pq_cb + ((size_t)m * s.pq_ksub + j) * s.pq_dsub;
      const float* qs = q + (size_t)m * s.pq_dsub;
      if (kmode == KEY_EXACT) {
        double acc = 0.0;
        for (int t = 0; t < s.pq_dsub; ++t) {
          if (s.metric == MET_IP) acc += (double)qs[t] * (double)c[t];
          else { double u = (double)qs[t] - (double)c[t]; acc += u * u; }
        }
        lut[m * s.pq_ksub + j] = (T)acc;
      } else {
        float acc = 0.0f;
        for (int t = 0; t < s.pq_dsub; ++t) {
          if (s.metric == MET_IP) acc = std::fmaf(qs[t], c[t], acc);
          else { float u = qs[t] - c[t]; acc = std::fmaf(u, u, acc); }
        }
        lut[m * s.pq_ksub + j] = (T)acc;
      }
    }
}

// ADC key: sum over subspaces of the table entry selected by the code.
float adc_key_exact(const Store& s, const double* lut64, int64_t r) {
  const uint8_t* code = s.pq_codes + (size_t)r * s.pq_m;
  double acc = 0.0;
  for (int m = 0; m < s.pq_m; ++m) acc += lut64[m * s.pq_ksub + code[m]];
  return (float)(s.metric == MET_IP ? -acc : acc);
}

float adc_key_canon(const Store& s, const float* lut, int64_t r) {
  const uint8_t* code = s.pq_codes + (size_t)r * s.pq_m;
  float p[64];
  for (int l = 0; l < 64; ++l) p[l] = 0.0f;
  for (int m = 0; m < s.pq_m; ++m) p[m % 64] = p[m % 64] + lut[m * s.pq_ksub + code[m]];
  xor_tree(p);
  return s.metric == MET_IP ? -p[0] : p[0];
}

// A query bound to a store: key(id).
struct Evaluator {
  const Store* s; int kmode;
  const float* q = nullptr;                 // dense / PQ
  const uint16_t* qid = nullptr; const float* qv = nullptr; int qn = 0;  // sparse
  std::vector<float> lut;
  std::vector<double> lut64;
  int64_t evals = 0;
  Evaluator(const Store* st, int km) : s(st), kmode(km) {}
  void bind_dense(const float* query) {
    q = query;
    if (s->mode == MODE_PQ) {
      if (kmode == KEY_EXACT) {
        lut64.assign((size_t)s->pq_m * s->pq_ksub, 0.0);
        pq_lut(*s, q, lut64.data(), kmode);
      } else {
        lut.assign((size_t)s->pq_m * s->pq_ksub, 0.f);
        pq_lut(*s, q, lut.data(), kmode);
      }
    }
  }
  void bind_sparse(const uint16_t* ids, const float* vals, int n) { qid = ids; qv = vals; qn = n; }
  float key(int64_t r) {
    ++evals;
    if (s->mode == MODE_PQ)
      return kmode == KEY_EXACT ? adc_key_exact(*s, lut64.data(), r) : adc_key_canon(*s, lut.data(), r);
    if (s->mode == MODE_SPARSE) return sparse_key(*s, qid, qv, qn, r, kmode);
    return dense_key(*s, q, r, kmode);
  }
};

// ---------------------------------------------------------------------------
// Total order on (key, id)
// ---------------------------------------------------------------------------

struct KI { float k; int32_t id; };
inline bool lt(const KI& a, const KI& b) { return a.k < b.k || (a.k == b.k && a.id < b.id); }
struct MinFirst { bool operator()(const KI& a, const KI& b) const { return lt(b, a); } };
struct MaxFirst { bool operator()(const KI& a, const KI& b) const { return lt(a, b); } };

// ---------------------------------------------------------------------------
// Graph in the exchange layout
//   levels u8[n]; adj0 i32[n][M0] (-1 padded); upper_off i32[n] = index of the
//   node's level-1 list in upper_adj (lists for levels 1..level follow), or -1;
//   upper_adj i32[n_lists][M] (-1 padded).
// ---------------------------------------------------------------------------

struct GraphView {
  int64_t n; int M, M0, max_level; int32_t entry;
  const uint8_t* levels; const int32_t* adj0; const int32_t* upper_off; const int32_t* upper_adj;
  // neighbours of v at level lc: pointer + capacity
  const int32_t* nbrs(int64_t v, int lc, int* cap) const {
    if (lc == 0) { *cap = M0; return adj0 + (size_t)v * M0; }
    *cap = M;
    return upper_adj + ((size_t)upper_off[v] + (lc - 1)) * M;
  }
};

// Visited marks with epochs, one array per thread.
struct Visited {
  std::vector<uint32_t> mark; uint32_t epoch = 0;
  explicit Visited(int64_t n) : mark((size_t)n, 0u) {}
  void reset() { if (++epoch == 0) { std::fill(mark.begin(), mark.end(), 0u); epoch = 1; } }
  bool test_set(int64_t v) { if (mark[v] == epoch) return true; mark[v] = epoch; return false; }
};

// SEARCH-LAYER (HNSW Algorithm 2): a min-queue C of candidates, a bounded
// max-queue W of results, a visited set.  Returns W sorted by (key, id).
// `nb(v, &cnt)` yields the neighbour list of v at this layer.
template <class NbFn>
std::vector<KI> search_layer(Evaluator& ev, const std::vector<KI>& eps, int ef, NbFn nb,
                             Visited& vis, std::vector<int32_t>* visited_out,
                             int64_t* expansions) {
  vis.reset();
  std::priority_queue<KI, std::vector<KI>, MinFirst> C;
  std::priority_queue<KI, std::vector<KI>, MaxFirst> W;
  for (const KI& e : eps) {
    vis.test_set(e.id);
    if (visited_out) visited_out->push_back(e.id);
    C.push(e); W.push(e);
    if ((int)W.size() > ef) W.pop();
  }
  while (!C.empty()) {
    KI c = C.top(); C.pop();
    if (lt(W.top(), c)) break;              // c is worse than the furthest of W
    if (expansions) ++*expansions;
    int cnt; const int32_t* lst = nb(c.id, &cnt);
    for (int j = 0; j < cnt; ++j) {
      int32_t e = lst[j];
      if (e < 0) break;
      if (vis.test_set(e)) continue;
      if (visited_out) visited_out->push_back(e);
      KI ke{ev.key(e), e};
      if ((int)W.size() < ef || lt(ke, W.top())) {
        C.push(ke); W.push(ke);
        if ((int)W.size() > ef) W.pop();
      }
    }
  }
  std::vector<KI> out;
  out.reserve(W.size());
  while (!W.empty()) { out.push_back(W.top()); W.pop(); }
  std::reverse(out.begin(), out.end());
  return out;
}

// ---------------------------------------------------------------------------
// HNSW construction (Algorithms 1 and 4), optionally in batches
// ---------------------------------------------------------------------------

struct Builder {
  const float* X; int64_t n; int d; int metric; int M, M0, efc;
  Store st;
  std::vector<uint8_t> level;
  std::vector<std::vector<std::vector<int32_t>>> adj;   // adj[v][lc]
  int max_level = -1; int32_t entry = -1;

  // key between two base points: CANON FP32 for dense rows (symmetric); for
  // sparse rows the EXACT merge-join key (symmetric, and cheaper to build with)
  float key2(int64_t a, int64_t b) const {
    if (st.mode == MODE_SPARSE) {
      const int64_t o = st.sp_ptr[a];
      return sparse_key(st, st.sp_ids + o, st.sp_vals + o, (int)(st.sp_ptr[a + 1] - o), b, KEY_EXACT);
    }
    return dense_key(st, X + (size_t)a * d, b, KEY_CANON);
  }

  // Algorithm 4 without candidate extension and without keeping pruned
  // connections: walk candidates by increasing (key, id) to the base and keep
  // one iff it is strictly closer to the base than to every kept one.
  std::vector<int32_t> heuristic(const std::vector<KI>& cand_sorted, int cap) const {
    std::vector<int32_t> R;
    for (const KI& e : cand_sorted) {
      if ((int)R.size() >= cap) break;
      bool keep = true;
      for (int32_t r : R) {
        if (!(e.k < key2(e.id, r))) { keep = false; break; }
      }
      if (keep) R.push_back(e.id);
    }
    return R;
  }

  std::vector<KI> layer_search(Evaluator& ev, const std::vector<KI>& eps, int ef, int lc,
                               Visited& vis) {
    auto nb = [&](int32_t v, int* cnt) -> const int32_t* {
      const auto& L = adj[v][lc];
      *cnt = (int)L.size();
      return L.data();
    };
    return search_layer(ev, eps, ef, nb, vis, nullptr, nullptr);
  }

  // Phase 1 for node i against the current (frozen) graph: per-layer
  // neighbour choices, levels min(L, l_i) .. 0.
  std::vector<std::vector<int32_t>> choose(int64_t i, Visited& vis) {
    std::vector<std::vector<int32_t>> N((size_t)level[i] + 1);
    if (entry < 0) return N;
    Evaluator ev(&st, st.mode == MODE_SPARSE ? KEY_EXACT : KEY_CANON);
    if (st.mode == MODE_SPARSE) {
      const int64_t o = st.sp_ptr[i];
      ev.bind_sparse(st.sp_ids + o, st.sp_vals + o, (int)(st.sp_ptr[i + 1] - o));
    } else {
      ev.bind_dense(X + (size_t)i * d);
    }
    std::vector<KI> W{KI{ev.key(entry), entry}};
    const int L = max_level, li = level[i];
    for (int lc = L; lc > li; --lc) W = std::vector<KI>{layer_search(ev, W, 1, lc, vis)[0]};
    for (int lc = std::min(L, li); lc >= 0; --lc) {
      W = layer_search(ev, W, efc, lc, vis);
      N[lc] = heuristic(W, M);
    }
    return N;
  }

  void prune(int64_t e, int lc) {
    const int cap = lc == 0 ? M0 : M;
    auto& L = adj[e][lc];
    if ((int)L.size() <= cap) return;
    std::vector<KI> c;
    c.reserve(L.size());
    for (int32_t v : L) c.push_back(KI{key2(e, v), v});
    std::sort(c.begin(), c.end(), lt);
    L = heuristic(c, cap);
  }

  void build(const double* u, int64_t seq_prefix, double batch_frac, int64_t batch_cap,
             int threads) {
    const double mL = 1.0 / std::log((double)M);
    level.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      double l = std::floor(-std::log(1.0 - u[i]) * mL);
      level[i] = (uint8_t)std::min(l, 30.0);
    }
    adj.resize(n);
    std::vector<Visited> vis;
    for (int t = 0; t < threads; ++t) vis.emplace_back(n);
    int64_t done = 0;
    while (done < n) {
      int64_t b = 1;
      if (done >= seq_prefix && batch_frac > 0)
        b = std::max<int64_t>(1, std::min<int64_t>(batch_cap, (int64_t)(done * batch_frac)));
      b = std::min(b, n - done);
      std::vector<std::vector<std::vector<int32_t>>> N(b);
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) if (b > 1)
      for (int64_t t = 0; t < b; ++t) N[t] = choose(done + t, vis[omp_get_thread_num()]);
      // Phase 2: own lists, then reverse links grouped by target.
      std::vector<std::pair<int64_t, int32_t>> rev;   // (target*32+lc, source)
      for (int64_t t = 0; t < b; ++t) {
        const int64_t i = done + t;
        adj[i].assign((size_t)level[i] + 1, {});
        for (int lc = 0; lc < (int)N[t].size(); ++lc) {
          adj[i][lc] = N[t][lc];
          for (int32_t e : N[t][lc]) rev.emplace_back((int64_t)e * 32 + lc, (int32_t)i);
        }
      }
      std::stable_sort(rev.begin(), rev.end(),
                       [](const auto& a, const auto& c) { return a.first < c.first; });
      std::vector<size_t> starts;
      for (size_t j = 0; j < rev.size(); ++j)
        if (j == 0 || rev[j].first != rev[j - 1].first) starts.push_back(j);
      starts.push_back(rev.size());
      const int64_t ngroups = (int64_t)starts.size() - 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads) if (b > 1)
      for (int64_t g = 0; g < ngroups; ++g) {
        const int64_t e = rev[starts[g]].first / 32;
        const int lc = (int)(rev[starts[g]].first % 32);
        for (size_t j = starts[g]; j < starts[g + 1]; ++j) {
          adj[e][lc].push_back(rev[j].second);
          prune(e, lc);
        }
      }
      for (int64_t t = 0; t < b; ++t) {
        const int64_t i = done + t;
        if ((int)level[i] > max_level) { max_level = level[i]; entry = (int32_t)i; }
      }
      const int64_t step = std::max<int64_t>(1, n / 20);
      if (n >= 100000 && (done + b) / step != done / step)
        std::fprintf(stderr, "[oracle build] %lld / %lld nodes\n", (long long)(done + b), (long long)n);
      done += b;
    }
  }
};

// ---------------------------------------------------------------------------
// k-means for PQ (Lloyd, EXACT distances, deterministic tie and empty rules)
// ---------------------------------------------------------------------------

double sqd(const float* a, const float* b, int ds) {
  double acc = 0.0;
  for (int t = 0; t < ds; ++t) { double u = (double)a[t] - (double)b[t]; acc += u * u; }
  return acc;
}

int argmin_centroid(const float* x, const float* cb, int ksub, int ds, double* best_out) {
  int best = 0; double bd = sqd(x, cb, ds);
  for (int j = 1; j < ksub; ++j) {
    double dd = sqd(x, cb + (size_t)j * ds, ds);
    if (dd < bd) { bd = dd; best = j; }
  }
  if (best_out) *best_out = bd;
  return best;
}

}  // namespace

// ===========================================================================
// C interface (ctypes)
// ===========================================================================

extern "C" {

int or_version() { return 4; }

void or_to_f16(const float* x, int64_t n, uint16_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = f32_to_f16(x[i]);
}
void or_from_f16(const uint16_t* h, int64_t n, float* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = f16_to_f32(h[i]);
}
void or_to_bf16(const float* x, int64_t n, uint16_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = f32_to_bf16(x[i]);
}
void or_from_bf16(const uint16_t* h, int64_t n, float* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = bf16_to_f32(h[i]);
}
void or_to_e4m3(const float* x, int64_t n, uint8_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = f32_to_e4m3(x[i]);
}
void or_from_e4m3(const uint8_t* b, int64_t n, float* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = e4m3_to_f32(b[i]);
}

// Per-vector scaled E4M3 copy: s = max|x_i| / 448 (1 for a zero row),
// code_i = E4M3(x_i / s).
void or_encode_fp8_rows(const float* X, int64_t n, int d, uint8_t* codes, float* scale,
                        int threads) {
#pragma omp parallel for schedule(static) num_threads(threads)
  for (int64_t r = 0; r < n; ++r) {
    const float* x = X + (size_t)r * d;
    float mx = 0.0f;
    for (int i = 0; i < d; ++i) mx = std::max(mx, std::fabs(x[i]));
    float s = mx > 0.0f ? mx / 448.0f : 1.0f;
    scale[r] = s;
    for (int i = 0; i < d; ++i) codes[(size_t)r * d + i] = f32_to_e4m3(x[i] / s);
  }
}

// Store descriptor shared by the key and search entry points.
struct or_store {
  int32_t mode, metric, d, pad;
  const float* f32; const uint16_t* f16; const uint8_t* fp8; const float* fp8_scale;
  int32_t pq_m, pq_ksub, pq_dsub, pad2;
  const float* pq_cb; const uint8_t* pq_codes;
  const int64_t* sp_ptr; const uint16_t* sp_ids; const float* sp_vals;
};

static Store to_store(const or_store* s) {
  Store t;
  t.mode = s->mode; t.metric = s->metric; t.d = s->d;
  t.f32 = s->f32; t.f16 = s->f16; t.fp8 = s->fp8; t.fp8_scale = s->fp8_scale;
  t.pq_m = s->pq_m; t.pq_ksub = s->pq_ksub; t.pq_dsub = s->pq_dsub;
  t.pq_cb = s->pq_cb; t.pq_codes = s->pq_codes;
  t.sp_ptr = s->sp_ptr; t.sp_ids = s->sp_ids; t.sp_vals = s->sp_vals;
  return t;
}

// keys[i][j] = key(query i, row rows[i][j]) for dense/PQ stores.
void or_keys_dense(const or_store* s, const float* Q, int64_t nq, const int64_t* rows,
                   int64_t per_q, int kmode, float* out, int threads) {
  Store st = to_store(s);
  const int qd = (st.mode == MODE_PQ) ? st.pq_m * st.pq_dsub : st.d;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
  for (int64_t i = 0; i < nq; ++i) {
    Evaluator ev(&st, kmode);
    ev.bind_dense(Q + (size_t)i * qd);
    for (int64_t j = 0; j < per_q; ++j) out[i * per_q + j] = ev.key(rows[i * per_q + j]);
  }
}

void or_keys_sparse(const or_store* s, const int64_t* qptr, const uint16_t* qids,
                    const float* qvals, int64_t nq, const int64_t* rows, int64_t per_q,
                    int kmode, float* out, int threads) {
  Store st = to_store(s);
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
  for (int64_t i = 0; i < nq; ++i) {
    Evaluator ev(&st, kmode);
    ev.bind_sparse(qids + qptr[i], qvals + qptr[i], (int)(qptr[i + 1] - qptr[i]));
    for (int64_t j = 0; j < per_q; ++j) out[i * per_q + j] = ev.key(rows[i * per_q + j]);
  }
}

// PQ lookup tables for nq queries: out[nq][m][ksub].
void or_pq_luts(const or_store* s, const float* Q, int64_t nq, int kmode, float* out) {
  Store st = to_store(s);
  const int qd = st.pq_m * st.pq_dsub;
  for (int64_t i = 0; i < nq; ++i)
    pq_lut(st, Q + (size_t)i * qd, out + (size_t)i * st.pq_m * st.pq_ksub, kmode);
}

// Exact k-NN by scanning every row: keys in `kmode`, order (key, id).
void or_bruteforce(const or_store* s, const float* Q, const int64_t* qptr,
                   const uint16_t* qids, const float* qvals, int64_t nq, int64_t n, int k,
                   int kmode, int64_t* out_ids, float* out_keys, int threads) {
  Store st = to_store(s);
  const int qd = (st.mode == MODE_PQ) ? st.pq_m * st.pq_dsub : st.d;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
  for (int64_t i = 0; i < nq; ++i) {
    Evaluator ev(&st, kmode);
    if (st.mode == MODE_SPARSE)
      ev.bind_sparse(qids + qptr[i], qvals + qptr[i], (int)(qptr[i + 1] - qptr[i]));
    else
      ev.bind_dense(Q + (size_t)i * qd);
    std::vector<KI> all((size_t)n);
    for (int64_t r = 0; r < n; ++r) all[r] = KI{ev.key(r), (int32_t)r};
    const int kk = (int)std::min<int64_t>(k, n);
    std::partial_sort(all.begin(), all.begin() + kk, all.end(), lt);
    for (int j = 0; j < k; ++j) {
      out_ids[i * k + j] = j < kk ? all[j].id : -1;
      out_keys[i * k + j] = j < kk ? all[j].k : INFINITY;
    }
  }
}

// --- HNSW build --------------------------------------------------------------

struct or_graph {
  int64_t n; int32_t M, M0, max_level, entry;
  std::vector<uint8_t> levels;
  std::vector<int32_t> adj0, upper_off, upper_adj;
};

// Builds the graph on the FP32 originals X (n x d).  u[i] in [0,1) gives the
// level floor(-ln(1 - u_i) / ln M).  Nodes are inserted in id order; when
// batch_frac > 0 and at least seq_prefix nodes are in, nodes are inserted in
// batches of max(1, min(batch_cap, done * batch_frac)) whose neighbour
// searches all see the graph as it was before the batch.  A batch of one is
// exactly sequential insertion.
static void* export_graph(Builder& B);

void* or_hnsw_build(const float* X, int64_t n, int d, int metric, int M, int efc,
                    const double* u, int64_t seq_prefix, double batch_frac,
                    int64_t batch_cap, int threads) {
  Builder B;
  B.X = X; B.n = n; B.d = d; B.metric = metric; B.M = M; B.M0 = 2 * M; B.efc = efc;
  B.st.mode = MODE_F32; B.st.metric = metric; B.st.d = d; B.st.f32 = X;
  B.build(u, seq_prefix, batch_frac, batch_cap, std::max(1, threads));
  return export_graph(B);
}

// The same construction over sparse rows (inner product), with EXACT
// merge-join keys.
void* or_hnsw_build_sparse(const int64_t* indptr, const uint16_t* ids, const float* vals,
                           int64_t n, int vocab, int M, int efc, const double* u,
                           int64_t seq_prefix, double batch_frac, int64_t batch_cap,
                           int threads) {
  Builder B;
  B.X = nullptr; B.n = n; B.d = vocab; B.metric = MET_IP; B.M = M; B.M0 = 2 * M; B.efc = efc;
  B.st.mode = MODE_SPARSE; B.st.metric = MET_IP; B.st.d = vocab;
  B.st.sp_ptr = indptr; B.st.sp_ids = ids; B.st.sp_vals = vals;
  B.build(u, seq_prefix, batch_frac, batch_cap, std::max(1, threads));
  return export_graph(B);
}

static void* export_graph(Builder& B) {
  const int64_t n = B.n;
  const int M = B.M;
  auto* g = new or_graph;
  g->n = n; g->M = M; g->M0 = 2 * M; g->max_level = B.max_level; g->entry = B.entry;
  g->levels = B.level;
  g->adj0.assign((size_t)n * g->M0, -1);
  g->upper_off.assign((size_t)n, -1);
  int64_t lists = 0;
  for (int64_t v = 0; v < n; ++v) {
    const auto& a0 = B.adj[v][0];
    for (size_t j = 0; j < a0.size(); ++j) g->adj0[(size_t)v * g->M0 + j] = a0[j];
    if (B.level[v] > 0) { g->upper_off[v] = (int32_t)lists; lists += B.level[v]; }
  }
  g->upper_adj.assign((size_t)lists * M, -1);
  for (int64_t v = 0; v < n; ++v)
    for (int lc = 1; lc <= B.level[v]; ++lc) {
      const auto& a = B.adj[v][lc];
      for (size_t j = 0; j < a.size(); ++j)
        g->upper_adj[((size_t)g->upper_off[v] + lc - 1) * M + j] = a[j];
    }
  return g;
}

void or_graph_info(const void* gp, int64_t* info) {
  const or_graph* g = (const or_graph*)gp;
  info[0] = g->n; info[1] = g->M; info[2] = g->M0; info[3] = g->max_level; info[4] = g->entry;
  info[5] = (int64_t)(g->upper_adj.size() / std::max(1, g->M));
}

void or_graph_export(const void* gp, uint8_t* levels, int32_t* adj0, int32_t* upper_off,
                     int32_t* upper_adj) {
  const or_graph* g = (const or_graph*)gp;
  std::memcpy(levels, g->levels.data(), g->levels.size());
  std::memcpy(adj0, g->adj0.data(), g->adj0.size() * 4);
  std::memcpy(upper_off, g->upper_off.data(), g->upper_off.size() * 4);
  std::memcpy(upper_adj, g->upper_adj.data(), g->upper_adj.size() * 4);
}

void or_graph_free(void* gp) { delete (or_graph*)gp; }

// --- HNSW search (Algorithms 5 and 2), instrumented --------------------------

struct or_graph_in {
  int64_t n; int32_t M, M0, max_level, entry;
  const uint8_t* levels; const int32_t* adj0; const int32_t* upper_off;
  const int32_t* upper_adj;
};

// stats per query: [0] distance evaluations (all layers), [1] layer-0
// evaluations, [2] layer-0 expansions, [3] |layer-0 visited set|, [4] |W|.
void or_hnsw_search(const or_graph_in* gi, const or_store* s, const float* Q,
                    const int64_t* qptr, const uint16_t* qids, const float* qvals,
                    int64_t nq, const int32_t* k_arr, const int32_t* ef_arr, int k_max,
                    int kmode, const float* rerank_f32, int rerank_depth, int rerank_kmode,
                    int64_t* out_ids, float* out_keys, int64_t* stats,
                    int32_t* w_ids, float* w_keys, int w_cap,
                    int32_t* visited, int64_t visited_cap, int threads) {
  Store st = to_store(s);
  GraphView G{gi->n, gi->M, gi->M0, gi->max_level, gi->entry, gi->levels, gi->adj0,
              gi->upper_off, gi->upper_adj};
  const int qd = (st.mode == MODE_PQ) ? st.pq_m * st.pq_dsub : st.d;
  std::vector<Visited> vis;
  for (int t = 0; t < std::max(1, threads); ++t) vis.emplace_back(G.n);
#pragma omp parallel for schedule(dynamic, 1) num_threads(std::max(1, threads))
  for (int64_t i = 0; i < nq; ++i) {
    Visited& V = vis[omp_get_thread_num()];
    const int k = k_arr[i];
    const int ef = std::max(ef_arr[i], k);
    Evaluator ev(&st, kmode);
    if (st.mode == MODE_SPARSE)
      ev.bind_sparse(qids + qptr[i], qvals + qptr[i], (int)(qptr[i + 1] - qptr[i]));
    else
      ev.bind_dense(Q + (size_t)i * qd);
    std::vector<KI> W;
    int64_t ev0 = 0, exp0 = 0;
    std::vector<int32_t> vset;
    if (G.n > 0 && G.entry >= 0) {
      W.push_back(KI{ev.key(G.entry), G.entry});
      for (int lc = G.max_level; lc >= 1; --lc) {
        auto nb = [&](int32_t v, int* cnt) { return G.nbrs(v, lc, cnt); };
        W = std::vector<KI>{search_layer(ev, W, 1, nb, V, nullptr, nullptr)[0]};
      }
      const int64_t before = ev.evals;
      auto nb0 = [&](int32_t v, int* cnt) { return G.nbrs(v, 0, cnt); };
      W = search_layer(ev, W, ef, nb0, V, &vset, &exp0);
      ev0 = ev.evals - before;
    }
    std::vector<KI> res = W;
    if (rerank_f32 && rerank_depth > 0) {
      Store orig; orig.mode = MODE_F32; orig.metric = st.metric; orig.d = st.d;
      orig.f32 = rerank_f32;
      const int R = std::min<int>((int)W.size(), std::max(rerank_depth, k));
      res.resize(R);
      for (int j = 0; j < R; ++j) res[j].k = dense_key(orig, Q + (size_t)i * qd, W[j].id, rerank_kmode);
      std::sort(res.begin(), res.end(), lt);
    }
    for (int j = 0; j < k_max; ++j) {
      const bool ok = j < k && j < (int)res.size();
      out_ids[i * k_max + j] = ok ? res[j].id : -1;
      out_keys[i * k_max + j] = ok ? res[j].k : INFINITY;
    }
    if (stats) {
      stats[i * 5 + 0] = ev.evals; stats[i * 5 + 1] = ev0; stats[i * 5 + 2] = exp0;
      stats[i * 5 + 3] = (int64_t)vset.size(); stats[i * 5 + 4] = (int64_t)W.size();
    }
    if (w_ids)
      for (int j = 0; j < w_cap; ++j) {
        w_ids[i * w_cap + j] = j < (int)W.size() ? W[j].id : -1;
        w_keys[i * w_cap + j] = j < (int)W.size() ? W[j].k : INFINITY;
      }
    if (visited) {
      std::sort(vset.begin(), vset.end());
      for (int64_t j = 0; j < visited_cap; ++j)
        visited[i * visited_cap + j] = j < (int64_t)vset.size() ? vset[j] : -1;
    }
  }
}

// --- k-means (PQ per subspace, IVF coarse quantizer) -------------------------

}  // extern "C"

namespace {

// Lloyd's k-means on ns points of ds dimensions (pts row-major).  Centroid j
// starts at point init[j].  Each iteration assigns every point to its EXACT
// nearest centroid (lower index on ties), stops when no assignment changed,
// else replaces each centroid by the FP64 mean of its points (summed in
// ascending point order, rounded once to FP32).  An empty cluster takes the
// point of largest current error (lower position on ties) not already used
// for re-seeding in this step, clusters in ascending order.  Runs at most
// max_iter iterations; returns the number run.  obj[it] += the summed error
// of iteration it's assignment.  `threads` splits the assignment over points
// (it changes nothing but the rounding of obj).
int lloyd(const float* pts, int64_t ns, int ds, const int64_t* init, int ksub, int max_iter,
          float* C, double* obj, int threads) {
  for (int j = 0; j < ksub; ++j)
    for (int t = 0; t < ds; ++t) C[(size_t)j * ds + t] = pts[(size_t)init[j] * ds + t];
  std::vector<int> asg((size_t)ns, -1);
  std::vector<double> err((size_t)ns);
  int it = 0;
  for (; it < max_iter; ++it) {
    int changed = 0;
    double total = 0.0;
#pragma omp parallel for schedule(static) num_threads(threads) if (threads > 1) reduction(| : changed) reduction(+ : total)
    for (int64_t a = 0; a < ns; ++a) {
      double e;
      int j = argmin_centroid(&pts[(size_t)a * ds], C, ksub, ds, &e);
      if (j != asg[a]) { changed = 1; asg[a] = j; }
      err[a] = e; total += e;
    }
    obj[it] += total;
    if (!changed) break;
    std::vector<double> sum((size_t)ksub * ds, 0.0);
    std::vector<int64_t> cnt((size_t)ksub, 0);
    for (int64_t a = 0; a < ns; ++a) {
      ++cnt[asg[a]];
      for (int t = 0; t < ds; ++t) sum[(size_t)asg[a] * ds + t] += (double)pts[(size_t)a * ds + t];
    }
    std::vector<int64_t> order;   // point positions by decreasing error
    size_t next = 0;
    for (int j = 0; j < ksub; ++j) {
      if (cnt[j] > 0) {
        for (int t = 0; t < ds; ++t) C[(size_t)j * ds + t] = (float)(sum[(size_t)j * ds + t] / (double)cnt[j]);
      } else {
        if (order.empty()) {
          order.resize((size_t)ns);
          for (int64_t a = 0; a < ns; ++a) order[a] = a;
          std::stable_sort(order.begin(), order.end(),
                           [&](int64_t x, int64_t y) { return err[x] > err[y]; });
        }
        const int64_t pick = order[std::min(next++, order.size() - 1)];
        for (int t = 0; t < ds; ++t) C[(size_t)j * ds + t] = pts[(size_t)pick * ds + t];
      }
    }
  }
  return it + (it < max_iter ? 1 : 0);
}

}  // namespace

extern "C" {

// --- PQ training and encoding ------------------------------------------------

// k-means (lloyd above) per subspace on the sample rows (ids into X); init[j]
// indexes the sample.  Returns the largest iteration count of a subspace;
// objective[it] receives the summed error of the assignment made in
// iteration it (max_iter entries, may be NULL).
int or_pq_train(const float* X, int d, const int64_t* sample, int64_t ns, const int64_t* init,
                int m, int ksub, int max_iter, float* cb, double* objective, int threads) {
  const int ds = d / m;
  int iters_run = 0;
  std::vector<double> obj_sum((size_t)max_iter, 0.0);
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(max: iters_run)
  for (int sub = 0; sub < m; ++sub) {
    std::vector<float> pts((size_t)ns * ds);
    for (int64_t a = 0; a < ns; ++a)
      for (int t = 0; t < ds; ++t) pts[(size_t)a * ds + t] = X[(size_t)sample[a] * d + sub * ds + t];
    std::vector<double> obj((size_t)max_iter, 0.0);
    const int it = lloyd(pts.data(), ns, ds, init, ksub, max_iter, cb + (size_t)sub * ksub * ds,
                         obj.data(), 1);
#pragma omp critical
    for (int t = 0; t < max_iter; ++t) obj_sum[t] += obj[t];
    iters_run = std::max(iters_run, it);
  }
  if (objective)
    for (int it = 0; it < max_iter; ++it) objective[it] = obj_sum[it];
  return iters_run;
}

// codes[r][sub] = EXACT nearest centroid (lower index on ties).
void or_pq_encode(const float* X, int64_t n, int d, const float* cb, int m, int ksub,
                  uint8_t* codes, int threads) {
  const int ds = d / m;
#pragma omp parallel for schedule(static) num_threads(threads)
  for (int64_t r = 0; r < n; ++r)
    for (int sub = 0; sub < m; ++sub)
      codes[(size_t)r * m + sub] = (uint8_t)argmin_centroid(
          X + (size_t)r * d + sub * ds, cb + (size_t)sub * ksub * ds, ksub, ds, nullptr);
}


// --- IVF: inverted lists over a coarse quantizer ------------------------------
//
// The paper names IVF (Section 1) as one of the index families an ANN library
// offers, and plans more index types (Section 4, Conclusions and Future Work).  The coarse quantizer is
// k-means over the whole vector (lloyd above on a sample, L2), every row
// belongs to the list of its EXACT nearest centroid, and a query scans the
// lists of its nprobe nearest centroids.

// Coarse centroids: lloyd on the sample rows of X; init[j] indexes the sample.
int or_ivf_train(const float* X, int d, const int64_t* sample, int64_t ns, const int64_t* init,
                 int nlist, int max_iter, float* cent, double* objective, int threads) {
  std::vector<float> pts((size_t)ns * d);
  for (int64_t a = 0; a < ns; ++a)
    std::memcpy(&pts[(size_t)a * d], X + (size_t)sample[a] * d, sizeof(float) * d);
  std::vector<double> obj((size_t)max_iter, 0.0);
  const int it = lloyd(pts.data(), ns, d, init, nlist, max_iter, cent, obj.data(), threads);
  if (objective)
    for (int t = 0; t < max_iter; ++t) objective[t] = obj[t];
  return it;
}

// list[r] = EXACT nearest centroid of row r (lower index on ties).
void or_ivf_assign(const float* X, int64_t n, int d, const float* cent, int nlist, int32_t* list,
                   int threads) {
#pragma omp parallel for schedule(static) num_threads(threads)
  for (int64_t r = 0; r < n; ++r) list[r] = argmin_centroid(X + (size_t)r * d, cent, nlist, d, nullptr);
}

// IVF search.  For query i:
//  * probe keys: squared L2 from the FP32 query to every FP32 centroid, in
//    `kmode` (CANON: the FP32 fixed order of a dense FP32 row);
//  * probes: the min(nprobe, nlist) smallest (key, list id);
//  * candidates: every row of the probed lists, keyed in `kmode` on the
//    store's representation with the index metric, sorted by (key, id);
//  * with rerank_depth R > 0 the first min(max(R, k), #candidates) are
//    re-keyed on the FP32 rows (rerank_kmode) and re-sorted;
//  * out_ids/out_keys [nq][k]: the first k, -1 / +inf padded.
// out_probes [nq][nprobe] (-1 padded), stats [nq][2] = distance evaluations
// (candidates) and lists probed, w_ids/w_keys [nq][w_cap] the first w_cap
// sorted candidates before the rerank; each may be NULL.
void or_ivf_search(const or_store* s, const float* Q, int64_t nq, const float* cent, int nlist,
                   const int64_t* list_off, const int32_t* list_ids, int nprobe, int k, int kmode,
                   const float* rerank_f32, int rerank_depth, int rerank_kmode, int64_t* out_ids,
                   float* out_keys, int32_t* out_probes, int64_t* stats, int32_t* w_ids,
                   float* w_keys, int w_cap, int threads) {
  Store st = to_store(s);
  Store cs; cs.mode = MODE_F32; cs.metric = MET_L2; cs.d = st.d; cs.f32 = cent;
  const int np = std::min(nprobe, nlist);
#pragma omp parallel for schedule(dynamic, 1) num_threads(std::max(1, threads))
  for (int64_t i = 0; i < nq; ++i) {
    const float* q = Q + (size_t)i * st.d;
    std::vector<KI> pk((size_t)nlist);
    for (int j = 0; j < nlist; ++j) pk[j] = KI{dense_key(cs, q, j, kmode), j};
    std::sort(pk.begin(), pk.end(), lt);
    Evaluator ev(&st, kmode);
    ev.bind_dense(q);
    std::vector<KI> cand;
    for (int p = 0; p < np; ++p) {
      const int l = pk[p].id;
      for (int64_t t = list_off[l]; t < list_off[l + 1]; ++t)
        cand.push_back(KI{ev.key(list_ids[t]), list_ids[t]});
    }
    std::sort(cand.begin(), cand.end(), lt);
    std::vector<KI> res = cand;
    if (rerank_f32 && rerank_depth > 0) {
      Store orig; orig.mode = MODE_F32; orig.metric = st.metric; orig.d = st.d; orig.f32 = rerank_f32;
      const int R = (int)std::min<int64_t>((int64_t)cand.size(), std::max(rerank_depth, k));
      res.resize(R);
      for (int j = 0; j < R; ++j) res[j].k = dense_key(orig, q, cand[j].id, rerank_kmode);
      std::sort(res.begin(), res.end(), lt);
    }
    for (int j = 0; j < k; ++j) {
      const bool ok = j < (int)res.size();
      out_ids[i * k + j] = ok ? res[j].id : -1;
      out_keys[i * k + j] = ok ? res[j].k : INFINITY;
    }
    if (out_probes)
      for (int p = 0; p < nprobe; ++p) out_probes[i * nprobe + p] = p < np ? pk[p].id : -1;
    if (stats) { stats[i * 2 + 0] = (int64_t)cand.size(); stats[i * 2 + 1] = np; }
    if (w_ids)
      for (int j = 0; j < w_cap; ++j) {
        w_ids[i * w_cap + j] = j < (int)cand.size() ? cand[j].id : -1;
        w_keys[i * w_cap + j] = j < (int)cand.size() ? cand[j].k : INFINITY;
      }
  }
}

}  // extern "C"
