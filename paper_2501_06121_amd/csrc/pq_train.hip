// Product Quantization on the device: training (k-means per subspace) and
// encoding, the two halves of the paper's quantizer (Section 2, Product
// Quantization, and its citation, Jegou et al.).
//
// Every distance is the squared L2 distance of a subspace slice to a
// centroid, summed in FP64 from the FP32 inputs in ascending dimension order
// (one multiply and one add per dimension, no fusion), and the nearest
// centroid is the first minimum (lower index on ties).  Training is Lloyd's
// iteration: assign every sample point, stop a subspace when no assignment
// changed, else replace each centroid by the FP64 mean of its points (summed
// in ascending sample order, rounded once to FP32); an empty cluster takes
// the sample point of largest current error (lower sample position on ties,
// each point used once per step), clusters in ascending order.  The results
// are therefore fixed bit for bit by the inputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "ann.h"
#include "internal.h"

namespace ann {
namespace {

constexpr int kMaxSub = 32;       // dimensions per subspace held in registers
constexpr int kMaxKsub = 256;     // centroids per subspace (8-bit codes)

// Nearest centroid of point slices.  Grid: (points / 256, m); the block's 256
// threads take one point each for subspace blockIdx.y; the subspace's
// centroids sit in LDS.  Point a is row rows[a] of X (or row a when rows is
// NULL).  Writes codes8[row * m + sub] (encoding) or asg[sub * np + a] and
// err[sub * np + a] (training, where changed[sub] is set when an assignment
// differs from the previous one).
__global__ void __launch_bounds__(256) pq_assign(const float* X, int d, const int64_t* rows,
                                                 int64_t np, const float* cb, int m, int ksub,
                                                 uint8_t* codes8, int32_t* asg, double* err,
                                                 int32_t* changed, const int32_t* active) {
  __shared__ float C[kMaxKsub * kMaxSub];
  const int sub = blockIdx.y;
  if (active && !active[sub]) return;
  const int ds = d / m;
  const float* cs = cb + (size_t)sub * ksub * ds;
  for (int i = threadIdx.x; i < ksub * ds; i += blockDim.x) C[i] = cs[i];
  __syncthreads();
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= np) return;
  const int64_t r = rows ? rows[a] : a;
  double x[kMaxSub];
#pragma unroll
  for (int t = 0; t < kMaxSub; ++t) x[t] = t < ds ? (double)X[(size_t)r * d + (size_t)sub * ds + t] : 0.0;
  int best = 0;
  double bd = 0.0;
  for (int j = 0; j < ksub; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < kMaxSub; ++t) {
      if (t < ds) {
        const double u = x[t] - (double)C[j * ds + t];
        acc = acc + u * u;
      }
    }
    if (j == 0 || acc < bd) { bd = acc; best = j; }
  }
  if (codes8) codes8[(size_t)r * m + sub] = (uint8_t)best;
  if (asg) {
    const size_t o = (size_t)sub * np + a;
    if (asg[o] != best) { asg[o] = best; changed[sub] = 1; }
    err[o] = bd;
  }
}

// Centroid j of subspace sub (one thread each): the FP64 sum of its points in
// ascending sample order, divided by their count, rounded to FP32.  The
// block (all centroids of one subspace when ksub <= 256) stages the
// assignments through LDS in chunks; each thread walks them in order.  Empty
// clusters are flagged in empty[sub * ksub + j] and left as they are.
__global__ void __launch_bounds__(256) pq_update(const float* X, int d, const int64_t* sample,
                                                 int64_t ns, int m, int ksub, const int32_t* asg,
                                                 float* cb, int32_t* empty, const int32_t* active) {
  constexpr int kChunk = 4096;
  __shared__ int32_t A[kChunk];
  const int sub = blockIdx.y;
  if (!active[sub]) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int ds = d / m;
  double sum[kMaxSub];
#pragma unroll
  for (int t = 0; t < kMaxSub; ++t) sum[t] = 0.0;
  int64_t cnt = 0;
  const int32_t* as = asg + (size_t)sub * ns;
  for (int64_t a0 = 0; a0 < ns; a0 += kChunk) {
    const int len = ns - a0 < kChunk ? (int)(ns - a0) : kChunk;
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += blockDim.x) A[i] = as[a0 + i];
    __syncthreads();
    if (j < ksub) {
      for (int i = 0; i < len; ++i) {
        if (A[i] != j) continue;
        ++cnt;
        const float* xs = X + (size_t)sample[a0 + i] * d + (size_t)sub * ds;
#pragma unroll
        for (int t = 0; t < kMaxSub; ++t)
          if (t < ds) sum[t] = sum[t] + (double)xs[t];
      }
    }
  }
  if (j >= ksub) return;
  float* c = cb + ((size_t)sub * ksub + j) * ds;
  if (cnt > 0) {
#pragma unroll
    for (int t = 0; t < kMaxSub; ++t)
      if (t < ds) c[t] = (float)(sum[t] / (double)cnt);
  }
  empty[(size_t)sub * ksub + j] = cnt == 0 ? 1 : 0;
}

// Empty clusters of subspace blockIdx.x, in ascending order, each take the
// sample point of largest error not taken before (lower position on ties):
// one block-wide argmax per empty cluster; a taken point's error becomes -1.
__global__ void __launch_bounds__(256) pq_reseed(const float* X, int d, const int64_t* sample,
                                                 int64_t ns, int m, int ksub, double* err,
                                                 const int32_t* empty, float* cb,
                                                 const int32_t* active) {
  __shared__ double bk[256];
  __shared__ int64_t bi[256];
  const int sub = blockIdx.x;
  if (!active[sub]) return;
  const int ds = d / m;
  double* es = err + (size_t)sub * ns;
  for (int j = 0; j < ksub; ++j) {
    if (!empty[(size_t)sub * ksub + j]) continue;
    double mk = -2.0;
    int64_t mi = INT64_MAX;
    for (int64_t a = threadIdx.x; a < ns; a += blockDim.x) {
      const double e = es[a];
      if (e > mk) { mk = e; mi = a; }        // ascending a: the first maximum stays
    }
    bk[threadIdx.x] = mk;
    bi[threadIdx.x] = mi;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
      if ((int)threadIdx.x < s) {
        const double ok = bk[threadIdx.x + s];
        const int64_t oi = bi[threadIdx.x + s];
        if (ok > bk[threadIdx.x] || (ok == bk[threadIdx.x] && oi < bi[threadIdx.x])) {
          bk[threadIdx.x] = ok;
          bi[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    const int64_t pick = bi[0];
    if ((int)threadIdx.x < ds) {
      cb[((size_t)sub * ksub + j) * ds + threadIdx.x] = X[(size_t)sample[pick] * d + (size_t)sub * ds + threadIdx.x];
    }
    if (threadIdx.x == 0) es[pick] = -1.0;
    __syncthreads();
  }
}

// Centroid j of every subspace starts at sample point init[j].
__global__ void pq_init(const float* X, int d, const int64_t* sample, const int64_t* init, int m,
                        int ksub, float* cb) {
  const int ds = d / m;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // over m * ksub * ds
  if (i >= (int64_t)m * ksub * ds) return;
  const int t = (int)(i % ds);
  const int j = (int)((i / ds) % ksub);
  const int sub = (int)(i / ((int64_t)ds * ksub));
  cb[i] = X[(size_t)sample[init[j]] * d + (size_t)sub * ds + t];
}

int check_pq_shape(int64_t n, int d, int m, int ksub) {
  if (n < 1) return fail(ANN_EINVAL, "n < 1");
  if (d < 1 || m < 1 || d % m != 0) return fail(ANN_EINVAL, "d %d not a multiple of m %d", d, m);
  if (d / m > kMaxSub) return fail(ANN_EUNSUP, "subspaces of %d dimensions (at most %d)", d / m, kMaxSub);
  if (ksub < 1 || ksub > kMaxKsub) return fail(ANN_EINVAL, "ksub %d outside [1, %d]", ksub, kMaxKsub);
  if (m > 65535) return fail(ANN_EINVAL, "m %d too large", m);
  return ANN_OK;
}

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" int ann_pq_encode(const float* X, int64_t n, int32_t d, const float* codebook, int32_t m,
                             int32_t ksub, uint8_t* out_codes, void* stream) {
  int rc = check_pq_shape(n, d, m, ksub);
  if (rc) return rc;
  if (!X || !codebook || !out_codes) return fail(ANN_EINVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)m);
  hipLaunchKernelGGL(pq_assign, grid, dim3(256), 0, st, X, d, (const int64_t*)nullptr, n, codebook,
                     m, ksub, out_codes, (int32_t*)nullptr, (double*)nullptr, (int32_t*)nullptr,
                     (const int32_t*)nullptr);
  HIP_OR_RETURN(hipGetLastError(), "pq_assign launch");
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "pq encode");
  return ANN_OK;
}

extern "C" int ann_pq_train(const float* X, int64_t n, int32_t d, const int64_t* sample, int64_t ns,
                            const int64_t* init, int32_t m, int32_t ksub, int32_t max_iter,
                            float* out_codebook, int32_t* out_iters, void* stream) {
  int rc = check_pq_shape(n, d, m, ksub);
  if (rc) return rc;
  if (!X || !sample || !init || !out_codebook) return fail(ANN_EINVAL, "NULL pointer");
  if (ns < ksub) return fail(ANN_EINVAL, "sample of %lld points for %d centroids", (long long)ns, ksub);
  if (max_iter < 1) return fail(ANN_EINVAL, "max_iter < 1");
  hipStream_t st = (hipStream_t)stream;
  int32_t *asg = nullptr, *flags = nullptr;
  double* err = nullptr;
  // asg [m][ns] (-1 at first: iteration 0 always changes), err [m][ns],
  // flags: changed [m], active [m], empty [m][ksub]
  const size_t nflag = (size_t)m * 2 + (size_t)m * ksub;
  auto cleanup = [&]() {
    if (asg) (void)hipFree(asg);
    if (err) (void)hipFree(err);
    if (flags) (void)hipFree(flags);
  };
  if (hipMalloc((void**)&asg, sizeof(int32_t) * (size_t)m * ns) != hipSuccess ||
      hipMalloc((void**)&err, sizeof(double) * (size_t)m * ns) != hipSuccess ||
      hipMalloc((void**)&flags, sizeof(int32_t) * nflag) != hipSuccess) {
    cleanup();
    return fail(ANN_ENOMEM, "PQ training scratch");
  }
  int32_t* changed = flags;
  int32_t* active = flags + m;
  int32_t* empty = flags + 2 * m;
  std::vector<int32_t> h_changed((size_t)m), h_active((size_t)m, 1);
  int iters = 0;
  hipError_t e = hipMemsetAsync(asg, 0xFF, sizeof(int32_t) * (size_t)m * ns, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(active, h_active.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    const int64_t tot = (int64_t)m * ksub * (d / m);
    hipLaunchKernelGGL(pq_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, d, sample,
                       init, m, ksub, out_codebook);
    e = hipGetLastError();
  }
  for (int it = 0; it < max_iter && e == hipSuccess; ++it) {
    e = hipMemsetAsync(changed, 0, sizeof(int32_t) * m, st);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(pq_assign, dim3((unsigned)((ns + 255) / 256), (unsigned)m), dim3(256), 0, st,
                       X, d, sample, ns, out_codebook, m, ksub, (uint8_t*)nullptr, asg, err, changed,
                       active);
    if ((e = hipGetLastError()) != hipSuccess) break;
    e = hipMemcpyAsync(h_changed.data(), changed, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) break;
    // a subspace whose assignment did not change stops here (iterations it + 1)
    bool any = false;
    for (int s = 0; s < m; ++s) {
      if (h_active[s] && !h_changed[s]) { h_active[s] = 0; iters = std::max(iters, it + 1); }
      any = any || h_active[s];
    }
    if (!any) break;
    if (it + 1 == max_iter) iters = max_iter;
    e = hipMemcpyAsync(active, h_active.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(pq_update, dim3((unsigned)((ksub + 255) / 256), (unsigned)m), dim3(256), 0, st,
                       X, d, sample, ns, m, ksub, asg, out_codebook, empty, active);
    if ((e = hipGetLastError()) != hipSuccess) break;
    hipLaunchKernelGGL(pq_reseed, dim3((unsigned)m), dim3(256), 0, st, X, d, sample, ns, m, ksub, err,
                       empty, out_codebook, active);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "PQ training");
  if (out_iters) *out_iters = iters;
  return ANN_OK;
}
