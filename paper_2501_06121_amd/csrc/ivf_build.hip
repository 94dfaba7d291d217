// Construction of the IVF index on the device: k-means training of the coarse
// centroids and the assignment of every row to its list.  The paper names the
// IVF family (Section 1) and plans more index types (Section 4, Conclusions and Future Work); the coarse
// quantizer is Lloyd's k-means over whole vectors, the procedure the PQ
// training applies per subspace (Section 2 and its citation, Jegou et al.).
//
// Every distance is the squared L2 distance of a row to a centroid, summed in
// FP64 from the FP32 inputs in ascending dimension order (one subtraction,
// one multiply and one add per dimension, no fusion); the nearest centroid is
// the first minimum (lower index on ties).  Training assigns every sample
// point, stops when no assignment changed, else replaces each centroid by the
// FP64 mean of its points (summed in ascending sample order, rounded once to
// FP32); an empty cluster takes the sample point of largest current error
// (lower position on ties, each point used once per step), clusters in
// ascending order.  The results are therefore fixed bit for bit by the inputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "ann.h"
#include "internal.h"

namespace ann {
namespace {

constexpr int kRows = 64;     // rows per workgroup of the assignment
constexpr int kCents = 64;    // centroids per tile
constexpr int kDims = 32;     // dimensions per LDS stage
constexpr int kMaxLists = 8192;    // the largest list count the IVF search takes

// Nearest centroid of np rows (row a is rows[a] of X, or a when rows is NULL).
// 256 threads: thread (tx, ty) = (tid % 16, tid / 16) accumulates rows
// ty + 16 i (i < 4) against centroids tx + 16 j (j < 4) of each 64-centroid
// tile, dimension by dimension from LDS stages of 32 dimensions; each keeps the
// first minimum over its centroids (visited in ascending order) and the 16
// threads of a row then take the smallest (distance, index).  Writes asg[a];
// when err is given also err[a], and changed[0] = 1 when asg[a] differs from
// its previous value.
__global__ void __launch_bounds__(256) ivf_assign(const float* X, int d, const int64_t* rows,
                                                  int64_t np, const float* cent, int nlist,
                                                  int32_t* asg, double* err, int32_t* changed) {
  __shared__ float xs[kDims][kRows + 1];
  __shared__ float cs[kDims][kCents + 1];
  __shared__ double rd[kRows][17];
  __shared__ int32_t ri[kRows][17];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  double bd[4];
  int bi[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) { bd[i] = __builtin_inf(); bi[i] = 0x7FFFFFFF; }
  for (int c0 = 0; c0 < nlist; c0 += kCents) {
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int t0 = 0; t0 < d; t0 += kDims) {
      __syncthreads();
      for (int e = tid; e < kRows * kDims; e += 256) {
        const int r = e / kDims, t = e % kDims;
        const int64_t a = r0 + r;
        float v = 0.0f;
        if (a < np && t0 + t < d) v = X[(size_t)(rows ? rows[a] : a) * d + t0 + t];
        xs[t][r] = v;
      }
      for (int e = tid; e < kCents * kDims; e += 256) {
        const int c = e / kDims, t = e % kDims;
        float v = 0.0f;
        if (c0 + c < nlist && t0 + t < d) v = cent[(size_t)(c0 + c) * d + t0 + t];
        cs[t][c] = v;
      }
      __syncthreads();
      const int tl = d - t0 < kDims ? d - t0 : kDims;
      for (int t = 0; t < tl; ++t) {
        double xv[4], cv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) xv[i] = (double)xs[t][ty + 16 * i];
#pragma unroll
        for (int j = 0; j < 4; ++j) cv[j] = (double)cs[t][tx + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double u = xv[i] - cv[j];
            acc[i][j] = acc[i][j] + u * u;
          }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tx + 16 * j;
      if (c < nlist) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (acc[i][j] < bd[i]) { bd[i] = acc[i][j]; bi[i] = c; }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) { rd[ty + 16 * i][tx] = bd[i]; ri[ty + 16 * i][tx] = bi[i]; }
  __syncthreads();
  if (tid < kRows) {
    const int64_t a = r0 + tid;
    if (a < np) {
      double best = rd[tid][0];
      int bj = ri[tid][0];
      for (int x = 1; x < 16; ++x) {
        const double v = rd[tid][x];
        const int vj = ri[tid][x];
        if (v < best || (v == best && vj < bj)) { best = v; bj = vj; }
      }
      if (err) {
        if (asg[a] != bj) changed[0] = 1;
        err[a] = best;
      }
      asg[a] = bj;
    }
  }
}

// Centroid j = blockIdx.x, dimensions blockIdx.y * 256 + tid: the FP64 sum of
// its sample points in ascending sample order (the block walks the assignment
// in LDS chunks; the membership test is the same for all its threads), divided
// by their count and rounded to FP32.  Clusters without points keep their
// centroid and are flagged in empty[j].
__global__ void __launch_bounds__(256) ivf_update(const float* X, int d, const int64_t* sample,
                                                  int64_t ns, const int32_t* asg, float* cent,
                                                  int32_t* empty) {
  constexpr int kChunk = 4096;
  __shared__ int32_t A[kChunk];
  const int j = blockIdx.x;
  const int t = blockIdx.y * 256 + threadIdx.x;
  double sum = 0.0;
  int64_t cnt = 0;
  for (int64_t a0 = 0; a0 < ns; a0 += kChunk) {
    const int len = ns - a0 < kChunk ? (int)(ns - a0) : kChunk;
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += 256) A[i] = asg[a0 + i];
    __syncthreads();
    for (int i = 0; i < len; ++i) {
      if (A[i] != j) continue;
      ++cnt;
      if (t < d) sum = sum + (double)X[(size_t)sample[a0 + i] * d + t];
    }
  }
  if (cnt > 0 && t < d) cent[(size_t)j * d + t] = (float)(sum / (double)cnt);
  if (blockIdx.y == 0 && threadIdx.x == 0) empty[j] = cnt == 0 ? 1 : 0;
}

// Empty clusters, in ascending order, each take the sample point of largest
// error not taken before (lower position on ties): one block-wide argmax per
// empty cluster; a taken point's error becomes -1 (errors are >= 0).
__global__ void __launch_bounds__(256) ivf_reseed(const float* X, int d, const int64_t* sample,
                                                  int64_t ns, int nlist, double* err,
                                                  const int32_t* empty, float* cent) {
  __shared__ double bk[256];
  __shared__ int64_t bi[256];
  for (int j = 0; j < nlist; ++j) {
    if (!empty[j]) continue;
    double mk = -2.0;
    int64_t mi = INT64_MAX;
    for (int64_t a = threadIdx.x; a < ns; a += blockDim.x) {
      const double e = err[a];
      if (e > mk) { mk = e; mi = a; }
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
    for (int t = threadIdx.x; t < d; t += blockDim.x)
      cent[(size_t)j * d + t] = X[(size_t)sample[pick] * d + t];
    __syncthreads();
    if (threadIdx.x == 0) err[pick] = -1.0;
    __syncthreads();
  }
}

// Centroid j starts at sample point init[j].
__global__ void ivf_init(const float* X, int d, const int64_t* sample, const int64_t* init,
                         int nlist, float* cent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nlist * d) return;
  const int t = (int)(i % d);
  const int j = (int)(i / d);
  cent[i] = X[(size_t)sample[init[j]] * d + t];
}

int check_shape(int64_t n, int d, int nlist) {
  if (n < 1) return fail(ANN_EINVAL, "n < 1");
  if (d < 1) return fail(ANN_EINVAL, "d < 1");
  if (nlist < 1 || nlist > kMaxLists) return fail(ANN_EINVAL, "nlist %d outside [1, %d]", nlist, kMaxLists);
  return ANN_OK;
}

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" int ann_ivf_assign(const float* X, int64_t n, int32_t d, const float* centroids,
                              int32_t nlist, int32_t* out_list, void* stream) {
  int rc = check_shape(n, d, nlist);
  if (rc) return rc;
  if (!X || !centroids || !out_list) return fail(ANN_EINVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(ivf_assign, dim3((unsigned)((n + kRows - 1) / kRows)), dim3(256), 0, st, X, d,
                     (const int64_t*)nullptr, n, centroids, nlist, out_list, (double*)nullptr,
                     (int32_t*)nullptr);
  HIP_OR_RETURN(hipGetLastError(), "ivf_assign launch");
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "IVF assignment");
  return ANN_OK;
}

extern "C" int ann_ivf_train(const float* X, int64_t n, int32_t d, const int64_t* sample, int64_t ns,
                             const int64_t* init, int32_t nlist, int32_t max_iter,
                             float* out_centroids, int32_t* out_iters, void* stream) {
  int rc = check_shape(n, d, nlist);
  if (rc) return rc;
  if (!X || !sample || !init || !out_centroids) return fail(ANN_EINVAL, "NULL pointer");
  if (ns < nlist) return fail(ANN_EINVAL, "sample of %lld points for %d centroids", (long long)ns, nlist);
  if (max_iter < 1) return fail(ANN_EINVAL, "max_iter < 1");
  hipStream_t st = (hipStream_t)stream;
  // the kernels index rows through these: check them on the host first
  {
    std::vector<int64_t> hs((size_t)ns), hi((size_t)nlist);
    HIP_OR_RETURN(hipMemcpyAsync(hs.data(), sample, sizeof(int64_t) * (size_t)ns, hipMemcpyDeviceToHost, st), "sample copy");
    HIP_OR_RETURN(hipMemcpyAsync(hi.data(), init, sizeof(int64_t) * (size_t)nlist, hipMemcpyDeviceToHost, st), "init copy");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sample copy");
    for (int64_t a = 0; a < ns; ++a)
      if (hs[a] < 0 || hs[a] >= n) return fail(ANN_EINVAL, "sample[%lld] = %lld outside [0, %lld)", (long long)a, (long long)hs[a], (long long)n);
    for (int j = 0; j < nlist; ++j)
      if (hi[j] < 0 || hi[j] >= ns) return fail(ANN_EINVAL, "init[%d] = %lld outside [0, %lld)", j, (long long)hi[j], (long long)ns);
  }
  int32_t *asg = nullptr, *flags = nullptr;
  double* err = nullptr;
  auto cleanup = [&]() {
    if (asg) (void)hipFree(asg);
    if (err) (void)hipFree(err);
    if (flags) (void)hipFree(flags);
  };
  if (hipMalloc((void**)&asg, sizeof(int32_t) * (size_t)ns) != hipSuccess ||
      hipMalloc((void**)&err, sizeof(double) * (size_t)ns) != hipSuccess ||
      hipMalloc((void**)&flags, sizeof(int32_t) * (size_t)(1 + nlist)) != hipSuccess) {
    cleanup();
    return fail(ANN_ENOMEM, "IVF training scratch");
  }
  int32_t* changed = flags;
  int32_t* empty = flags + 1;
  int32_t h_changed = 0;
  int iters = max_iter;
  hipError_t e = hipMemsetAsync(asg, 0xFF, sizeof(int32_t) * (size_t)ns, st);
  if (e == hipSuccess) {
    const int64_t tot = (int64_t)nlist * d;
    hipLaunchKernelGGL(ivf_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, d, sample,
                       init, nlist, out_centroids);
    e = hipGetLastError();
  }
  for (int it = 0; it < max_iter && e == hipSuccess; ++it) {
    e = hipMemsetAsync(changed, 0, sizeof(int32_t), st);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(ivf_assign, dim3((unsigned)((ns + kRows - 1) / kRows)), dim3(256), 0, st, X, d,
                       sample, ns, (const float*)out_centroids, nlist, asg, err, changed);
    if ((e = hipGetLastError()) != hipSuccess) break;
    e = hipMemcpyAsync(&h_changed, changed, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) break;
    if (!h_changed) { iters = it + 1; break; }
    hipLaunchKernelGGL(ivf_update, dim3((unsigned)nlist, (unsigned)((d + 255) / 256)), dim3(256), 0, st,
                       X, d, sample, ns, asg, out_centroids, empty);
    if ((e = hipGetLastError()) != hipSuccess) break;
    hipLaunchKernelGGL(ivf_reseed, dim3(1), dim3(256), 0, st, X, d, sample, ns, nlist, err, empty,
                       out_centroids);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "IVF training");
  if (out_iters) *out_iters = iters;
  return ANN_OK;
}

extern "C" int ann_ivf_group(const int32_t* list, int64_t n, int32_t nlist, int64_t* list_off,
                             int32_t* list_ids) {
  if (!list || !list_off || !list_ids) return fail(ANN_EINVAL, "NULL pointer");
  if (n < 0 || n > INT32_MAX) return fail(ANN_EINVAL, "n %lld outside [0, 2^31 - 1]", (long long)n);
  if (nlist < 1) return fail(ANN_EINVAL, "nlist < 1");
  std::vector<int64_t> cnt((size_t)nlist + 1, 0);
  for (int64_t r = 0; r < n; ++r) {
    if (list[r] < 0 || list[r] >= nlist) return fail(ANN_EINVAL, "row %lld in list %d outside [0, %d)", (long long)r, list[r], nlist);
    ++cnt[(size_t)list[r] + 1];
  }
  for (int l = 0; l < nlist; ++l) cnt[(size_t)l + 1] += cnt[l];
  std::copy(cnt.begin(), cnt.end(), list_off);
  for (int64_t r = 0; r < n; ++r) list_ids[cnt[list[r]]++] = (int32_t)r;
  return ANN_OK;
}
