// FP64 products with a small output and a long K: C (M x N, M, N <= 16) = alpha A B^T + beta C
// with A [M][K] and B [N][K] K-contiguous rows.  These are dot products of long rows and bound
// by HBM: the K range is split over many workgroups, each staging 128-long slices of the rows
// of A and B in LDS (coalesced row reads) and summing its part of every dot product (one
// thread per output element, ascending k); a second kernel adds the partial sums of each
// element in a fixed order and tree, so the result is deterministic.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace dcsd {

namespace {

constexpr int kSmall = 16, kSlice = 128;
constexpr int64_t kChunk = 2048;  // K per workgroup of the first kernel (a multiple of kSlice)

__global__ __launch_bounds__(256) void small_dots_kernel(const double* A, int64_t lda, const double* B, int64_t ldb,
                                                         int M, int N, int64_t K, int64_t kchunk, double* W) {
  __shared__ double sa[kSmall][kSlice + 1];
  __shared__ double sb[kSmall][kSlice + 1];
  const int t = threadIdx.x, m = t / kSmall, n = t % kSmall;
  const int64_t kbeg = (int64_t)blockIdx.x * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  double acc = 0.0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kSlice) {
    for (int e = t; e < kSmall * kSlice; e += 256) {
      const int row = e / kSlice, kk = e % kSlice;
      const bool in = k0 + kk < kend;
      sa[row][kk] = row < M && in ? A[row * lda + k0 + kk] : 0.0;
      sb[row][kk] = row < N && in ? B[row * ldb + k0 + kk] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kSlice; ++kk) acc = __builtin_fma(sa[m][kk], sb[n][kk], acc);
    __syncthreads();
  }
  if (m < M && n < N) W[(int64_t)blockIdx.x * M * N + m * N + n] = acc;
}

// one workgroup per output element: thread t adds partials t, t + 256, ... in order, then a
// fixed binary tree over the threads
__global__ __launch_bounds__(256) void small_reduce_kernel(const double* W, double* C, int M, int N, int64_t ldc,
                                                           bool c_nc, int nsplit, double alpha, double beta) {
  __shared__ double part[256];
  const int e = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int z = t; z < nsplit; z += 256) s += W[(int64_t)z * M * N + e];
  part[t] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) part[t] += part[t + h];
    __syncthreads();
  }
  if (t == 0) {
    const int m = e / N, n = e % N;
    double* c = C + (c_nc ? m * ldc + n : m + n * ldc);
    double v = alpha * part[0];
    if (beta != 0.0) v += beta * *c;
    *c = v;
  }
}

}  // namespace

int64_t gemm_f64_small_work(const GemmArgs& g) {
  if (g.M < 1 || g.N < 1 || g.M > kSmall || g.N > kSmall || g.batch != 1 || g.a_mc || g.b_nc || g.K < 65536)
    return 0;
  const int64_t nsplit = (g.K + kChunk - 1) / kChunk;
  return nsplit < ((int64_t)1 << 31) ? nsplit * g.M * g.N : 0;
}

bool gemm_f64_small(const GemmArgs& g, double* work, int64_t work_cap, hipStream_t s) {
  const int64_t need = gemm_f64_small_work(g);
  if (need == 0 || !work || need > work_cap) return false;
  const int64_t kchunk = kChunk, nsplit = (g.K + kchunk - 1) / kchunk;
  hipLaunchKernelGGL(small_dots_kernel, dim3((unsigned)nsplit), dim3(256), 0, s, g.A, g.lda, g.B, g.ldb, (int)g.M,
                     (int)g.N, g.K, kchunk, work);
  DCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(small_reduce_kernel, dim3((unsigned)(g.M * g.N)), dim3(256), 0, s, (const double*)work, g.C,
                     (int)g.M, (int)g.N, g.ldc, g.c_nc, (int)nsplit, g.alpha, g.beta);
  DCSD_CHECK_LAUNCH();
  return true;
}

}  // namespace dcsd
