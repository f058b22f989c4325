// The library's FP64 GEMM with explicit operand layouts, for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).  Same arguments and the same kernels as
// dcsd_selftest_gemm_layout; the scratch that call allocates (split-K partial
// sums, or the partial dot products of small outputs over a long K, and the
// zero-padded operand copies) lives in a file-scope device array instead.  Each GPU holds its own copy of the array
// at its own address, looked up once per device with hipGetSymbolAddress; the
// array's name is never used as a device address in host code.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/libdcsd.h"
#include "common.h"
#include "kernels.h"

namespace dcsd {
void set_call_error(const char* msg);
}

namespace {

// 32 MiB of FP64 scratch per GPU, kept until the process ends.
constexpr int64_t kScratchDoubles = (int64_t)1 << 22;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double* g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up on the first call on a device).
hipError_t scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" dcsd_status dcsd_selftest_gemm_layout_noalloc(int64_t M, int64_t N, int64_t K, const double* A_dev,
                                                         int64_t lda, int32_t a_mc, const double* B_dev,
                                                         int64_t ldb, int32_t b_nc, double* C_dev, int64_t ldc,
                                                         double alpha, double beta, int32_t ksplit,
                                                         void* hip_stream) {
  if (M <= 0 || N <= 0 || K <= 0 || !A_dev || !B_dev || !C_dev || ksplit < 1) {
    dcsd::set_call_error("gemm_layout_noalloc: non-positive size, NULL pointer or ksplit < 1");
    return DCSD_ERR_ARG;
  }
  if (lda < (a_mc ? M : K) || ldb < (b_nc ? N : K) || ldc < N) {
    dcsd::set_call_error("gemm_layout_noalloc: leading dimension smaller than the stored extent");
    return DCSD_ERR_ARG;
  }
  const hipStream_t st = (hipStream_t)hip_stream;
  dcsd::GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A_dev; g.lda = lda; g.a_mc = a_mc != 0;
  g.B = B_dev; g.ldb = ldb; g.b_nc = b_nc != 0;
  g.C = C_dev; g.ldc = ldc; g.c_nc = true;
  g.alpha = alpha; g.beta = beta;
  g.ksplit = ksplit;
  // the same dispatch as dcsd_selftest_gemm_layout, with the same scratch sizes
  const int64_t small = ksplit == 1 ? dcsd::gemm_f64_small_work(g) : 0;
  // split-K partials, then (16-byte aligned) the zero-padded operand copies
  const int64_t split = small > 0 || ksplit == 1 ? 0 : (ksplit * M * ldc + 1) / 2 * 2;
  const int64_t padw = small > 0 ? 0 : dcsd::gemm_f64_pad_work(g);
  const double need = small > 0 ? (double)small : (double)split + (double)padw;
  if (need > (double)kScratchDoubles) {
    dcsd::set_call_error("gemm_layout_noalloc: the scratch it needs exceeds its 4194304 doubles (32 MiB)");
    return DCSD_ERR_ARG;
  }
  try {
    double* work = nullptr;
    if (need > 0.0 && scratch_on_current_device(&work) != hipSuccess) {
      dcsd::set_call_error("gemm_layout_noalloc: hipGetSymbolAddress of the scratch array failed");
      return DCSD_ERR_HIP;
    }
    if (small > 0) {
      if (!dcsd::gemm_f64_small(g, work, kScratchDoubles, st)) {
        dcsd::set_call_error("gemm_layout_noalloc: small-output product refused");
        return DCSD_ERR_HIP;
      }
    } else {
      g.work = split > 0 ? work : nullptr;
      if (padw > 0) {
        g.pad = work + split;
        g.pad_cap = padw;
      }
      dcsd::gemm_f64(g, st);
    }
    if (hipStreamSynchronize(st) != hipSuccess) return DCSD_ERR_HIP;
  } catch (const dcsd::ArgError& e) {
    dcsd::set_call_error(e.what());
    return DCSD_ERR_ARG;
  } catch (...) {
    dcsd::set_call_error("gemm_layout_noalloc: HIP error");
    return DCSD_ERR_HIP;
  }
  return DCSD_OK;
}
