// Internal declarations shared by the libdcsd sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace dcsd {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define DCSD_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::dcsd::HipError(std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

#define DCSD_CHECK_LAUNCH() DCSD_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Dense FP64 GEMM on MFMA:  C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n)
//
// Operand element addresses (one of the two strides of each operand is 1):
//   A(m,k): a_mc ? A[m + k*lda] : A[m*lda + k]
//   B(k,n): b_nc ? B[n + k*ldb] : B[n*ldb + k]
//   C(m,n): c_nc ? C[m*ldc + n] : C[m + n*ldc]
// Batched over `batch` with element strides sA, sB, sC.  With beta == 0, C is
// not read.  `ksplit` > 1 splits K across workgroups into a workspace and
// reduces in a fixed order (deterministic); it needs a workspace of
// ksplit*batch*M*N doubles.
// ---------------------------------------------------------------------------
struct GemmArgs {
  int64_t M = 0, N = 0, K = 0;
  const double* A = nullptr;
  int64_t lda = 0;
  bool a_mc = false;
  const double* B = nullptr;
  int64_t ldb = 0;
  bool b_nc = true;
  double* C = nullptr;
  int64_t ldc = 0;
  bool c_nc = true;
  double alpha = 1.0, beta = 0.0;
  int64_t batch = 1, sA = 0, sB = 0, sC = 0;
  int ksplit = 1;
  double* work = nullptr;
  // Workspace (pad_cap doubles, 16-byte aligned) for zero-padded copies of operands that the
  // direct-to-LDS kernel cannot stream as they are (an odd contiguous extent or leading
  // dimension, a base off 16 bytes, an odd batch stride); NULL: such products take the
  // register-staged kernel.
  double* pad = nullptr;
  int64_t pad_cap = 0;
};
void gemm_f64(const GemmArgs& g, hipStream_t s);
// Doubles of `pad` that gemm_f64 uses for g (0 if it copies no operand).
int64_t gemm_f64_pad_work(const GemmArgs& g);

// Generic strided copy with scaling, up to 6 dimensions:
//   dst[sum_d i_d*ds[d]] = alpha * src[sum_d i_d*ss[d]] + beta * dst[...]
struct Strided {
  int nd = 0;
  int64_t dims[6] = {1, 1, 1, 1, 1, 1};
  int64_t ds[6] = {0, 0, 0, 0, 0, 0};
  int64_t ss[6] = {0, 0, 0, 0, 0, 0};
};
void strided_copy(double* dst, const double* src, const Strided& st, double alpha, double beta,
                  hipStream_t s);

}  // namespace dcsd
