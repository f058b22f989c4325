// Deterministic reductions: a fixed grid of per-block partial sums, then a
// single block sums the partials in a fixed order, so repeated calls are
// bitwise identical.  FP64 throughout.
#include "kernels.h"

namespace dcsd {

namespace {
constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;
}  // namespace

__device__ double block_sum(double v) {
  __shared__ double sh[RED_THREADS];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}
__device__ double block_max(double v) {
  __shared__ double sh[RED_THREADS];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  return sh[0];
}

__global__ void dot_partial(const double* x, const double* y, int64_t n, double* part) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ void maxabs_partial(const double* x, int64_t n, double* part, int* nonfinite) {
  double m = 0.0;
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double a = fabs(x[i]);
    if (!(a <= 1.7976931348623157e308)) bad = 1;
    else m = fmax(m, a);
  }
  m = block_max(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
  if (bad) nonfinite[0] = 1;
}
__global__ void final_sum(const double* part, int np, double* out, int mode) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s = mode ? fmax(s, part[i]) : s + part[i];
  s = mode ? block_max(s) : block_sum(s);
  if (threadIdx.x == 0) *out = s;
}

void dot(const double* x, const double* y, int64_t n, double* out_dev, double* part, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, y, n, part);
  DCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(final_sum, dim3(1), dim3(RED_THREADS), 0, s, (const double*)part, RED_BLOCKS, out_dev, 0);
  DCSD_CHECK_LAUNCH();
}
void maxabs(const double* x, int64_t n, double* out_dev, int* nonfinite_dev, double* part, hipStream_t s) {
  hipLaunchKernelGGL(maxabs_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, n, part, nonfinite_dev);
  DCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(final_sum, dim3(1), dim3(RED_THREADS), 0, s, (const double*)part, RED_BLOCKS, out_dev, 1);
  DCSD_CHECK_LAUNCH();
}

// Energy of Phi_A's amplitudes (undressed integrals):
//   dE_A = sum_s f^s_ia t1^s_ia + 1/2 sum (ia|jb)_ss tau^ss + 1/2 sum (IA|JB) tau^bb
//        + sum (ia|JB) tau^ab,   tau = t2 + t1 t1 (antisymmetrised for equal spins).
__global__ void energy_partial(const double* T, const double* Isc, const double* fa, const double* fb, int nc, int o,
                               int v, int n, double* part) {
  const int64_t ov = (int64_t)o * v, s2 = ov * ov, tov = 2 * ov;
  const int64_t total = 2 * ov + 3 * s2;
  double acc = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (x < 2 * ov) {
      const int spin = (int)(x / ov);
      const int i = (int)((x % ov) / v), a = (int)(x % v);
      const double* f = spin ? fb : fa;
      acc += f[(int64_t)i * n + o + a] * T[x];
      continue;
    }
    const int64_t y = x - 2 * ov;
    const int blk = (int)(y / s2);
    int64_t r = y % s2;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o);
    const int i = (int)(r / o);
    const int si = blk == 1 ? 1 : 0, sj = blk == 0 ? 0 : 1;
    const double* t1i = T + si * ov;
    const double* t1j = T + sj * ov;
    double tau = T[x] + t1i[i * v + a] * t1j[j * v + b];
    double fac = 1.0;
    if (blk < 2) {
      tau -= t1i[i * v + b] * t1j[j * v + a];
      fac = 0.5;
    }
    const double I = Isc[(si * ov + (int64_t)i * v + a) * tov + sj * ov + (int64_t)j * v + b];
    acc += fac * I * tau;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
void energy(const double* T, const double* Isc, const double* fa, const double* fb, int nc, int o, int v, int n,
            double* out_dev, double* part, hipStream_t s) {
  hipLaunchKernelGGL(energy_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, T, Isc, fa, fb, nc, o, v, n, part);
  DCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(final_sum, dim3(1), dim3(RED_THREADS), 0, s, (const double*)part, RED_BLOCKS, out_dev, 0);
  DCSD_CHECK_LAUNCH();
}

}  // namespace dcsd
