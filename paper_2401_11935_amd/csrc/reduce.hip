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

// Energy of the reference's amplitudes (undressed integrals):
//   dE = sum_s f^s_ia t1^s_ia + 1/2 sum (ia|jb)_ss tau^ss + 1/2 sum (IA|JB) tau^bb
//        + sum (ia|JB) tau^ab,   tau = t2 + t1 t1 (antisymmetrised for equal spins).
__global__ void energy_partial(const double* T, const double* Isc, const double* fa, const double* fb, SpinLayout L,
                               double* part) {
  const int n = L.n;
  const int64_t tov = L.ov(0) + L.ov(1), total = L.total(), t1end = L.t2_off(0);
  double acc = 0.0;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (x < t1end) {
      const int spin = x < L.ov(0) ? 0 : 1;
      const int64_t y = x - L.t1_off(spin);
      const int v = L.v[spin], o = L.o[spin];
      const int i = (int)(y / v), a = (int)(y % v);
      const double* f = spin ? fb : fa;
      acc += f[(int64_t)i * n + o + a] * T[x];
      continue;
    }
    const int blk = x < L.t2_off(1) ? 0 : (x < L.t2_off(2) ? 1 : 2);
    const int si = blk == 1 ? 1 : 0, sj = blk == 0 ? 0 : 1;
    int64_t r = x - L.t2_off(blk);
    const int vi = L.v[si], vj = L.v[sj], oj = L.o[sj];
    const int b = (int)(r % vj); r /= vj;
    const int a = (int)(r % vi); r /= vi;
    const int j = (int)(r % oj);
    const int i = (int)(r / oj);
    const double* t1i = T + L.t1_off(si);
    const double* t1j = T + L.t1_off(sj);
    double tau = T[x] + t1i[i * vi + a] * t1j[j * vj + b];
    double fac = 1.0;
    if (blk < 2) {
      tau -= t1i[i * vi + b] * t1j[j * vj + a];
      fac = 0.5;
    }
    const double I = Isc[(L.t1_off(si) + (int64_t)i * vi + a) * tov + L.t1_off(sj) + (int64_t)j * vj + b];
    acc += fac * I * tau;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
void energy(const double* T, const double* Isc, const double* fa, const double* fb, const SpinLayout& L,
            double* out_dev, double* part, hipStream_t s) {
  hipLaunchKernelGGL(energy_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, T, Isc, fa, fb, L, part);
  DCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(final_sum, dim3(1), dim3(RED_THREADS), 0, s, (const double*)part, RED_BLOCKS, out_dev, 0);
  DCSD_CHECK_LAUNCH();
}

}  // namespace dcsd
