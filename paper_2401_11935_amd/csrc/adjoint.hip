// Adjoints (vector-Jacobian products) of the residual's non-GEMM device
// operations.  Each kernel accumulates into the shadow ("bar") arrays of its
// inputs what the forward operation's output cotangent implies; outputs that
// the forward operation overwrote are cleared by the caller.  Gathers are used
// wherever a forward scatter touched each element once, so that these sums are
// deterministic; only the coupling adjoint scatters with atomics.
#include "kernels.h"

namespace dcsd {

namespace {
__device__ inline int occ_sp(int spin, int i, int nc) { return i < nc ? i : nc + spin; }
__device__ inline int vir_sp(int spin, int a, int nc) { return a > 0 ? nc + 1 + a : nc + 1 - spin; }
// spatial orbital p -> occupied / virtual index of the given spin (-1 if not of that kind)
__device__ inline int occ_of(int spin, int p, int nc) { return p < nc ? p : (p == nc + spin ? nc : -1); }
__device__ inline int vir_of(int spin, int p, int nc) {
  return p >= nc + 2 ? p - nc - 1 : (p == nc + 1 - spin ? 0 : -1);
}
__device__ inline void row_spins(int64_t r, int64_t o2, int64_t npair, int& s1, int& s2) {
  if (r < o2) { s1 = 0; s2 = 1; }
  else if (r < o2 + npair) { s1 = 0; s2 = 0; }
  else { s1 = 1; s2 = 1; }
}
inline unsigned nb(int64_t total, int threads = 256) {
  int64_t b = (total + threads - 1) / threads;
  if (b > (1 << 20)) b = 1 << 20;
  return (unsigned)(b < 1 ? 1 : b);
}
}  // namespace

// ---- t <-> u exchange: src_bar[P][p][q] += dst_bar[P][swap p][swap q] --------------
__global__ void swap_tu_acc_kernel(double* acc, const double* src, int64_t batch, int n, int nc) {
  const int64_t n2 = (int64_t)n * n, total = batch * n2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t P = idx / n2;
    int p = (int)((idx % n2) / n), q = (int)(idx % n);
    p = p == nc ? nc + 1 : (p == nc + 1 ? nc : p);
    q = q == nc ? nc + 1 : (q == nc + 1 ? nc : q);
    acc[idx] += src[P * n2 + (int64_t)p * n + q];
  }
}
void swap_tu_adj(double* src_bar, const double* dst_bar, int64_t batch, int n, int nc, hipStream_t s) {
  hipLaunchKernelGGL(swap_tu_acc_kernel, dim3(nb(batch * (int64_t)n * n)), dim3(256), 0, s, src_bar, dst_bar, batch,
                     n, nc);
  DCSD_CHECK_LAUNCH();
}

// ---- J[P] = sum_{k<o} Ba[P,k,k] + Bb[P,k,k] ------------------------------------------
__global__ void jvec_adj_kernel(double* Ba_bar, double* Bb_bar, const double* J_bar, int64_t naux, int n, int o) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= naux * o) return;
  const int64_t P = idx / o;
  const int k = (int)(idx % o);
  const int64_t off = P * n * n + (int64_t)k * n + k;
  Ba_bar[off] += J_bar[P];
  Bb_bar[off] += J_bar[P];
}
void jvector_adj(double* Ba_bar, double* Bb_bar, const double* J_bar, int64_t naux, int n, int o, hipStream_t s) {
  hipLaunchKernelGGL(jvec_adj_kernel, dim3(nb(naux * o)), dim3(256), 0, s, Ba_bar, Bb_bar, J_bar, naux, n, o);
  DCSD_CHECK_LAUNCH();
}

// ---- dst[od] += alpha sum_b src[b*bstride + r*ld + c] ------------------------------------
__global__ void batch_reduce_adj_kernel(double* src_bar, const double* dst_bar, int64_t nbat, int64_t bstride,
                                        int rows, int cols, int64_t ld, int64_t ldd, int transpose, double alpha) {
  const int64_t rc = (int64_t)rows * cols, total = nbat * rc;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / rc;
    const int r = (int)((idx % rc) / cols), c = (int)(idx % cols);
    const int64_t od = transpose ? (int64_t)c * ldd + r : (int64_t)r * ldd + c;
    src_bar[b * bstride + (int64_t)r * ld + c] += alpha * dst_bar[od];
  }
}
void batch_reduce_adj(double* src_bar, const double* dst_bar, int64_t nbat, int64_t bstride, int rows, int cols,
                      int64_t ld, int64_t ldd, bool transpose, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(batch_reduce_adj_kernel, dim3(nb(nbat * (int64_t)rows * cols)), dim3(256), 0, s, src_bar,
                     dst_bar, nbat, bstride, rows, cols, ld, ldd, transpose ? 1 : 0, alpha);
  DCSD_CHECK_LAUNCH();
}

// ---- ladder amplitude stack: t2_bar += gather of the stack's cotangent ---------------
// (inverse of the stack's union-virtual maps: alpha vir c -> u = c + 1, beta vir d -> 0 (t) or d + 1)
__device__ inline int upos_alpha(int c) { return c + 1; }
__device__ inline int upos_beta(int d) { return d == 0 ? 0 : d + 1; }
__global__ void ladder_stack_adj_kernel(double* t2aa_bar, double* t2bb_bar, double* t2ab_bar, const double* Sbar,
                                        int o, int v, int vu, int npair) {
  const int64_t vv = (int64_t)v * v, s2 = (int64_t)o * o * vv, vu2 = (int64_t)vu * vu, o2 = (int64_t)o * o;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < 3 * s2;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int blk = (int)(x / s2);
    const int64_t y = x % s2;
    const int d = (int)(y % v), c = (int)((y / v) % v);
    const int64_t ij = y / vv;
    const int i = (int)(ij / o), j = (int)(ij % o);
    if (blk == 2) {
      const int cu = upos_alpha(c), du = upos_beta(d);
      double g = Sbar[ij * vu2 + (int64_t)cu * vu + du];
      g += Sbar[(o2 + 2 * npair + ij) * vu2 + (int64_t)du * vu + cu];  // transposed rows
      t2ab_bar[y] += g;
    } else if (i < j) {
      const int64_t q = (int64_t)i * o - (int64_t)i * (i + 1) / 2 + (j - i - 1);
      const int64_t row = o2 + (blk == 0 ? q : npair + q);
      const int cu = blk == 0 ? upos_alpha(c) : upos_beta(c), du = blk == 0 ? upos_alpha(d) : upos_beta(d);
      (blk == 0 ? t2aa_bar : t2bb_bar)[y] += Sbar[row * vu2 + (int64_t)cu * vu + du];
    }
  }
}
void ladder_stack_adj(double* t2aa_bar, double* t2bb_bar, double* t2ab_bar, const double* Sbar, int o, int v, int vu,
                      int npair, hipStream_t s) {
  const int64_t s2 = (int64_t)o * o * v * v;
  hipLaunchKernelGGL(ladder_stack_adj_kernel, dim3(nb(3 * s2)), dim3(256), 0, s, t2aa_bar, t2bb_bar, t2ab_bar, Sbar, o,
                     v, vu, npair);
  DCSD_CHECK_LAUNCH();
}

// ---- one ladder batch: Rb_bar = gather of Rp_bar (inverse of the scatter) --------------
__global__ void ladder_scatter_adj_kernel(double* Rb_bar, const double* Rp_bar, int64_t rows_used, int64_t nrow_main,
                                          int64_t nsame_begin, int n, int p0, int np, int q0, int nq, int diag) {
  const int64_t npq = (int64_t)np * nq, total = rows_used * npq, n2 = (int64_t)n * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / npq;
    const int p = p0 + (int)((idx % npq) / nq), q = q0 + (int)(idx % nq);
    double g;
    if (r < nrow_main) {
      g = Rp_bar[r * n2 + (int64_t)p * n + q];
      if (!diag && r >= nsame_begin) g -= Rp_bar[r * n2 + (int64_t)q * n + p];
    } else {
      g = Rp_bar[(r - nrow_main) * n2 + (int64_t)q * n + p];
    }
    Rb_bar[idx] = g;
  }
}
void ladder_scatter_adj(double* Rb_bar, const double* Rp_bar, int64_t rows_used, int64_t nrow_main,
                        int64_t nsame_begin, int n, int p0, int np, int q0, int nq, bool diag, hipStream_t s) {
  hipLaunchKernelGGL(ladder_scatter_adj_kernel, dim3(nb(rows_used * (int64_t)np * nq)), dim3(256), 0, s, Rb_bar,
                     Rp_bar, rows_used, nrow_main, nsame_begin, n, p0, np, q0, nq, diag ? 1 : 0);
  DCSD_CHECK_LAUNCH();
}

// ---- T1 back-transformation of the ladder -------------------------------------------
// Forward, per row r with spins (s1, s2):
//   S[r][p][b]    = Rp[r][p][vir(s2,b)] - sum_l t1_s2[l,b] Rp[r][p][occ(s2,l)]
//   val[r][a][b]  = S[r][vir(s1,a)][b]  - sum_k t1_s1[k,a] S[r][occ(s1,k)][b]
//   R2 += val (alpha-beta rows), R2[i,j] += val and R2[j,i] -= val (pair rows).
// VB = cotangent of val.
__global__ void mt_valbar_kernel(double* VB, const double* R2aa_bar, const double* R2bb_bar, const double* R2ab_bar,
                                 const int* pair_i, const int* pair_j, int64_t rows, int64_t o2, int64_t npair, int o,
                                 int v) {
  const int64_t vv = (int64_t)v * v, total = rows * vv;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / vv, ab = idx % vv;
    if (r < o2) {
      VB[idx] = R2ab_bar[r * vv + ab];
    } else {
      const int64_t q = r < o2 + npair ? r - o2 : r - o2 - npair;
      const double* R = r < o2 + npair ? R2aa_bar : R2bb_bar;
      const int i = pair_i[q], j = pair_j[q];
      VB[idx] = R[((int64_t)i * o + j) * vv + ab] - R[((int64_t)j * o + i) * vv + ab];
    }
  }
}
// S_bar[r][p][b] from VB (second step)
__global__ void mt2_adj_S_kernel(double* Sbar, const double* VB, const double* t1a, const double* t1b, int64_t rows,
                                 int64_t o2, int64_t npair, int n, int nc, int v) {
  const int64_t total = rows * n * v;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / ((int64_t)n * v);
    const int p = (int)((idx / v) % n), b = (int)(idx % v);
    int s1, s2;
    row_spins(r, o2, npair, s1, s2);
    const double* VBr = VB + r * (int64_t)v * v;
    double g = 0.0;
    const int a = vir_of(s1, p, nc);
    if (a >= 0) {
      g = VBr[(int64_t)a * v + b];
    } else {
      const int k = occ_of(s1, p, nc);
      const double* t1 = s1 == 0 ? t1a : t1b;
      for (int aa = 0; aa < v; ++aa) g -= t1[(int64_t)k * v + aa] * VBr[(int64_t)aa * v + b];
    }
    Sbar[idx] = g;
  }
}
// t1_bar[s][k][a] -= sum_{rows with s1 = s} sum_b VB[r][a][b] S[r][occ(s,k)][b]   (one thread per (s,k,a))
__global__ void mt2_adj_t1_kernel(double* t1bar, const double* VB, const double* S, int64_t rows, int64_t o2,
                                  int64_t npair, int n, int nc, int o, int v) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= 2 * (int64_t)o * v) return;
  const int s = (int)(id / ((int64_t)o * v));
  const int k = (int)((id / v) % o), a = (int)(id % v);
  const int pk = occ_sp(s, k, nc);
  double acc = 0.0;
  for (int64_t r = 0; r < rows; ++r) {
    int s1, s2;
    row_spins(r, o2, npair, s1, s2);
    if (s1 != s) continue;
    const double* VBr = VB + r * (int64_t)v * v + (int64_t)a * v;
    const double* Sr = S + (r * n + pk) * (int64_t)v;
    for (int b = 0; b < v; ++b) acc += VBr[b] * Sr[b];
  }
  t1bar[id] -= acc;
}
// Rp_bar[r][p][q] += contribution of S_bar (first step)
__global__ void mt1_adj_R_kernel(double* Rpbar, const double* Sbar, const double* t1a, const double* t1b,
                                 int64_t rows, int64_t o2, int64_t npair, int n, int nc, int v) {
  const int64_t n2 = (int64_t)n * n, total = rows * n2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / n2;
    const int p = (int)((idx % n2) / n), q = (int)(idx % n);
    int s1, s2;
    row_spins(r, o2, npair, s1, s2);
    const double* Sb = Sbar + (r * n + p) * (int64_t)v;
    double g = 0.0;
    const int b = vir_of(s2, q, nc);
    if (b >= 0) {
      g = Sb[b];
    } else {
      const int l = occ_of(s2, q, nc);
      const double* t1 = s2 == 0 ? t1a : t1b;
      for (int bb = 0; bb < v; ++bb) g -= t1[(int64_t)l * v + bb] * Sb[bb];
    }
    Rpbar[idx] += g;
  }
}
// t1_bar[s][l][b] -= sum_{rows with s2 = s} sum_p S_bar[r][p][b] Rp[r][p][occ(s,l)]   (one thread per (s,l,b))
__global__ void mt1_adj_t1_kernel(double* t1bar, const double* Sbar, const double* Rp, int64_t rows, int64_t o2,
                                  int64_t npair, int n, int nc, int o, int v) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= 2 * (int64_t)o * v) return;
  const int s = (int)(id / ((int64_t)o * v));
  const int l = (int)((id / v) % o), b = (int)(id % v);
  const int pl = occ_sp(s, l, nc);
  const int64_t n2 = (int64_t)n * n;
  double acc = 0.0;
  for (int64_t r = 0; r < rows; ++r) {
    int s1, s2;
    row_spins(r, o2, npair, s1, s2);
    if (s2 != s) continue;
    for (int p = 0; p < n; ++p) acc += Sbar[(r * n + p) * (int64_t)v + b] * Rp[r * n2 + (int64_t)p * n + pl];
  }
  t1bar[id] -= acc;
}
void ladder_mtransform_adj(double* Rpbar, double* t1bar, const double* R2aa_bar, const double* R2bb_bar,
                           const double* R2ab_bar, const double* Rp, const double* t1a, const double* t1b,
                           const int* pair_i, const int* pair_j, int64_t rows, int64_t o2, int64_t npair, int n,
                           int nc, int o, int v, double* VB, double* S, double* Sbar, hipStream_t s) {
  const int64_t vv = (int64_t)v * v;
  hipLaunchKernelGGL(mt_valbar_kernel, dim3(nb(rows * vv)), dim3(256), 0, s, VB, R2aa_bar, R2bb_bar, R2ab_bar, pair_i,
                     pair_j, rows, o2, npair, o, v);
  DCSD_CHECK_LAUNCH();
  // S of the forward (first step), recomputed
  ladder_mt1(S, Rp, t1a, t1b, rows, o2, npair, n, nc, o, v, s);
  hipLaunchKernelGGL(mt2_adj_S_kernel, dim3(nb(rows * n * v)), dim3(256), 0, s, Sbar, VB, t1a, t1b, rows, o2, npair,
                     n, nc, v);
  DCSD_CHECK_LAUNCH();
  if (t1bar) {
    hipLaunchKernelGGL(mt2_adj_t1_kernel, dim3(nb(2 * (int64_t)o * v, 64)), dim3(64), 0, s, t1bar, VB, S, rows, o2,
                       npair, n, nc, o, v);
    DCSD_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(mt1_adj_R_kernel, dim3(nb(rows * (int64_t)n * n)), dim3(256), 0, s, Rpbar, Sbar, t1a, t1b, rows,
                     o2, npair, n, nc, v);
  DCSD_CHECK_LAUNCH();
  if (t1bar) {
    hipLaunchKernelGGL(mt1_adj_t1_kernel, dim3(nb(2 * (int64_t)o * v, 64)), dim3(64), 0, s, t1bar, Sbar, Rp, rows,
                       o2, npair, n, nc, o, v);
    DCSD_CHECK_LAUNCH();
  }
}

// ---- energy of Phi_A: E = sum f_ia t_ia + sum fac (ia|jb) tau --------------------------
// Tbar += Ebar dE/dT (T with the layout of the packed amplitudes); with Ibar /
// fabar / fbbar non-null also the integral and Fock cotangents.
__global__ void energy_adj_kernel(double* Tbar, double* Ibar, double* fabar, double* fbbar, const double* T,
                                  const double* Isc, const double* fa, const double* fb, const double* Ebar, int o,
                                  int v, int n) {
  const int64_t ov = (int64_t)o * v, s2 = ov * ov, tov = 2 * ov, total = 2 * ov + 3 * s2;
  const double E = *Ebar;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (x < 2 * ov) {
      const int sp = (int)(x / ov);
      const int k = (int)((x % ov) / v), c = (int)(x % v);
      const double* f = sp ? fb : fa;
      const double* Irow = Isc + x * tov;  // (sp, k, c) row
      double g = f[(int64_t)k * n + o + c];
      for (int64_t y = 0; y < tov; ++y) g += Irow[y] * T[y];
      const double* t1 = T + sp * ov;
      for (int j = 0; j < o; ++j)
        for (int a = 0; a < v; ++a)
          g -= Isc[(sp * ov + (int64_t)k * v + a) * tov + sp * ov + (int64_t)j * v + c] * t1[(int64_t)j * v + a];
      Tbar[x] += E * g;
      if (fabar) (sp ? fbbar : fabar)[(int64_t)k * n + o + c] += E * T[x];
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
    const double fac = blk < 2 ? 0.5 : 1.0;
    const int64_t ii = (si * ov + (int64_t)i * v + a) * tov + sj * ov + (int64_t)j * v + b;
    Tbar[x] += E * fac * Isc[ii];
    if (Ibar) {
      const double* t1i = T + si * ov;
      const double* t1j = T + sj * ov;
      double tau = T[x] + t1i[i * v + a] * t1j[j * v + b];
      if (blk < 2) tau -= t1i[i * v + b] * t1j[j * v + a];
      Ibar[ii] += E * fac * tau;
    }
  }
}
void energy_adj(double* Tbar, double* Ibar, double* fabar, double* fbbar, const double* T, const double* Isc,
                const double* fa, const double* fb, const double* Ebar, int o, int v, int n, hipStream_t s) {
  const int64_t ov = (int64_t)o * v, total = 2 * ov + 3 * ov * ov;
  hipLaunchKernelGGL(energy_adj_kernel, dim3(nb(total)), dim3(256), 0, s, Tbar, Ibar, fabar, fbbar, T, Isc, fa, fb,
                     Ebar, o, v, n);
  DCSD_CHECK_LAUNCH();
}

// dst = src with the equal-spin doubles blocks projected on antisymmetric
// amplitudes: dst[ijab] = (src[ijab] - src[jiab] - src[ijba] + src[jiba]) / 4.
// The equal-spin amplitudes are stored in full but only their antisymmetric
// combinations are unknowns, so a cotangent with respect to T counts only
// through this projection.
__global__ void antisym_copy_kernel(double* dst, const double* src, int o, int v) {
  const int64_t ov = (int64_t)o * v, s2 = ov * ov, vv = (int64_t)v * v, total = 2 * ov + 3 * s2;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (x < 2 * ov || x >= 2 * ov + 2 * s2) {
      dst[x] = src[x];
      continue;
    }
    const int64_t base = x < 2 * ov + s2 ? 2 * ov : 2 * ov + s2;
    const int64_t y = x - base;
    const int b = (int)(y % v), a = (int)((y / v) % v);
    const int j = (int)((y / vv) % o), i = (int)(y / (vv * o));
    auto at = [&](int p, int q, int c, int d) { return src[base + (((int64_t)p * o + q) * v + c) * v + d]; };
    dst[x] = 0.25 * (at(i, j, a, b) - at(j, i, a, b) - at(i, j, b, a) + at(j, i, b, a));
  }
}
void antisym_copy(double* dst, const double* src, int o, int v, hipStream_t s) {
  const int64_t ov = (int64_t)o * v;
  hipLaunchKernelGGL(antisym_copy_kernel, dim3(nb(2 * ov + 3 * ov * ov)), dim3(256), 0, s, dst, src, o, v);
  DCSD_CHECK_LAUNCH();
}

// out[P][p][q] = (in[P][p][q] + in[P][q][p]) / 2 (gradient with respect to a symmetric matrix
// whose two mirrored entries move together by half the step each)
__global__ void symmetrize_kernel(double* out, const double* in, int64_t batch, int n) {
  const int64_t n2 = (int64_t)n * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < batch * n2;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t P = idx / n2;
    const int p = (int)((idx % n2) / n), q = (int)(idx % n);
    out[idx] = 0.5 * (in[idx] + in[P * n2 + (int64_t)q * n + p]);
  }
}
void symmetrize(double* out, const double* in, int64_t batch, int n, hipStream_t s) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nb(batch * (int64_t)n * n)), dim3(256), 0, s, out, in, batch, n);
  DCSD_CHECK_LAUNCH();
}

}  // namespace dcsd
