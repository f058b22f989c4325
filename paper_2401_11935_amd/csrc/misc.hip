// Element-wise, reduction and ladder bookkeeping kernels of the residual.
// All arithmetic is FP64; reductions use a fixed grid and a fixed summation
// order, so repeated calls give bitwise identical results.
#include "kernels.h"

namespace dcsd {

namespace {
inline unsigned nblocks(int64_t total, int threads, int64_t cap = 1 << 20) {
  int64_t b = (total + threads - 1) / threads;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}
}  // namespace

// ---------------------------------------------------------------------------
__global__ void fill_kernel(double* p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
void fill(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, p, v, n);
  DCSD_CHECK_LAUNCH();
}

__global__ void axpby_kernel(double* y, const double* x, double a, double b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];  // b == 0: y is not read
}
void axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, y, x, a, b, n);
  DCSD_CHECK_LAUNCH();
}

// J[P] = sum_k Bt_a[P,k,k] + sum_k Bt_b[P,k,k] over the occupied orbitals of each spin.
__global__ void jvec_kernel(double* J, const double* Ba, const double* Bb, int64_t naux, int n, int oa, int ob) {
  const int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (P >= naux) return;
  const double* a = Ba + P * n * n;
  const double* b = Bb + P * n * n;
  double s = 0.0;
  for (int k = 0; k < oa; ++k) s += a[k * n + k];
  for (int k = 0; k < ob; ++k) s += b[k * n + k];
  J[P] = s;
}
void jvector(double* J, const double* Ba, const double* Bb, int64_t naux, int n, int oa, int ob, hipStream_t s) {
  hipLaunchKernelGGL(jvec_kernel, dim3(nblocks(naux, 256)), dim3(256), 0, s, J, Ba, Bb, naux, n, oa, ob);
  DCSD_CHECK_LAUNCH();
}

// dst(r,c) += alpha * sum_b src[b*bstride + r*ld + c]   (dst(r,c) at dst[r*ldd + c], or transposed)
__global__ void batch_reduce_kernel(double* dst, const double* src, int64_t nb, int64_t bstride, int rows, int cols,
                                    int64_t ld, int64_t ldd, int transpose, double alpha) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rows * cols) return;
  const int r = (int)(idx / cols), c = (int)(idx % cols);
  double s = 0.0;
  for (int64_t b = 0; b < nb; ++b) s += src[b * bstride + r * ld + c];
  const int64_t od = transpose ? (int64_t)c * ldd + r : (int64_t)r * ldd + c;
  dst[od] += alpha * s;
}
void batch_reduce(double* dst, const double* src, int64_t nb, int64_t bstride, int rows, int cols, int64_t ld,
                  int64_t ldd, bool transpose, double alpha, hipStream_t s) {
  const int64_t total = (int64_t)rows * cols;
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, dst, src, nb, bstride, rows,
                     cols, ld, ldd, transpose ? 1 : 0, alpha);
  DCSD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Ladder: amplitude stack.  Row r of the stack is a Vu x Vu matrix over the
// union virtual space [t, u, virt] (spatial orbitals nc..n-1).  Row order:
// [ab (o0*o1) | aa pairs i<j | bb pairs i<j | ab transposed (o0*o1)].
// Virtual index of spin s at union position u, or -1 if u is not virtual for s.
__device__ inline int union_to_vir(const SpinLayout& L, int s, int u) {
  const int sp = L.nc + u;
  if (L.swap_tu) {
    if (sp == L.nc + s) return -1;  // t for alpha, u for beta: occupied
    return u >= 2 ? u - 1 : 0;
  }
  const int a = sp - L.o[s];
  return a >= 0 ? a : -1;
}

__global__ void ladder_stack_kernel(double* S, const double* t2aa, const double* t2bb, const double* t2ab,
                                    const int* pair_i, const int* pair_j, SpinLayout L, int vu, int64_t rows) {
  const int64_t vu2 = (int64_t)vu * vu;
  const int64_t total = rows * vu2;
  const int o0 = L.o[0], o1 = L.o[1], v0 = L.v[0], v1 = L.v[1];
  const int64_t oab = (int64_t)o0 * o1;
  const int64_t np0 = (int64_t)o0 * (o0 - 1) / 2, np1 = (int64_t)o1 * (o1 - 1) / 2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / vu2;
    const int cu = (int)((idx % vu2) / vu), du = (int)(idx % vu);
    double val = 0.0;
    if (r < oab) {  // ab: tau[c,d] = t2ab[i,J,c(alpha), D(beta)]
      const int c = union_to_vir(L, 0, cu), d = union_to_vir(L, 1, du);
      if (c >= 0 && d >= 0) val = t2ab[(r * v0 + c) * v1 + d];
    } else if (r < oab + np0) {
      const int64_t q = r - oab;
      const int c = union_to_vir(L, 0, cu), d = union_to_vir(L, 0, du);
      if (c >= 0 && d >= 0) val = t2aa[(((int64_t)pair_i[q] * o0 + pair_j[q]) * v0 + c) * v0 + d];
    } else if (r < oab + np0 + np1) {
      const int64_t q = r - oab - np0;
      const int c = union_to_vir(L, 1, cu), d = union_to_vir(L, 1, du);
      if (c >= 0 && d >= 0) val = t2bb[(((int64_t)pair_i[np0 + q] * o1 + pair_j[np0 + q]) * v1 + c) * v1 + d];
    } else {  // ab transposed: tau^T[c,d] = tau[d,c]
      const int64_t q = r - oab - np0 - np1;
      const int c = union_to_vir(L, 0, du), d = union_to_vir(L, 1, cu);
      if (c >= 0 && d >= 0) val = t2ab[(q * v0 + c) * v1 + d];
    }
    S[idx] = val;
  }
}
void ladder_stack(double* S, const double* t2aa, const double* t2bb, const double* t2ab, const int* pair_i,
                  const int* pair_j, const SpinLayout& L, int vu, int64_t rows, hipStream_t s) {
  const int64_t total = rows * (int64_t)vu * vu;
  hipLaunchKernelGGL(ladder_stack_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, S, t2aa, t2bb, t2ab, pair_i,
                     pair_j, L, vu, rows);
  DCSD_CHECK_LAUNCH();
}

// Scatter one batch result Rb[row][pl*nq + ql] into Rp[row'][p][q] (n x n per row).
__global__ void ladder_scatter_kernel(double* Rp, const double* Rb, int64_t rows_used, int64_t nrow_main,
                                      int64_t nsame_begin, int n, int p0, int np, int q0, int nq, int diag) {
  const int64_t npq = (int64_t)np * nq;
  const int64_t total = rows_used * npq;
  const int64_t n2 = (int64_t)n * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / npq;
    const int pl = (int)((idx % npq) / nq), ql = (int)(idx % nq);
    const int p = p0 + pl, q = q0 + ql;
    const double val = Rb[idx];
    if (r < nrow_main) {
      Rp[r * n2 + (int64_t)p * n + q] = val;
      if (!diag && r >= nsame_begin) Rp[r * n2 + (int64_t)q * n + p] = -val;
    } else {
      Rp[(r - nrow_main) * n2 + (int64_t)q * n + p] = val;  // ab transposed rows
    }
  }
}
void ladder_scatter(double* Rp, const double* Rb, int64_t rows_used, int64_t nrow_main, int64_t nsame_begin, int n,
                    int p0, int np, int q0, int nq, bool diag, hipStream_t s) {
  const int64_t total = rows_used * (int64_t)np * nq;
  hipLaunchKernelGGL(ladder_scatter_kernel, dim3(nblocks(total, 256)), dim3(256), 0, s, Rp, Rb, rows_used, nrow_main,
                     nsame_begin, n, p0, np, q0, nq, diag ? 1 : 0);
  DCSD_CHECK_LAUNCH();
}

// T1 back-transformation of the spatial ladder result (the dressed vv block is
// B_vv - t1^T B_ov, so (ac|bd)~ = sum_pq M_ap M_bq (pc|qd)):
//   step 1: S[row][p][b] = Rp[row][p][vir(b)] - sum_l t1[l,b] Rp[row][p][occ(l)]   (second-index spin)
//   step 2: out[row][a][b] = S[row][vir(a)][b] - sum_k t1[k,a] S[row][occ(k)][b]   (first-index spin)
// S rows hold n x vm entries, vm = max(v0, v1).
__device__ inline void row_spins(int64_t r, int64_t oab, int64_t np0, int& s1, int& s2) {
  if (r < oab) { s1 = 0; s2 = 1; }
  else if (r < oab + np0) { s1 = 0; s2 = 0; }
  else { s1 = 1; s2 = 1; }
}
__global__ void ladder_mt1_kernel(double* S, const double* Rp, const double* t1a, const double* t1b, int64_t rows,
                                  SpinLayout L) {
  const int n = L.n, vm = L.v[0] > L.v[1] ? L.v[0] : L.v[1];
  const int64_t total = rows * n * vm;
  const int64_t n2 = (int64_t)n * n;
  const int64_t oab = (int64_t)L.o[0] * L.o[1], np0 = (int64_t)L.o[0] * (L.o[0] - 1) / 2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / ((int64_t)n * vm);
    const int p = (int)((idx / vm) % n), b = (int)(idx % vm);
    int s1, s2;
    row_spins(r, oab, np0, s1, s2);
    const int v = L.v[s2], o = L.o[s2];
    if (b >= v) continue;
    const double* t1 = s2 == 0 ? t1a : t1b;
    const double* row = Rp + r * n2 + (int64_t)p * n;
    double val = row[L.vir(s2, b)];
    for (int l = 0; l < o; ++l) val -= t1[l * v + b] * row[L.occ(s2, l)];
    S[idx] = val;
  }
}
__global__ void ladder_mt2_kernel(double* R2aa, double* R2bb, double* R2ab, const double* S, const double* t1a,
                                  const double* t1b, const int* pair_i, const int* pair_j, int64_t rows,
                                  SpinLayout L) {
  const int n = L.n, vm = L.v[0] > L.v[1] ? L.v[0] : L.v[1];
  const int64_t total = rows * vm * vm;
  const int64_t oab = (int64_t)L.o[0] * L.o[1], np0 = (int64_t)L.o[0] * (L.o[0] - 1) / 2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / ((int64_t)vm * vm);
    const int a = (int)((idx / vm) % vm), b = (int)(idx % vm);
    int s1, s2;
    row_spins(r, oab, np0, s1, s2);
    const int va = L.v[s1], vb = L.v[s2], o = L.o[s1];
    if (a >= va || b >= vb) continue;
    const double* t1 = s1 == 0 ? t1a : t1b;
    const double* Sr = S + r * (int64_t)n * vm;
    double val = Sr[(int64_t)L.vir(s1, a) * vm + b];
    for (int k = 0; k < o; ++k) val -= t1[k * va + a] * Sr[(int64_t)L.occ(s1, k) * vm + b];
    if (r < oab) {
      R2ab[(r * va + a) * vb + b] += val;
    } else {
      const int64_t q = r - oab;  // pair index in the combined alpha-then-beta list
      double* R2 = r < oab + np0 ? R2aa : R2bb;
      const int i = pair_i[q], j = pair_j[q];
      R2[((((int64_t)i * o + j) * va) + a) * va + b] += val;
      R2[((((int64_t)j * o + i) * va) + a) * va + b] -= val;
    }
  }
}
void ladder_mt1(double* S, const double* Rp, const double* t1a, const double* t1b, int64_t rows, int64_t o2,
                int64_t npair, int n, int nc, int o, int v, hipStream_t s) {
  (void)o2;
  (void)npair;
  SpinLayout L;
  L.nc = nc;
  L.n = n;
  L.o[0] = L.o[1] = o;
  L.v[0] = L.v[1] = v;
  hipLaunchKernelGGL(ladder_mt1_kernel, dim3(nblocks(rows * n * v, 256)), dim3(256), 0, s, S, Rp, t1a, t1b, rows, L);
  DCSD_CHECK_LAUNCH();
}
void ladder_mtransform(double* R2aa, double* R2bb, double* R2ab, double* S, const double* Rp, const double* t1a,
                       const double* t1b, const int* pair_i, const int* pair_j, int64_t rows, const SpinLayout& L,
                       hipStream_t s) {
  const int vm = L.v[0] > L.v[1] ? L.v[0] : L.v[1];
  const int64_t t1tot = rows * L.n * vm;
  hipLaunchKernelGGL(ladder_mt1_kernel, dim3(nblocks(t1tot, 256)), dim3(256), 0, s, S, Rp, t1a, t1b, rows, L);
  DCSD_CHECK_LAUNCH();
  const int64_t t2tot = rows * (int64_t)vm * vm;
  hipLaunchKernelGGL(ladder_mt2_kernel, dim3(nblocks(t2tot, 256)), dim3(256), 0, s, R2aa, R2bb, R2ab, S, t1a, t1b,
                     pair_i, pair_j, rows, L);
  DCSD_CHECK_LAUNCH();
}

// Jacobi step with orbital-energy denominators from the diagonal of the
// reference Fock matrix (spin order): Tn = T + R / (D - shift), e = Tn - T.
// <pq||pq> for spin-orbitals p, q (spin, spatial): J_pq - [same spin] K_pq.
__device__ inline double pq_pq(const double* J, const double* K, int n, int sp, int p, int sq, int q) {
  return J[(int64_t)p * n + q] - (sp == sq ? K[(int64_t)p * n + q] : 0.0);
}

__global__ void jacobi_kernel(double* Tn, double* E, const double* T, const double* R, const double* fa,
                              const double* fb, const double* J, const double* K, SpinLayout L, double shift) {
  const int n = L.n;
  const int64_t t1end = L.t2_off(0), total = L.total();
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    double D;
    if (x < t1end) {
      const int sp = x < L.ov(0) ? 0 : 1;
      const int64_t y = x - L.t1_off(sp);
      const int v = L.v[sp], o = L.o[sp];
      const double* f = sp ? fb : fa;
      const int i = (int)(y / v), a = (int)(y % v);
      D = f[(int64_t)i * n + i] - f[(int64_t)(o + a) * n + o + a];
      if (J) D += pq_pq(J, K, n, sp, L.occ(sp, i), sp, L.vir(sp, a));  // D - s, s = -<ia||ia>
    } else {
      const int blk = x < L.t2_off(1) ? 0 : (x < L.t2_off(2) ? 1 : 2);
      const int si = blk == 1 ? 1 : 0, sj = blk == 0 ? 0 : 1;
      int64_t r = x - L.t2_off(blk);
      const int vi = L.v[si], vj = L.v[sj], oi = L.o[si], oj = L.o[sj];
      const int b = (int)(r % vj); r /= vj;
      const int a = (int)(r % vi); r /= vi;
      const int j = (int)(r % oj);
      const int i = (int)(r / oj);
      const double* fi = si ? fb : fa;
      const double* fj = sj ? fb : fa;
      D = fi[(int64_t)i * n + i] + fj[(int64_t)j * n + j] - fi[(int64_t)(oi + a) * n + oi + a] -
          fj[(int64_t)(oj + b) * n + oj + b];
      if (J) {
        const int pi = L.occ(si, i), pj = L.occ(sj, j), pa = L.vir(si, a), pb = L.vir(sj, b);
        const double sEN = pq_pq(J, K, n, si, pa, sj, pb) + pq_pq(J, K, n, si, pi, sj, pj) -
                           pq_pq(J, K, n, si, pi, si, pa) - pq_pq(J, K, n, si, pi, sj, pb) -
                           pq_pq(J, K, n, sj, pj, si, pa) - pq_pq(J, K, n, sj, pj, sj, pb);
        D -= sEN;
      }
    }
    // R = 0 exactly (the A->B double, whose Epstein-Nesbet denominator also
    // vanishes): no step
    const double step = R[x] == 0.0 ? 0.0 : R[x] / (D - shift);
    Tn[x] = T[x] + step;
    if (E) E[x] = step;
  }
}
void jacobi(double* Tn, double* E, const double* T, const double* R, const double* fa, const double* fb,
            const double* J, const double* K, const SpinLayout& L, double shift, hipStream_t s) {
  hipLaunchKernelGGL(jacobi_kernel, dim3(nblocks(L.total(), 256)), dim3(256), 0, s, Tn, E, T, R, fa, fb, J, K, L,
                     shift);
  DCSD_CHECK_LAUNCH();
}

// K[pq] = sum_P B[P][pq]^2 (exchange integrals (pq|qp) of a symmetric factor).
__global__ void sumsq_kernel(double* K, const double* B, int64_t nb, int64_t n2) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n2) return;
  double s = 0.0;
  for (int64_t P = 0; P < nb; ++P) {
    const double b = B[P * n2 + idx];
    s += b * b;
  }
  K[idx] = s;
}
void sumsq_batch(double* K, const double* B, int64_t nb, int64_t n2, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(nblocks(n2, 256)), dim3(256), 0, s, K, B, nb, n2);
  DCSD_CHECK_LAUNCH();
}

// T = sum_i c_i V_i (DIIS extrapolation; c on the device).
__global__ void combine_kernel(double* T, const double* V, int64_t stride, const double* c, int m, int64_t n) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += c[i] * V[i * stride + x];
    T[x] = s;
  }
}
void combine(double* T, const double* V, int64_t stride, const double* c, int m, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, T, V, stride, c, m, n);
  DCSD_CHECK_LAUNCH();
}

}  // namespace dcsd

namespace dcsd {
// dst[P][p][q] = src[P][pi(p)][pi(q)] with pi exchanging orbitals nc (t) and nc+1 (u).
__global__ void swap_tu_kernel(double* dst, const double* src, int64_t batch, int n, int nc) {
  const int64_t n2 = (int64_t)n * n, total = batch * n2;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t P = idx / n2;
    int p = (int)((idx % n2) / n), q = (int)(idx % n);
    p = p == nc ? nc + 1 : (p == nc + 1 ? nc : p);
    q = q == nc ? nc + 1 : (q == nc + 1 ? nc : q);
    dst[idx] = src[P * n2 + (int64_t)p * n + q];
  }
}
void swap_tu(double* dst, const double* src, int64_t batch, int n, int nc, hipStream_t s) {
  const int64_t total = batch * (int64_t)n * n;
  int64_t b = (total + 255) / 256;
  if (b > 1 << 20) b = 1 << 20;
  hipLaunchKernelGGL(swap_tu_kernel, dim3((unsigned)b), dim3(256), 0, s, dst, src, batch, n, nc);
  DCSD_CHECK_LAUNCH();
}
// ---------------------------------------------------------------------------
// Strided copy dst[od] = alpha * src[os] + beta * dst[od] over an index box of up to
// six dimensions (od, os: sums of index times stride).  Two kernels, both HBM-bound:
//  * rows: a workgroup per row of the box (or per few rows, when rows are short), the
//    row being every dimension but one (`in`), its offsets decomposed once per row;
//    the threads run along `in`.  Used when the destination and the source have their
//    unit stride in the same dimension (both accesses coalesced).
//  * tiles: the destination's unit-stride dimension a and the source's b are tiled
//    32 x 32 through LDS, so that both the reads (along b) and the writes (along a)
//    are coalesced; a workgroup per tile and per index of the remaining dimensions.
struct CopyPlan {
  int nd;
  int64_t dims[6], ds[6], ss[6];
};

// offsets of index `r` of the box with dimensions `skip0` and `skip1` removed
__device__ inline void copy_outer(const CopyPlan& p, int64_t r, int skip0, int skip1, int64_t& od, int64_t& os) {
  od = 0;
  os = 0;
  for (int d = p.nd - 1; d >= 0; --d) {
    if (d == skip0 || d == skip1) continue;
    const int64_t i = r % p.dims[d];
    r /= p.dims[d];
    od += i * p.ds[d];
    os += i * p.ss[d];
  }
}

// A workgroup takes rpb consecutive rows (rpb > 1 only for rows of at most 2048 elements), their
// offsets decomposed once each into LDS; the threads run over the rpb x n elements.
constexpr int kCopyMaxRows = 64;
__global__ __launch_bounds__(256) void copy_rows_kernel(double* dst, const double* src, CopyPlan p, int in,
                                                        int64_t rows, int rpb, double alpha, double beta) {
  __shared__ int64_t rod[kCopyMaxRows], ros[kCopyMaxRows];
  const int64_t n = p.dims[in], sd = p.ds[in], ss = p.ss[in];
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int nr = rows - r0 < rpb ? (int)(rows - r0) : rpb;
  if ((int)threadIdx.x < nr) copy_outer(p, r0 + threadIdx.x, in, -1, rod[threadIdx.x], ros[threadIdx.x]);
  __syncthreads();
  if (rpb == 1) {
    const int64_t od = rod[0], os = ros[0];
    for (int64_t i = threadIdx.x; i < n; i += 256) {
      double v = alpha * src[os + i * ss];
      if (beta != 0.0) v += beta * dst[od + i * sd];
      dst[od + i * sd] = v;
    }
    return;
  }
  const unsigned un = (unsigned)n, total = (unsigned)nr * un;
  for (unsigned e = threadIdx.x; e < total; e += 256) {
    const unsigned r = e / un, i = e - r * un;
    const int64_t o = rod[r] + (int64_t)i * sd;
    double v = alpha * src[ros[r] + (int64_t)i * ss];
    if (beta != 0.0) v += beta * dst[o];
    dst[o] = v;
  }
}

__global__ __launch_bounds__(256) void copy_tiles_kernel(double* dst, const double* src, CopyPlan p, int a, int b,
                                                         double alpha, double beta) {
  __shared__ double t[32][33];
  const int64_t na = p.dims[a], nb = p.dims[b];
  const int64_t ta = (na + 31) / 32, tb = (nb + 31) / 32;
  const int64_t bid = blockIdx.x;
  const int64_t ia0 = (bid % ta) * 32, ib0 = ((bid / ta) % tb) * 32;
  int64_t od, os;
  copy_outer(p, bid / (ta * tb), a, b, od, os);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // read along b (the source's unit stride)
  for (int r = ty; r < 32; r += 8) {
    const int64_t ia = ia0 + r, ib = ib0 + tx;
    if (ia < na && ib < nb) t[r][tx] = src[os + ia * p.ss[a] + ib * p.ss[b]];
  }
  __syncthreads();
  // write along a (the destination's unit stride)
  for (int r = ty; r < 32; r += 8) {
    const int64_t ia = ia0 + tx, ib = ib0 + r;
    if (ia < na && ib < nb) {
      const int64_t o = od + ia * p.ds[a] + ib * p.ds[b];
      double v = alpha * t[tx][r];
      if (beta != 0.0) v += beta * dst[o];
      dst[o] = v;
    }
  }
}

void strided_copy(double* dst, const double* src, const Strided& st, double alpha, double beta,
                  hipStream_t s) {
  if (st.nd < 1 || st.nd > 6) throw ArgError("strided_copy: 1 to 6 dimensions");
  CopyPlan p{};
  p.nd = st.nd;
  int64_t total = 1;
  for (int d = 0; d < st.nd; ++d) {
    p.dims[d] = st.dims[d];
    p.ds[d] = st.ds[d];
    p.ss[d] = st.ss[d];
    total *= st.dims[d];
  }
  if (total <= 0) return;
  // the destination's and the source's unit-stride dimensions (the last, if none)
  int a = st.nd - 1, b = -1;
  for (int d = st.nd - 1; d >= 0; --d)
    if (st.ds[d] == 1) {
      a = d;
      break;
    }
  for (int d = st.nd - 1; d >= 0; --d)
    if (st.ss[d] == 1) {
      b = d;
      break;
    }
  if (b >= 0 && b != a && st.dims[a] >= 16 && st.dims[b] >= 16) {
    const int64_t tiles = ((st.dims[a] + 31) / 32) * ((st.dims[b] + 31) / 32) * (total / (st.dims[a] * st.dims[b]));
    if (tiles >= ((int64_t)1 << 31)) throw ArgError("strided_copy: box too large");
    hipLaunchKernelGGL(copy_tiles_kernel, dim3((unsigned)tiles), dim3(256), 0, s, dst, src, p, a, b, alpha, beta);
  } else {
    // a short unit-stride dimension would leave most of each workgroup idle: run the rows
    // along the longest dimension instead
    int in = a;
    if (st.dims[a] < 32)
      for (int d = 0; d < st.nd; ++d)
        if (st.dims[d] > st.dims[in]) in = d;
    const int64_t rows = total / st.dims[in];
    const int rpb = st.dims[in] > 2048 ? 1 : (int)std::min<int64_t>(kCopyMaxRows, std::max<int64_t>(1, 2048 / st.dims[in]));
    const int64_t blocks = (rows + rpb - 1) / rpb;
    if (blocks >= ((int64_t)1 << 31)) throw ArgError("strided_copy: box too large");
    hipLaunchKernelGGL(copy_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, p, in, rows, rpb, alpha,
                       beta);
  }
  DCSD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Left factor of the T1 dressing of a batch of n x n matrices X (slice stride n2),
// X <- (1 - t1^T) X with t1 an o x v block (rows/cols 0..o-1 occupied, o..n-1 virtual):
//   X[o+a][j] -= sum_i t1[i][a] X[i][j]   (a < v, every column j)
// One HBM stream over the virtual rows; the sum runs in ascending i with fused
// multiply-adds (the order of the MFMA product it replaces, so results are bitwise equal).
constexpr int kDressMaxO = 32;

__global__ __launch_bounds__(256) void dress_left_kernel(double* X, const double* t1, int n, int o, int v, int64_t n2,
                                                         int row_blocks) {
  __shared__ double ts[kDressMaxO][32];
  double* S = X + (int64_t)(blockIdx.x / row_blocks) * n2;
  const int a0 = (int)(blockIdx.x % row_blocks) * 32;
  const int na = v - a0 < 32 ? v - a0 : 32;
  for (int e = threadIdx.x; e < o * 32; e += 256) {
    const int i = e >> 5, cc = e & 31;
    ts[i][cc] = cc < na ? t1[(int64_t)i * v + a0 + cc] : 0.0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += 256) {
    double top[kDressMaxO];
#pragma unroll
    for (int i = 0; i < kDressMaxO; ++i) top[i] = i < o ? S[(int64_t)i * n + j] : 0.0;
#pragma unroll 8
    for (int a = 0; a < na; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < kDressMaxO; ++i)
        if (i < o) acc = __builtin_fma(ts[i][a], top[i], acc);
      double* p = S + (int64_t)(o + a0 + a) * n + j;
      *p = *p - acc;
    }
  }
}

bool dress_left(double* X, const double* t1, int n, int o, int v, int64_t n2, int64_t batch, hipStream_t s) {
  if (o < 1 || o > kDressMaxO || batch <= 0) return false;
  const int lb = (v + 31) / 32;
  if (batch * lb >= ((int64_t)1 << 31)) return false;
  hipLaunchKernelGGL(dress_left_kernel, dim3((unsigned)(batch * lb)), dim3(256), 0, s, X, t1, n, o, v, n2, lb);
  DCSD_CHECK_LAUNCH();
  return true;
}

}  // namespace dcsd
