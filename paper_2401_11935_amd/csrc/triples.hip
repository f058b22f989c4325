// Device kernels of the perturbative triples correction of the M_s = 1
// determinant: spin-orbital unpacking of the amplitudes, integral assembly from
// spatial DF products and the per-triple energy reduction.  The contractions themselves are FP64 MFMA GEMMs (triples.cpp).
//
// Spin-orbital order: occupied [alpha occupied (oa) | beta occupied (ob)],
// virtual [alpha virtual (va) | beta virtual (vb)].  For the M_s = 1
// determinant both spins keep the spatial order, so the occupied spatial index
// of I is I (alpha) or I - oa (beta), and the virtual A sits at spatial
// oa + A (alpha) or ob + A - va (beta).  The integral products run over the
// union of the virtual spaces, U = spatial [ob, n), with alpha virtuals at
// U index (oa - ob) + A and beta virtuals at A - va.
#include "kernels.h"

namespace dcsd {

namespace {

constexpr int TRI_THREADS = 256;
constexpr int TRI_BCHUNK = 16;  // values of b per workgroup of the energy pass

inline unsigned tri_blocks(int64_t total, int threads, int64_t cap = 1 << 20) {
  int64_t b = (total + threads - 1) / threads;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

__device__ inline int vspin(const TriDims& d, int A) { return A >= d.va; }
__device__ inline int vU(const TriDims& d, int A) { return A < d.va ? (d.oa - d.ob) + A : A - d.va; }
__device__ inline int ospin(const TriDims& d, int I) { return I >= d.oa; }
__device__ inline int osp(const TriDims& d, int I) { return I < d.oa ? I : I - d.oa; }

// t2so[I][J][A][B] from the packed blocks (t2aa, t2bb: full squares; t2ab: [i][j][a][b])
__global__ void tri_unpack_t2(double* t2so, const double* T, SpinLayout L, TriDims d) {
  const int64_t nO = d.nO(), nV = d.nV();
  const int64_t total = nO * nO * nV * nV;
  const double* aa = T + L.t2_off(0);
  const double* bb = T + L.t2_off(1);
  const double* ab = T + L.t2_off(2);
  const int64_t oa = d.oa, ob = d.ob, va = d.va, vb = d.vb;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t B = x % nV, A = (x / nV) % nV, J = (x / (nV * nV)) % nO, I = x / (nV * nV * nO);
    const int si = I >= oa, sj = J >= oa, sa = A >= va, sb = B >= va;
    const int64_t i = si ? I - oa : I, j = sj ? J - oa : J, a = sa ? A - va : A, b = sb ? B - va : B;
    double v = 0.0;
    if (si == sj) {
      if (sa == si && sb == si)
        v = si ? bb[((i * ob + j) * vb + a) * vb + b] : aa[((i * oa + j) * va + a) * va + b];
    } else if (sa != sb) {
      // alpha-beta block t_{i alpha, j beta}^{a alpha, b beta} and its antisymmetric images
      const int64_t ia = si ? j : i, jb = si ? i : j, aa_ = sa ? b : a, bb_ = sa ? a : b;
      const double sgn = (si == sa) ? 1.0 : -1.0;
      v = sgn * ab[((ia * ob + jb) * va + aa_) * vb + bb_];
    }
    t2so[x] = v;
  }
}

// t1so[I][A]; Fock diagonals fo[I], fv[A] and f_ov[I][A] from the per-spin Fock matrices
__global__ void tri_unpack_small(double* t1so, double* fo, double* fv, double* fov, const double* T,
                                 const double* fa, const double* fb, SpinLayout L, TriDims d) {
  const int nO = d.nO(), nV = d.nV(), n = d.n;
  const int64_t total = (int64_t)nO * nV;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int I = (int)(x / nV), A = (int)(x % nV);
    const int si = ospin(d, I), sa = vspin(d, A);
    const int i = osp(d, I), a = sa ? A - d.va : A;
    const double* f = si ? fb : fa;
    const int oo = si ? d.ob : d.oa;
    double t = 0.0, g = 0.0;
    if (si == sa) {
      t = T[L.t1_off(si) + (int64_t)i * (si ? d.vb : d.va) + a];
      g = f[(int64_t)i * n + oo + a];
    }
    t1so[x] = t;
    fov[x] = g;
    if (A == 0) fo[I] = f[(int64_t)i * n + i];
    if (I == 0) {
      const double* fs = sa ? fb : fa;
      const int p = (sa ? d.ob : d.oa) + a;
      fv[A] = fs[(int64_t)p * n + p];
    }
  }
}

// Slab X, row tri_row_e(E): <eX||bc> = (eb|Xc)[se = sb][sX = sc] - (ec|Xb)[se = sc][sX = sb]
// from S[(eU, bU)][(x, cU)] = (eb|xc), row length oa * nU
__global__ void tri_vovv(double* I, const double* S, TriDims d) {
  const int64_t nO = d.nO(), nV = d.nV(), nU = d.nU, R = d.slab_rows();
  const int64_t total = nO * nV * nV * nV, ldS = (int64_t)d.oa * nU;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int C = (int)(x % nV), B = (int)((x / nV) % nV), E = (int)((x / (nV * nV)) % nV);
    const int X = (int)(x / (nV * nV * nV));
    const int sx = ospin(d, X), se = vspin(d, E), sb = vspin(d, B), sc = vspin(d, C);
    const int64_t xs = osp(d, X), eU = vU(d, E), bU = vU(d, B), cU = vU(d, C);
    double v = 0.0;
    if (se == sb && sx == sc) v += S[(eU * nU + bU) * ldS + xs * nU + cU];
    if (se == sc && sx == sb) v -= S[(eU * nU + cU) * ldS + xs * nU + bU];
    I[((int64_t)X * R + d.row_e(E)) * nV * nV + (int64_t)B * nV + C] = v;
  }
}

// O[J][K][B][C] = <jk||bc> = (jb|kc)[sj = sb][sk = sc] - (jc|kb)[sj = sc][sk = sb]
// from S2[(j, bU)][(k, cU)] = (jb|kc), row length oa * nU
__global__ void tri_oovv(double* O, const double* S2, TriDims d) {
  const int64_t nO = d.nO(), nV = d.nV(), nU = d.nU;
  const int64_t total = nO * nO * nV * nV, ld = (int64_t)d.oa * nU;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int C = (int)(x % nV), B = (int)((x / nV) % nV), K = (int)((x / (nV * nV)) % nO);
    const int J = (int)(x / (nV * nV * nO));
    const int sj = ospin(d, J), sk = ospin(d, K), sb = vspin(d, B), sc = vspin(d, C);
    const int64_t js = osp(d, J), ks = osp(d, K), bU = vU(d, B), cU = vU(d, C);
    double v = 0.0;
    if (sj == sb && sk == sc) v += S2[(js * nU + bU) * ld + ks * nU + cU];
    if (sj == sc && sk == sb) v -= S2[(js * nU + cU) * ld + ks * nU + bU];
    O[x] = v;
  }
}

// Q[Y][Z][A][M] = <mA||yz> = (my|Az)[sm = sy][sA = sz] - (mz|Ay)[sm = sz][sA = sy]
// from S3[(m, y)][(aU, z)] = (my|az), row length nU * oa
__global__ void tri_ovoo(double* Q, const double* S3, TriDims d) {
  const int64_t nO = d.nO(), nV = d.nV(), oa = d.oa;
  const int64_t total = nO * nO * nV * nO, ld = (int64_t)d.nU * oa;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int M = (int)(x % nO), A = (int)((x / nO) % nV), Z = (int)((x / (nO * nV)) % nO);
    const int Y = (int)(x / (nO * nV * nO));
    const int sm = ospin(d, M), sa = vspin(d, A), sy = ospin(d, Y), sz = ospin(d, Z);
    const int64_t ms = osp(d, M), ys = osp(d, Y), zs = osp(d, Z), aU = vU(d, A);
    double v = 0.0;
    if (sm == sy && sa == sz) v += S3[(ms * oa + ys) * ld + aU * oa + zs];
    if (sm == sz && sa == sy) v -= S3[(ms * oa + zs) * ld + aU * oa + ys];
    Q[x] = v;
  }
}

// A[a][q*n + kk] (row stride lda, kk < n): for a of spin sa, segment q < g.nseg[sa] holds the
// order p = g.p[sa][q] of (i, j, k) -> (x; y z) = (i; j k), (j; i k), (k; j i) with its sign
// (+, -, -) of P(i/jk): over the spin s = s(y) + s(z) - s(a), the columns are t_yz^{a e} over the
// virtuals e of spin s, then -<m a||y z> over the occupied m of spin s (v_s + o_s = n columns),
// matching the slab rows row_e(e), row_m(m) of x.  Every other column is zero.
__global__ void tri_build_a(double* A, int64_t lda, const double* t2so, const double* Q, int i, int j, int k,
                            TriSegs g, TriDims d) {
  const int64_t nO = d.nO(), nV = d.nV(), n = d.n;
  const int64_t total = nV * lda;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = x / lda, col = x - a * lda, q = col / n, kk = col - q * n;
    const int sa = vspin(d, (int)a);
    double v = 0.0;
    if (q < g.nseg[sa]) {
      const int p = g.p[sa][q];
      const int64_t y = p == 0 ? j : (p == 1 ? i : j), z = p == 2 ? i : k;
      const int se = ospin(d, (int)y) + ospin(d, (int)z) - sa;  // 0 or 1 for a listed segment
      const int64_t nve = se ? d.vb : d.va;
      if (kk < nve)
        v = t2so[((y * nO + z) * nV + a) * nV + (se ? d.va : 0) + kk];
      else
        v = -Q[((y * nO + z) * nV + a) * nO + (se ? d.oa : 0) + (kk - nve)];
      if (p != 0) v = -v;
    }
    A[x] = v;
  }
}

// sum over a workgroup of TRI_THREADS threads (one- or two-dimensional), fixed order
__device__ double tri_block_sum(double v, double* sh) {
  const int t = threadIdx.y * blockDim.x + threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = TRI_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Partial sums of one occupied triple (i, j, k) over a < b < c: w = N^c / D, parts w N^c,
// w N^d1, w N^d2 with
//   N^c = Zt[a][b][c] - Zt[b][a][c] - Zt[c][b][a]          (Zt = P(i/jk) of the GEMM sums)
//   N^d = P(i/jk) P(a/bc) [t_i^a <jk||bc> + f_ia t_jk^bc]
// One workgroup per (32 c) x (32 a) tile and chunk of TRI_BCHUNK values of b (grid x, y, z),
// 32 x 8 threads, thread (tx, ty) on c = c0 + tx and the four a = a0 + ty + 8q.  For each b the
// tile Zt[c][b][a] (rows c, contiguous a) and the rows b of the six matrices of the disconnected
// numerator go through LDS, so that all three Zt reads run along their contiguous index; the
// matrix elements at (a, c) and the vectors at a and c, which do not depend on b, stay in
// registers.  part: three doubles per workgroup, in grid order (zeros where the tile holds no
// a < b < c).
__global__ void __launch_bounds__(TRI_THREADS)
tri_energy_tiled(double* part, const double* Zt, const double* t1so, const double* t2so, const double* oovv,
                 const double* fo, const double* fv, const double* fov, int i, int j, int k, TriDims d) {
  __shared__ double s3[32][33];
  __shared__ double sb[2][6][32];  // rows b of the six matrices at columns c0 + u ([0]) and a0 + u ([1])
  __shared__ double sh[TRI_THREADS];
  const int64_t nO = d.nO(), nV = d.nV(), nV2 = nV * nV;
  const int64_t a0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 32 + tx;
  const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const int64_t b0 = (int64_t)blockIdx.z * TRI_BCHUNK;
  const int64_t blo = b0 > a0 + 1 ? b0 : a0 + 1;  // some a < b in the tile
  int64_t bhi = b0 + TRI_BCHUNK < nV ? b0 + TRI_BCHUNK : nV;
  if (bhi > c0 + 31) bhi = c0 + 31;                // some c > b in the tile
  if (blo >= bhi) {                                // uniform over the workgroup
    if (tid == 0) part[3 * blk] = part[3 * blk + 1] = part[3 * blk + 2] = 0.0;
    return;
  }
  // matrices m < 3: <y z||..> of the orders p = m, m >= 3: t_yz of p = m - 3; vectors t1_x, f_x
  const int xs[3] = {i, j, k}, ys[3] = {j, i, j}, zs[3] = {k, k, i};
  const double sg[3] = {1.0, -1.0, -1.0};
  const double* Mx[6];
  const double* vx[6];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    Mx[p] = oovv + ((int64_t)ys[p] * nO + zs[p]) * nV2;
    Mx[3 + p] = t2so + ((int64_t)ys[p] * nO + zs[p]) * nV2;
    vx[p] = t1so + (int64_t)xs[p] * nV;
    vx[3 + p] = fov + (int64_t)xs[p] * nV;
  }
  const double fijk = fo[i] + fo[j] + fo[k];
  const int64_t c = c0 + tx;
  const bool cin = c < nV;
  double mac[4][6], va[4][6], vc[6], fva[4];
#pragma unroll
  for (int m = 0; m < 6; ++m) vc[m] = cin ? vx[m][c] : 0.0;
  const double fvc = cin ? fv[c] : 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t a = a0 + ty + 8 * q;
    const bool ain = a < nV;
    fva[q] = ain ? fv[a] : 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      mac[q][m] = ain && cin ? Mx[m][a * nV + c] : 0.0;
      va[q][m] = ain ? vx[m][a] : 0.0;
    }
  }
  double e4 = 0.0, e5 = 0.0, edt = 0.0;
  for (int64_t b = blo; b < bhi; ++b) {
    double vb[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) vb[m] = vx[m][b];
    const double fvb = fv[b];
    __syncthreads();  // the previous b's reads of s3 and sb are done
    for (int r = ty; r < 32; r += 8) {
      const int64_t cr = c0 + r, a = a0 + tx;
      s3[r][tx] = (cr < nV && a < nV) ? Zt[(cr * nV + b) * nV + a] : 0.0;
    }
    for (int t = tid; t < 2 * 6 * 32; t += TRI_THREADS) {
      const int h = t / 192, m = (t / 32) % 6, u = t % 32;
      const int64_t col = (h ? a0 : c0) + u;
      sb[h][m][u] = col < nV ? Mx[m][b * nV + col] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = ty + 8 * q;
      const int64_t a = a0 + r;
      if (a >= b || c <= b || !cin) continue;
      const double nc = Zt[(a * nV + b) * nV + c] - Zt[(b * nV + a) * nV + c] - s3[tx][r];
      if (nc == 0.0) continue;
      double d1 = 0.0, d2 = 0.0;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        d1 += sg[p] * (va[q][p] * sb[0][p][tx] - vb[p] * mac[q][p] - vc[p] * sb[1][p][r]);
        d2 += sg[p] * (va[q][3 + p] * sb[0][3 + p][tx] - vb[3 + p] * mac[q][3 + p] - vc[3 + p] * sb[1][3 + p][r]);
      }
      const double w = nc / (fijk - fva[q] - fvb - fvc);
      e4 += w * nc;
      e5 += w * d1;
      edt += w * d2;
    }
  }
  e4 = tri_block_sum(e4, sh);
  e5 = tri_block_sum(e5, sh);
  edt = tri_block_sum(edt, sh);
  if (tid == 0) {
    part[3 * blk + 0] = e4;
    part[3 * blk + 1] = e5;
    part[3 * blk + 2] = edt;
  }
}

// out[0..3] = scale * (sum of the partials of each part, and their total); fixed order
__global__ void __launch_bounds__(TRI_THREADS) tri_energy_reduce(double* out, const double* part, int nb,
                                                                 double scale) {
  __shared__ double sh[TRI_THREADS];
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += TRI_THREADS)
    for (int q = 0; q < 3; ++q) s[q] += part[3 * b + q];
  for (int q = 0; q < 3; ++q) s[q] = tri_block_sum(s[q], sh);
  if (threadIdx.x == 0) {
    out[0] = scale * s[0];
    out[1] = scale * s[1];
    out[2] = scale * s[2];
    out[3] = scale * (s[0] + s[1] + s[2]);
  }
}

}  // namespace

void tri_unpack(double* t1so, double* t2so, double* fo, double* fv, double* fov, const double* T, const double* fa,
                const double* fb, const SpinLayout& L, const TriDims& d, hipStream_t s) {
  const int64_t n2 = (int64_t)d.nO() * d.nO() * d.nV() * d.nV();
  hipLaunchKernelGGL(tri_unpack_t2, dim3(tri_blocks(n2, TRI_THREADS)), dim3(TRI_THREADS), 0, s, t2so, T, L, d);
  DCSD_CHECK_LAUNCH();
  const int64_t n1 = (int64_t)d.nO() * d.nV();
  hipLaunchKernelGGL(tri_unpack_small, dim3(tri_blocks(n1, TRI_THREADS)), dim3(TRI_THREADS), 0, s, t1so, fo, fv, fov,
                     T, fa, fb, L, d);
  DCSD_CHECK_LAUNCH();
}

void tri_operand_a(double* A, int64_t lda, const double* t2so, const double* Q, int i, int j, int k, const TriSegs& g,
                   const TriDims& d, hipStream_t s) {
  const int64_t total = (int64_t)d.nV() * lda;
  hipLaunchKernelGGL(tri_build_a, dim3(tri_blocks(total, TRI_THREADS)), dim3(TRI_THREADS), 0, s, A, lda, t2so, Q, i, j,
                     k, g, d);
  DCSD_CHECK_LAUNCH();
}

void tri_assemble_vovv(double* I, const double* S, const TriDims& d, hipStream_t s) {
  const int64_t nV = d.nV(), total = (int64_t)d.nO() * nV * nV * nV;
  hipLaunchKernelGGL(tri_vovv, dim3(tri_blocks(total, TRI_THREADS)), dim3(TRI_THREADS), 0, s, I, S, d);
  DCSD_CHECK_LAUNCH();
}

void tri_assemble_oovv(double* O, const double* S2, const TriDims& d, hipStream_t s) {
  const int64_t total = (int64_t)d.nO() * d.nO() * d.nV() * d.nV();
  hipLaunchKernelGGL(tri_oovv, dim3(tri_blocks(total, TRI_THREADS)), dim3(TRI_THREADS), 0, s, O, S2, d);
  DCSD_CHECK_LAUNCH();
}

void tri_assemble_ovoo(double* Q, const double* S3, const TriDims& d, hipStream_t s) {
  const int64_t total = (int64_t)d.nO() * d.nO() * d.nV() * d.nO();
  hipLaunchKernelGGL(tri_ovoo, dim3(tri_blocks(total, TRI_THREADS)), dim3(TRI_THREADS), 0, s, Q, S3, d);
  DCSD_CHECK_LAUNCH();
}

int64_t tri_energy_blocks(const TriDims& d) {
  const int64_t t = (d.nV() + 31) / 32;
  return t * t * ((d.nV() + TRI_BCHUNK - 1) / TRI_BCHUNK);
}

void tri_energy(double* out4, double* part, const double* Zt, const double* t1so, const double* t2so,
                const double* oovv, const double* fo, const double* fv, const double* fov, int i, int j, int k,
                const TriDims& d, hipStream_t s) {
  const int nV = d.nV();
  const dim3 grid((nV + 31) / 32, (nV + 31) / 32, (nV + TRI_BCHUNK - 1) / TRI_BCHUNK);
  hipLaunchKernelGGL(tri_energy_tiled, grid, dim3(32, TRI_THREADS / 32), 0, s, part, Zt, t1so, t2so, oovv, fo, fv,
                     fov, i, j, k, d);
  DCSD_CHECK_LAUNCH();
  // 1/36 of the sum over all orders of (i, j, k) and (a, b, c) = the sum over i < j < k, a < b < c
  hipLaunchKernelGGL(tri_energy_reduce, dim3(1), dim3(TRI_THREADS), 0, s, out4, part, (int)tri_energy_blocks(d), 1.0);
  DCSD_CHECK_LAUNCH();
}

}  // namespace dcsd
