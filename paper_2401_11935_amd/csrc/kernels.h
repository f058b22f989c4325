// Launchers of the libdcsd device kernels (internal).
#pragma once

#include <algorithm>
#include <vector>

#include "common.h"

namespace dcsd {

// Per-spin orbital spaces of the reference determinant.  In the orbital order
// of spin s the first o[s] orbitals are occupied and the next v[s] virtual.
// swap_tu = 1: Phi_A (alpha order [core, t | u, virt], beta order [core, u |
// t, virt], the beta order exchanging t and u); 0: the M_s = 1 determinant
// Phi_T (both spins in the spatial order, alpha [core, t, u | virt], beta
// [core | t, u, virt]).  Packed amplitudes: [t1a | t1b | t2aa | t2bb | t2ab]
// with blocks (o0,v0), (o1,v1), (o0,o0,v0,v0), (o1,o1,v1,v1), (o0,o1,v0,v1).
struct SpinLayout {
  int nc = 0, n = 0;
  int o[2] = {0, 0}, v[2] = {0, 0};
  int swap_tu = 1;
  __host__ __device__ int64_t ov(int s) const { return (int64_t)o[s] * v[s]; }
  __host__ __device__ int64_t t1_off(int s) const { return s ? ov(0) : 0; }
  __host__ __device__ int64_t t2_size(int b) const {  // 0 aa, 1 bb, 2 ab
    return b == 2 ? ov(0) * ov(1) : ov(b) * ov(b);
  }
  __host__ __device__ int64_t t2_off(int b) const {
    int64_t x = ov(0) + ov(1);
    for (int k = 0; k < b; ++k) x += t2_size(k);
    return x;
  }
  __host__ __device__ int64_t total() const { return t2_off(2) + t2_size(2); }
  // spatial index of occupied i / virtual a of spin s
  __host__ __device__ int occ(int s, int i) const { return swap_tu ? (i < nc ? i : nc + s) : i; }
  __host__ __device__ int vir(int s, int a) const { return swap_tu ? (a > 0 ? nc + 1 + a : nc + 1 - s) : o[s] + a; }
};

void fill(double* p, double v, int64_t n, hipStream_t s);
// X <- (1 - t1^T) X for `batch` n x n matrices (slice stride n2), t1 o x v; false (nothing
// launched) when o is outside the kernel's range
bool dress_left(double* X, const double* t1, int n, int o, int v, int64_t n2, int64_t batch, hipStream_t s);
void axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s);
void swap_tu(double* dst, const double* src, int64_t batch, int n, int nc, hipStream_t s);
// J[P] = sum_{k < oa} Ba[P,k,k] + sum_{k < ob} Bb[P,k,k]
void jvector(double* J, const double* Ba, const double* Bb, int64_t naux, int n, int oa, int ob, hipStream_t s);
void batch_reduce(double* dst, const double* src, int64_t nb, int64_t bstride, int rows, int cols, int64_t ld,
                  int64_t ldd, bool transpose, double alpha, hipStream_t s);

// ladder
// C(m,n) = alpha * sum_{q < nseg} sum_{k < segk} A[m*lda + q*segk + k] * bseg[q][k*ldb + n] + beta * C(m,n),
// C row-major (ldc), on the direct-to-LDS kernel: A K-contiguous (16-byte aligned, lda even; an odd
// K = nseg*segk needs A's column K zero), the bseg n-contiguous (aligned, N and ldb even), at least
// 128 output tiles of 128 x 128.  False (nothing launched) where these conditions fail.
bool gemm_f64_bseg(int64_t M, int64_t N, int64_t segk, int nseg, const double* A, int64_t lda,
                   const double* const* bseg, int64_t ldb, double* C, int64_t ldc, double alpha, double beta,
                   hipStream_t s);
void gemm_f64_pairs(const double* Bl, int64_t ld, int64_t vu, int64_t naux, int64_t p0, int64_t np, int64_t q0,
                    int64_t nq, double* V2, hipStream_t s);
// Stack rows: [ab (o0 o1) | aa pairs i<j (P0) | bb pairs i<j (P1) | ab transposed (o0 o1)], each a
// Vu x Vu matrix over the spatial virtual space [t, u, virt]; pair_i/pair_j list the alpha
// pairs, then the beta pairs.
void ladder_stack(double* S, const double* t2aa, const double* t2bb, const double* t2ab, const int* pair_i,
                  const int* pair_j, const SpinLayout& L, int vu, int64_t rows, hipStream_t s);
void ladder_scatter(double* Rp, const double* Rb, int64_t rows_used, int64_t nrow_main, int64_t nsame_begin, int n,
                    int p0, int np, int q0, int nq, bool diag, hipStream_t s);
// S: work of rows * n * max(v0, v1) doubles
void ladder_mtransform(double* R2aa, double* R2bb, double* R2ab, double* S, const double* Rp, const double* t1a,
                       const double* t1b, const int* pair_i, const int* pair_j, int64_t rows, const SpinLayout& L,
                       hipStream_t s);

// Coupling between the two determinants: R -= K(T) * W (the caller sets R at the A->B double to 0).
// coupling_prepare lists the patterns of the problem's sizes and checks each against its
// compile-time term table (once); coupling_apply launches them.
void coupling_prepare(int nc, int nv, std::vector<char>& launch_blob);
void coupling_apply(const std::vector<char>& launch_blob, const double* T, double* R, const double* W_dev, int nc,
                    int nv, hipStream_t s);

// ---- adjoints (accumulate into the cotangents of the inputs) -------------------------
void swap_tu_adj(double* src_bar, const double* dst_bar, int64_t batch, int n, int nc, hipStream_t s);
void jvector_adj(double* Ba_bar, double* Bb_bar, const double* J_bar, int64_t naux, int n, int o, hipStream_t s);
void batch_reduce_adj(double* src_bar, const double* dst_bar, int64_t nb, int64_t bstride, int rows, int cols,
                      int64_t ld, int64_t ldd, bool transpose, double alpha, hipStream_t s);
void ladder_stack_adj(double* t2aa_bar, double* t2bb_bar, double* t2ab_bar, const double* Sbar, int o, int v, int vu,
                      int npair, hipStream_t s);
void ladder_scatter_adj(double* Rb_bar, const double* Rp_bar, int64_t rows_used, int64_t nrow_main,
                        int64_t nsame_begin, int n, int p0, int np, int q0, int nq, bool diag, hipStream_t s);
void ladder_mt1(double* S, const double* Rp, const double* t1a, const double* t1b, int64_t rows, int64_t o2,
                int64_t npair, int n, int nc, int o, int v, hipStream_t s);
// t1bar may be NULL (amplitude cotangent of the T1 factors not wanted); VB, S,
// Sbar: work arrays of rows*v*v, rows*n*v, rows*n*v doubles.
void ladder_mtransform_adj(double* Rpbar, double* t1bar, const double* R2aa_bar, const double* R2bb_bar,
                           const double* R2ab_bar, const double* Rp, const double* t1a, const double* t1b,
                           const int* pair_i, const int* pair_j, int64_t rows, int64_t o2, int64_t npair, int n,
                           int nc, int o, int v, double* VB, double* S, double* Sbar, hipStream_t s);
void coupling_apply_adj(const std::vector<char>& launch_blob, const double* T, double* Tbar, const double* Rbar,
                        const double* W_dev, double* Wbar, int nc, int nv, hipStream_t s);
// dst = src with the equal-spin doubles blocks antisymmetrised (dst != src)
void antisym_copy(double* dst, const double* src, int o, int v, hipStream_t s);
// out[P][p][q] = (in[P][p][q] + in[P][q][p]) / 2 for batch n x n matrices (out != in)
void symmetrize(double* out, const double* in, int64_t batch, int n, hipStream_t s);
// Ibar, fabar, fbbar may be NULL (only the amplitude cotangent)
void energy_adj(double* Tbar, double* Ibar, double* fabar, double* fbbar, const double* T, const double* Isc,
                const double* fa, const double* fb, const double* Ebar, int o, int v, int n, hipStream_t s);

// reductions (deterministic); `part` needs 1024 doubles
void dot(const double* x, const double* y, int64_t n, double* out_dev, double* part, hipStream_t s);
void maxabs(const double* x, int64_t n, double* out_dev, int* nonfinite_dev, double* part, hipStream_t s);
// Isc: (kc|ld) as the (ov0 + ov1) x (ov0 + ov1) spin-conserving particle-hole matrix
void energy(const double* T, const double* Isc, const double* fa, const double* fb, const SpinLayout& L,
            double* out_dev, double* part, hipStream_t s);
// Jacobi step Tn = T + R/(D - s - shift); J, K (spatial (pp|qq), (pq|qp)) enable the
// Epstein-Nesbet diagonal s (NULL: s = 0).  E (may be NULL) receives Tn - T.
void jacobi(double* Tn, double* E, const double* T, const double* R, const double* fa, const double* fb,
            const double* J, const double* K, const SpinLayout& L, double shift, hipStream_t s);
// ---- low precision: FP32 or BF16 MFMA inputs, FP32 accumulation ---------------------
// Storage element size of a low precision (4 for DCSD_PREC_FP32, 2 for DCSD_PREC_BF16).
size_t lp_size(int precision);
// Leading dimension of low-precision K-contiguous rows: a multiple of 8 elements.
inline int64_t lp_ld(int64_t k) { return (k + 7) / 8 * 8; }
// dst[r*ldd + c] = src[i] - sub[i] (i = r*sr + c*sc; sub may be NULL) rounded (through FP32)
// to the precision, r < rows, c < cols.
void lp_convert(int precision, void* dst, int64_t ldd, const double* src, const double* sub, int64_t rows,
                int64_t cols, int64_t sr, int64_t sc, hipStream_t s);
// C(m,n) = alpha * sum_k A[m*lda + k] B[n*ldb + k] + beta * C(m,n), C in FP64 with the
// GemmArgs c_nc convention.  lda, ldb: multiples of 8; A, B: 16-byte aligned.
// ks > 1 splits K across workgroups; `work` then holds ks*M*N floats.
struct LpGemm {
  int precision = 0;
  int64_t M = 0, N = 0, K = 0;
  const void* A = nullptr;
  int64_t lda = 0;
  const void* B = nullptr;
  int64_t ldb = 0;
  double* C = nullptr;
  int64_t ldc = 0;
  bool c_nc = true;
  double alpha = 1.0, beta = 0.0;
  int ks = 1;
  float* work = nullptr;
  bool k_padded = false;  // every row of A and B holds zeros from K up to a multiple of 8 elements
  bool big_tiles = false; // BF16 split-K: 256 x 256 tiles on eight waves
};
void lp_gemm(const LpGemm& g, hipStream_t s);
// C = alpha A B^T + beta C for M, N <= 16, one batch, A [M][K] and B [N][K] K-contiguous and
// K >= 65536 (long dot products, split over K into `work`); false (nothing launched) otherwise
// Work (doubles) gemm_f64_small needs for g; 0 if g is not a small-output product it takes.
int64_t gemm_f64_small_work(const GemmArgs& g);
bool gemm_f64_small(const GemmArgs& g, double* work, int64_t work_cap, hipStream_t s);
// Pair-blocked ladder integrals V2[(p,q)][c][d] (row stride kp) = sum_P BlT[(p,c)][P] BlT[(q,d)][P]
// for p in [p0, p0+np), q in [q0, q0+nq), in the low precision; BlT rows have stride ldk.
void lp_pairs(int precision, const void* BlT, int64_t ldk, int64_t naux, int64_t vu, int64_t p0, int64_t np,
              int64_t q0, int64_t nq, int64_t kp, void* V2, hipStream_t s);

void sumsq_batch(double* K, const double* B, int64_t nb, int64_t n2, hipStream_t s);
void combine(double* T, const double* V, int64_t stride, const double* c, int m, int64_t n, hipStream_t s);

// ---- perturbative triples of the M_s = 1 determinant (triples.hip) ----------------
// Spin-orbital dimensions: occupied [alpha oa | beta ob], virtual [alpha va | beta vb];
// n spatial orbitals; nU = n - ob, the union of the virtual spaces (spatial [ob, n)).
struct TriDims {
  int oa = 0, ob = 0, va = 0, vb = 0, n = 0, nU = 0;
  __host__ __device__ int nO() const { return oa + ob; }
  __host__ __device__ int nV() const { return va + vb; }
  // Slab of occupied X: nV + nO rows of nV^2, ordered [alpha virtual e | alpha occupied m |
  // beta virtual e | beta occupied m]; rows e hold <eX||bc>, rows m the amplitudes t_Xm^bc.
  __host__ __device__ int slab_rows() const { return va + vb + oa + ob; }
  __host__ __device__ int row_e(int E) const { return E + (E >= va ? oa : 0); }
  __host__ __device__ int row_m(int M) const { return va + M + (M >= oa ? vb : 0); }
};
// t1so[nO][nV], t2so[nO][nO][nV][nV] (antisymmetric), Fock diagonals fo[nO], fv[nV] and f_ov[nO][nV]
void tri_unpack(double* t1so, double* t2so, double* fo, double* fv, double* fov, const double* T, const double* fa,
                const double* fb, const SpinLayout& L, const TriDims& d, hipStream_t s);
// slab rows row_e(E) of every X: <EX||BC> from S[(eU,bU)][(x,cU)] = (eb|xc) (x spatial occupied,
// row length oa*nU)
void tri_assemble_vovv(double* I, const double* S, const TriDims& d, hipStream_t s);
// Orders p of (i, j, k) that contribute to the virtuals a of each spin, in segment order.
struct TriSegs {
  int nseg[2] = {0, 0};
  int p[2][3] = {{0, 0, 0}, {0, 0, 0}};
};
// A[nV][lda]: per virtual a, the signed t2 / -<ma||yz> operands of its spin's orders side by
// side (n columns each), zeros after them (lda >= 3n)
void tri_operand_a(double* A, int64_t lda, const double* t2so, const double* Q, int i, int j, int k, const TriSegs& g,
                   const TriDims& d, hipStream_t s);
// O[J][K][B][C] = <JK||BC> from S2[(j,bU)][(k,cU)] = (jb|kc)
void tri_assemble_oovv(double* O, const double* S2, const TriDims& d, hipStream_t s);
// Q[Y][Z][A][M] = <MA||YZ> from S3[(m,y)][(aU,z)] = (my|az)
void tri_assemble_ovoo(double* Q, const double* S3, const TriDims& d, hipStream_t s);
// workgroups of tri_energy (its work space is 3 doubles per workgroup)
int64_t tri_energy_blocks(const TriDims& d);
// out4 = {E4, E5, EDT, total} of the occupied triple i < j < k (device, 4 doubles) from
// Zt[a][bc] = P(i/jk) of the GEMM sums; part: 3 * tri_energy_blocks(d) doubles
void tri_energy(double* out4, double* part, const double* Zt, const double* t1so, const double* t2so,
                const double* oovv, const double* fo, const double* fv, const double* fov, int i, int j, int k,
                const TriDims& d, hipStream_t s);

}  // namespace dcsd
