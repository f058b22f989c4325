// Coupling between the two reference determinants: R_x -= K_x * W.
//
// K_x = <A^x| e^{-T_A} e^{T_B} |B>, T_B the spin flip of T_A (Theory
// section: the renormalisation term M_x W of the singles and doubles
// equations, with M_x = -K_x; the internal-single products of the
// incomplete-active-space case are included, and terms with a repeated
// spin-orbital cannot occur in exact fermion algebra).
//
//   K_x = sum_{y subset of x} <A^x| e^{-T_A} |A^y> c_B(y),   c_B(y) = <A^y| e^{T_B} |B>,
//
// with the closed-form single and double terms of e^{-T_A}, and each CI
// coefficient c_B from the cluster expansion of e^{T_B} over the (at most
// four) holes and particles that separate A^y from B:
//   C = sum_sigma sgn(sigma) sum_matchings prod t1_B(h_k -> p_sigma(k)) prod 1/2 t2_B(...).
//
// Which amplitude products appear, and with which signs, depends only on
// which indices of x are the open-shell orbitals t, u (the "pattern"), not
// on the values of the core and virtual indices.  The host therefore
// expands every pattern once (dcsd_init) into a table of terms
//   coef * prod_f amplitude_f(i, j, a, b),
// fermion signs from occupation bitmasks over the <= 8 spin-orbitals
// involved; the device evaluates one pattern's table for all of its
// elements with a uniform instruction stream.
#include <algorithm>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "coupling_terms.h"
#include "kernels.h"

namespace dcsd {

namespace {

using namespace cpl;

// ---- device evaluation --------------------------------------------------------
struct Amp {
  const double* t1[2];
  const double* t2[3];
  int nc, o, v;
};

__device__ inline int slot_val(int slot, int i, int j, int a, int b) {
  return slot == 0 ? i : (slot == 1 ? j : (slot == 2 ? a : b));
}
__device__ inline int occ_pos(int kind, int idx, int nc) { return kind == CORE ? idx : nc; }
__device__ inline int vir_pos(int kind, int idx) { return kind == VIRT ? 1 + idx : 0; }

__device__ inline double factor(const Amp& A, const DFac& f, int i, int j, int a, int b) {
  if (f.type == 1) {
    const int h = occ_pos(f.kind[0], slot_val(f.slot[0], i, j, a, b), A.nc);
    const int p = vir_pos(f.kind[1], slot_val(f.slot[1], i, j, a, b));
    return A.t1[f.blk][h * A.v + p];
  }
  const int h1 = occ_pos(f.kind[0], slot_val(f.slot[0], i, j, a, b), A.nc);
  const int h2 = occ_pos(f.kind[1], slot_val(f.slot[1], i, j, a, b), A.nc);
  const int p1 = vir_pos(f.kind[2], slot_val(f.slot[2], i, j, a, b));
  const int p2 = vir_pos(f.kind[3], slot_val(f.slot[3], i, j, a, b));
  return A.t2[f.blk][(((int64_t)h1 * A.o + h2) * A.v + p1) * A.v + p2];
}

// Compile-time tables (generated at build time from the same expansion):
// Fixed<P> holds pattern P's distinct factors and its terms over them.
#include "coupling_tables.inc"

// p -> (lo, hi), lo < hi < n, enumerating the pairs row by row (hi fastest)
__device__ inline void tri_pair(int64_t p, int n, int& lo, int& hi) {
  const auto start = [n](int64_t r) { return r * (2 * (int64_t)n - r - 1) / 2; };
  const double b = 2.0 * n - 1.0;
  int64_t r = (int64_t)((b - sqrt(fmax(b * b - 8.0 * (double)p, 0.0))) * 0.5);
  r = r < 0 ? 0 : (r > n - 2 ? n - 2 : r);
  while (r > 0 && start(r) > p) --r;
  while (r < n - 2 && start(r + 1) <= p) ++r;
  lo = (int)r;
  hi = (int)(r + 1 + (p - start(r)));
}

// Element count of a pattern launch: equal-spin doubles with two core (two
// virtual) indices take i < j (a < b) only and write the antisymmetric copies.
template <class F>
__host__ __device__ inline void pair_counts(const PatternLaunch& pl, int64_t& nij, int64_t& nab) {
  constexpr bool same = F::block == 2 || F::block == 3;
  constexpr bool tri_ij = same && F::kind[0] == CORE && F::kind[1] == CORE;
  constexpr bool tri_ab = same && F::kind[2] == VIRT && F::kind[3] == VIRT;
  nij = tri_ij ? (int64_t)pl.cnt[0] * (pl.cnt[0] - 1) / 2 : (int64_t)pl.cnt[0] * pl.cnt[1];
  nab = tri_ab ? (int64_t)pl.cnt[2] * (pl.cnt[2] - 1) / 2 : (int64_t)pl.cnt[2] * pl.cnt[3];
}

// One pattern, one thread per element (i, j, a, b) (core and virtual indices
// 0-based): every distinct factor is loaded once, then the terms are summed
// with indices known at compile time.
template <int P>
__global__ __launch_bounds__(256) void coupling_fixed(PatternLaunch pl, Amp A, double* __restrict__ R,
                                                      const double* __restrict__ Wp) {
  using F = Fixed<P>;
  constexpr bool same = F::block == 2 || F::block == 3;
  constexpr bool tri_ij = same && F::kind[0] == CORE && F::kind[1] == CORE;
  constexpr bool tri_ab = same && F::kind[2] == VIRT && F::kind[3] == VIRT;
  int64_t nij, nab;
  pair_counts<F>(pl, nij, nab);
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= nij * nab) return;
  const int64_t pij = id / nab, pab = id % nab;
  int ii, jj, aa, bb;
  if (tri_ij) {
    tri_pair(pij, pl.cnt[0], ii, jj);
  } else {
    ii = (int)(pij / pl.cnt[1]);
    jj = (int)(pij % pl.cnt[1]);
  }
  if (tri_ab) {
    tri_pair(pab, pl.cnt[2], aa, bb);
  } else {
    aa = (int)(pab / pl.cnt[3]);
    bb = (int)(pab % pl.cnt[3]);
  }
  double fv[F::ND];
#pragma unroll
  for (int f = 0; f < F::ND; ++f) fv[f] = factor(A, F::fac[f], ii, jj, aa, bb);
  double K = 0.0;
#pragma unroll
  for (int t = 0; t < F::NT; ++t) {
    double v = F::term[t].coef;
#pragma unroll
    for (int q = 0; q < MAXF; ++q)
      if (q < F::term[t].nf) v *= fv[F::term[t].idx[q]];
    K += v;
  }
  const double KW = K * (*Wp);
  const int nc = A.nc, o = A.o, v = A.v;
  const int64_t ov = (int64_t)o * v, s2 = ov * ov;
  const int i = occ_pos(F::kind[0], ii, nc), a = vir_pos(F::kind[2], aa);
  if (F::block < 2) {
    R[F::block * ov + (int64_t)i * v + a] -= KW;
    return;
  }
  const int j = occ_pos(F::kind[1], jj, nc), b = vir_pos(F::kind[3], bb);
  double* Rb = R + 2 * ov + (int64_t)(F::block - 2) * s2;
  auto at = [&](int p, int q, int c, int d) -> double& { return Rb[(((int64_t)p * o + q) * v + c) * v + d]; };
  at(i, j, a, b) -= KW;
  if (same) {
    at(j, i, a, b) += KW;
    at(i, j, b, a) += KW;
    at(j, i, b, a) -= KW;
  }
}

template <int P>
void launch_fixed(const PatternLaunch& pl, const Amp& A, double* R, const double* Wp, hipStream_t s) {
  int64_t nij, nab;
  pair_counts<Fixed<P>>(pl, nij, nab);
  const int64_t tot = nij * nab;
  if (tot <= 0 || Fixed<P>::NT == 0) return;
  hipLaunchKernelGGL(coupling_fixed<P>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, pl, A, R, Wp);
}

// Does pattern P's compile-time table equal the fixed form of these terms?
template <int P>
bool fixed_matches(const PatternLaunch& pl, const DTerm* terms) {
  using F = Fixed<P>;
  if (pl.block != F::block) return false;
  for (int k = 0; k < 4; ++k)
    if (pl.kind[k] != F::kind[k]) return false;
  std::vector<DFac> fac;
  std::vector<FTerm> term;
  fixed_form(terms + pl.term_off, pl.nterms, fac, term);
  if ((int)fac.size() != F::ND || (int)term.size() != F::NT) return false;
  for (int k = 0; k < F::ND; ++k)
    if (!same_factor(fac[k], F::fac[k])) return false;
  for (int t = 0; t < F::NT; ++t)
    if (term[t].coef != F::term[t].coef || term[t].nf != F::term[t].nf ||
        !std::equal(term[t].idx, term[t].idx + term[t].nf, F::term[t].idx))
      return false;
  return true;
}

using FixedLaunch = void (*)(const PatternLaunch&, const Amp&, double*, const double*, hipStream_t);
using FixedMatch = bool (*)(const PatternLaunch&, const DTerm*);
#define DCSD_FIXED_LAUNCH(P) &launch_fixed<P>,
#define DCSD_FIXED_MATCH(P) &fixed_matches<P>,
const FixedLaunch kFixedLaunch[] = {DCSD_FIXED_PATTERNS(DCSD_FIXED_LAUNCH)};
const FixedMatch kFixedMatch[] = {DCSD_FIXED_PATTERNS(DCSD_FIXED_MATCH)};
#undef DCSD_FIXED_LAUNCH
#undef DCSD_FIXED_MATCH

}  // namespace


void coupling_prepare(int nc, int nv, std::vector<char>& launch_blob) {
  std::vector<PatternLaunch> pls;
  std::vector<DTerm> all;
  add_patterns(pls, all, nc, nv);
  // each pattern's compile-time table must be the fixed form of the terms expanded here
  for (PatternLaunch& pl : pls) {
    pl.fixed = -1;
    for (int p = 0; p < kFixedPatterns && pl.fixed < 0; ++p)
      if (kFixedMatch[p](pl, all.data())) pl.fixed = p;
    if (pl.fixed < 0) throw std::runtime_error("coupling: no compile-time table matches a pattern");
  }
  launch_blob.assign((const char*)pls.data(), (const char*)(pls.data() + pls.size()));
}

// Adjoint of one pattern: with rb the cotangent of -K_x W gathered over the
// element's (antisymmetric) copies, Tbar[f] += -W rb dK_x/dT_f (atomic: one
// amplitude enters many elements) and Wbar += -sum_x K_x rb.
__device__ inline int64_t factor_off(const Amp& A, const DFac& f, int i, int j, int a, int b, int& arr) {
  if (f.type == 1) {
    const int h = occ_pos(f.kind[0], slot_val(f.slot[0], i, j, a, b), A.nc);
    const int p = vir_pos(f.kind[1], slot_val(f.slot[1], i, j, a, b));
    arr = f.blk;
    return (int64_t)h * A.v + p;
  }
  const int h1 = occ_pos(f.kind[0], slot_val(f.slot[0], i, j, a, b), A.nc);
  const int h2 = occ_pos(f.kind[1], slot_val(f.slot[1], i, j, a, b), A.nc);
  const int p1 = vir_pos(f.kind[2], slot_val(f.slot[2], i, j, a, b));
  const int p2 = vir_pos(f.kind[3], slot_val(f.slot[3], i, j, a, b));
  arr = 2 + f.blk;
  return (((int64_t)h1 * A.o + h2) * A.v + p1) * A.v + p2;
}
__device__ inline double wave_sum(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
// Adjoint of one pattern with its compile-time table.  Every lane of a wave runs
// the same code (lanes past the end contribute zero), so that a factor whose
// cotangent address is the same in all 64 lanes - every factor that does not
// depend on the indices that vary within the wave, e.g. amplitudes with only
// t/u indices, which all elements of a pattern share - is summed in the wave
// first and added with one atomic instead of 64.  Each distinct factor gets one
// cotangent per element: dK/dfactor summed over the terms that contain it.
template <int P>
__global__ __launch_bounds__(256) void coupling_fixed_adj(PatternLaunch pl, Amp A, double* Tbar,
                                                          const double* __restrict__ Rbar,
                                                          const double* __restrict__ Wp, double* Wbar) {
  using F = Fixed<P>;
  constexpr bool same = F::block == 2 || F::block == 3;
  constexpr bool tri_ij = same && F::kind[0] == CORE && F::kind[1] == CORE;
  constexpr bool tri_ab = same && F::kind[2] == VIRT && F::kind[3] == VIRT;
  int64_t nij, nab;
  pair_counts<F>(pl, nij, nab);
  const int64_t tot = nij * nab;
  const int64_t id0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool inrange = id0 < tot;
  const int64_t id = inrange ? id0 : tot - 1;
  const int64_t pij = id / nab, pab = id % nab;
  int ii, jj, aa, bb;
  if (tri_ij) {
    tri_pair(pij, pl.cnt[0], ii, jj);
  } else {
    ii = (int)(pij / pl.cnt[1]);
    jj = (int)(pij % pl.cnt[1]);
  }
  if (tri_ab) {
    tri_pair(pab, pl.cnt[2], aa, bb);
  } else {
    aa = (int)(pab / pl.cnt[3]);
    bb = (int)(pab % pl.cnt[3]);
  }
  const int nc = A.nc, o = A.o, v = A.v;
  const int64_t ov = (int64_t)o * v, s2 = ov * ov;
  double rb = 0.0;
  if (inrange) {
    const int i = occ_pos(F::kind[0], ii, nc), a = vir_pos(F::kind[2], aa);
    if (F::block < 2) {
      rb = Rbar[F::block * ov + (int64_t)i * v + a];
    } else {
      const int j = occ_pos(F::kind[1], jj, nc), b = vir_pos(F::kind[3], bb);
      const double* Rb = Rbar + 2 * ov + (int64_t)(F::block - 2) * s2;
      auto at = [&](int p, int q, int c, int d) { return Rb[(((int64_t)p * o + q) * v + c) * v + d]; };
      rb = at(i, j, a, b);
      if (same) rb += -at(j, i, a, b) - at(i, j, b, a) + at(j, i, b, a);
    }
  }
  const double g = -(*Wp) * rb;  // cotangent of K_x
  double fv[F::ND], dfv[F::ND];
#pragma unroll
  for (int f = 0; f < F::ND; ++f) {
    fv[f] = factor(A, F::fac[f], ii, jj, aa, bb);
    dfv[f] = 0.0;
  }
  double K = 0.0;
#pragma unroll
  for (int t = 0; t < F::NT; ++t) {
    double prod = F::term[t].coef;
#pragma unroll
    for (int q = 0; q < MAXF; ++q)
      if (q < F::term[t].nf) prod *= fv[F::term[t].idx[q]];
    K += prod;
#pragma unroll
    for (int q = 0; q < MAXF; ++q) {
      if (q >= F::term[t].nf) continue;
      double part = F::term[t].coef;
#pragma unroll
      for (int q2 = 0; q2 < MAXF; ++q2)
        if (q2 < F::term[t].nf && q2 != q) part *= fv[F::term[t].idx[q2]];
      dfv[F::term[t].idx[q]] += part;
    }
  }
  double* bars[5] = {Tbar, Tbar + ov, Tbar + 2 * ov, Tbar + 2 * ov + s2, Tbar + 2 * ov + 2 * s2};
#pragma unroll
  for (int f = 0; f < F::ND; ++f) {
    int arr;
    const int64_t off = factor_off(A, F::fac[f], ii, jj, aa, bb, arr);
    const double val = g * dfv[f];
    const long long key = ((long long)arr << 40) | (long long)off;
    const long long k0 = __shfl(key, 0);
    if (__all(key == k0)) {
      const double sum = wave_sum(val);
      if (__lane_id() == 0 && sum != 0.0) atomicAdd(bars[arr] + off, sum);
    } else if (val != 0.0) {
      atomicAdd(bars[arr] + off, val);
    }
  }
  const double w = wave_sum(-K * rb);
  if (__lane_id() == 0 && w != 0.0) atomicAdd(Wbar, w);
}

template <int P>
void launch_fixed_adj(const PatternLaunch& pl, const Amp& A, double* Tbar, const double* Rbar, const double* Wp,
                      double* Wbar, hipStream_t s) {
  int64_t nij, nab;
  pair_counts<Fixed<P>>(pl, nij, nab);
  const int64_t tot = nij * nab;
  if (tot <= 0 || Fixed<P>::NT == 0) return;
  hipLaunchKernelGGL(coupling_fixed_adj<P>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, pl, A, Tbar, Rbar,
                     Wp, Wbar);
}
using FixedAdjLaunch = void (*)(const PatternLaunch&, const Amp&, double*, const double*, const double*, double*,
                                hipStream_t);
#define DCSD_FIXED_ADJ(P) &launch_fixed_adj<P>,
const FixedAdjLaunch kFixedAdjLaunch[] = {DCSD_FIXED_PATTERNS(DCSD_FIXED_ADJ)};
#undef DCSD_FIXED_ADJ

void coupling_apply_adj(const std::vector<char>& launch_blob, const double* T, double* Tbar, const double* Rbar,
                        const double* W_dev, double* Wbar, int nc, int nv, hipStream_t s) {
  Amp A;
  const int o = nc + 1, v = nv + 1;
  const int64_t ov = (int64_t)o * v, s2 = ov * ov;
  A.nc = nc; A.o = o; A.v = v;
  A.t1[0] = T;
  A.t1[1] = T + ov;
  A.t2[0] = T + 2 * ov;
  A.t2[1] = T + 2 * ov + s2;
  A.t2[2] = T + 2 * ov + 2 * s2;
  const PatternLaunch* pls = (const PatternLaunch*)launch_blob.data();
  const size_t np = launch_blob.size() / sizeof(PatternLaunch);
  for (size_t k = 0; k < np; ++k) {
    const PatternLaunch& pl = pls[k];
    if (pl.fixed < 0 || pl.fixed >= kFixedPatterns) throw std::runtime_error("coupling: pattern without a table");
    kFixedAdjLaunch[pl.fixed](pl, A, Tbar, Rbar, W_dev, Wbar, s);
    DCSD_CHECK_LAUNCH();
  }
}

void coupling_apply(const std::vector<char>& launch_blob, const double* T, double* R, const double* W_dev, int nc,
                    int nv, hipStream_t s) {
  Amp A;
  const int o = nc + 1, v = nv + 1;
  const int64_t ov = (int64_t)o * v, s2 = ov * ov;
  A.nc = nc; A.o = o; A.v = v;
  A.t1[0] = T;
  A.t1[1] = T + ov;
  A.t2[0] = T + 2 * ov;
  A.t2[1] = T + 2 * ov + s2;
  A.t2[2] = T + 2 * ov + 2 * s2;
  const PatternLaunch* pls = (const PatternLaunch*)launch_blob.data();
  const size_t np = launch_blob.size() / sizeof(PatternLaunch);
  for (size_t k = 0; k < np; ++k) {
    const PatternLaunch& pl = pls[k];
    if (pl.fixed < 0 || pl.fixed >= kFixedPatterns) throw std::runtime_error("coupling: pattern without a table");
    kFixedLaunch[pl.fixed](pl, A, R, W_dev, s);
    DCSD_CHECK_LAUNCH();
  }
}

size_t coupling_term_size() { return sizeof(DTerm); }

}  // namespace dcsd
