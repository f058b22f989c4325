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

#include "kernels.h"

namespace dcsd {

namespace {

enum Kind : int { CORE = 0, KT = 1, KU = 2, VIRT = 3 };

// A spin-orbital of a pattern: spin, kind and (for core/virtual) which index
// of x (0..3 = i, j, a, b) supplies its position.
struct Lo {
  int spin, kind, slot;
  bool operator==(const Lo& o) const { return spin == o.spin && kind == o.kind && slot == o.slot; }
};

bool occA(const Lo& d) { return d.kind == CORE || (d.kind == KT && d.spin == 0) || (d.kind == KU && d.spin == 1); }

// ---- device tables -----------------------------------------------------------
// Factor: a T_A amplitude.  type 1: t1[spin][occ(o0)][vir(o1)];
// type 2: t2[blk][occ(o0)][occ(o1)][vir(o2)][vir(o3)], blk 0 aa, 1 bb, 2 ab.
// Orbital reference: kind (CORE/VIRT use the x index `slot`, KT/KU are fixed).
struct DFac {
  signed char type, blk;
  signed char kind[4];
  signed char slot[4];
};
constexpr int MAXF = 6;
struct DTerm {
  double coef;
  int nf;
  DFac f[MAXF];
};

struct PatternLaunch {
  int block;       // 0 t1a, 1 t1b, 2 t2aa, 3 t2bb, 4 t2ab
  int kind[4];     // kinds of i, j, a, b (j, b unused for singles)
  int cnt[4];      // index range sizes
  int term_off, nterms;
};

// ---- host-side symbolic expansion -------------------------------------------
struct HTerm {
  double coef;
  std::vector<DFac> f;
};

int apply_ops_host(unsigned& mask, const std::vector<std::pair<int, int>>& ops) {
  int sign = 1;
  for (int q = (int)ops.size() - 1; q >= 0; --q) {
    const unsigned bit = 1u << ops[q].second;
    if (__builtin_popcount(mask & (bit - 1u)) & 1) sign = -sign;
    if (ops[q].first) {
      if (mask & bit) return 0;
      mask |= bit;
    } else {
      if (!(mask & bit)) return 0;
      mask ^= bit;
    }
  }
  return sign;
}

// T_A single amplitude (h -> p) as a device factor; false if it vanishes.
bool fac1(const Lo& h, const Lo& p, DFac& f) {
  if (h.spin != p.spin || !occA(h) || occA(p)) return false;
  f = DFac{};
  f.type = 1;
  f.blk = (signed char)h.spin;
  f.kind[0] = (signed char)h.kind; f.slot[0] = (signed char)h.slot;
  f.kind[1] = (signed char)p.kind; f.slot[1] = (signed char)p.slot;
  return true;
}

// T_A double amplitude (h1 h2 -> p1 p2) in the stored block order; returns
// the sign (0 if it vanishes).
int fac2(Lo h1, Lo h2, Lo p1, Lo p2, DFac& f) {
  if (!occA(h1) || !occA(h2) || occA(p1) || occA(p2)) return 0;
  if (h1 == h2 || p1 == p2) return 0;
  int sign = 1, blk;
  if (h1.spin == h2.spin) {
    if (p1.spin != h1.spin || p2.spin != h1.spin) return 0;
    blk = h1.spin;
  } else {
    if (p1.spin == p2.spin) return 0;
    if (h1.spin == 1) { std::swap(h1, h2); sign = -sign; }
    if (p1.spin == 1) { std::swap(p1, p2); sign = -sign; }
    blk = 2;
  }
  f = DFac{};
  f.type = 2;
  f.blk = (signed char)blk;
  const Lo o[4] = {h1, h2, p1, p2};
  for (int k = 0; k < 4; ++k) {
    f.kind[k] = (signed char)o[k].kind;
    f.slot[k] = (signed char)o[k].slot;
  }
  return sign;
}

Lo flip(Lo d) {
  d.spin ^= 1;
  return d;
}

const int kMatch[5][10][4] = {
    {},
    {{-1}},
    {{-1, -1}, {1, 0}},
    {{-1, -1, -1}, {-1, 2, 1}, {1, 0, -1}, {2, -1, 0}},
    {{-1, -1, -1, -1}, {-1, -1, 3, 2}, {-1, 2, 1, -1}, {-1, 3, -1, 1}, {1, 0, -1, -1},
     {1, 0, 3, 2}, {2, -1, 0, -1}, {2, 3, 0, 1}, {3, -1, -1, 0}, {3, 2, 1, 0}}};
const int kNMatch[5] = {1, 1, 2, 4, 10};

// Cluster expansion of the coefficient of a+_{P0}..a+_{P(r-1)} a_{H(r-1)}..a_{H0}|B>
// in e^{T_B}|B>, as a list of (coefficient, factors) with T_B = flipped T_A.
std::vector<HTerm> expand_cluster(const std::vector<Lo>& L, const std::vector<int>& H, const std::vector<int>& P) {
  const int r = (int)H.size();
  std::vector<HTerm> out;
  if (r == 0) {
    out.push_back({1.0, {}});
    return out;
  }
  std::vector<int> perm(r);
  for (int k = 0; k < r; ++k) perm[k] = k;
  do {
    int sgn = 1;
    for (int a = 0; a < r; ++a)
      for (int b = a + 1; b < r; ++b)
        if (perm[a] > perm[b]) sgn = -sgn;
    for (int m = 0; m < kNMatch[r]; ++m) {
      const int* mt = kMatch[r][m];
      HTerm t{(double)sgn, {}};
      bool ok = true;
      for (int k = 0; k < r && ok; ++k) {
        const int partner = mt[k];
        DFac f;
        if (partner < 0) {
          ok = fac1(flip(L[H[k]]), flip(L[P[perm[k]]]), f);
          if (ok) t.f.push_back(f);
        } else if (partner > k) {
          const int s = fac2(flip(L[H[k]]), flip(L[H[partner]]), flip(L[P[perm[k]]]), flip(L[P[perm[partner]]]), f);
          ok = s != 0;
          if (ok) {
            t.coef *= 0.5 * s;
            t.f.push_back(f);
          }
        }
      }
      if (ok) out.push_back(t);
    }
  } while (std::next_permutation(perm.begin(), perm.end()));
  return out;
}

// All terms of K_x for one pattern (x = holes -> parts).
std::vector<HTerm> expand_pattern(const std::vector<Lo>& holes, const std::vector<Lo>& parts) {
  std::vector<Lo> L = {{0, KT, -1}, {1, KU, -1}, {0, KU, -1}, {1, KT, -1}};  // t a, u b, u a, t b
  auto add = [&](const Lo& d) {
    for (size_t k = 0; k < L.size(); ++k)
      if (L[k] == d) return (int)k;
    L.push_back(d);
    return (int)L.size() - 1;
  };
  const int rank = (int)holes.size();
  int hi[2], pi[2];
  for (int k = 0; k < rank; ++k) hi[k] = add(holes[k]);
  for (int k = 0; k < rank; ++k) pi[k] = add(parts[k]);
  unsigned maskA = 0;
  for (size_t k = 0; k < L.size(); ++k)
    if (occA(L[k])) maskA |= 1u << k;
  unsigned maskB = maskA;
  const int sB = apply_ops_host(maskB, {{1, 2}, {1, 3}, {0, 1}, {0, 0}});  // a+_{ua} a+_{tb} a_{ub} a_{ta}

  // sub-excitations y of x with the e^{-T_A} matrix elements <A^x|e^{-T_A}|A^y>
  struct Y {
    std::vector<std::pair<int, int>> ops;
    std::vector<HTerm> e;
  };
  std::vector<Y> ys;
  auto mono = [](double c, std::initializer_list<std::pair<bool, DFac>> fs) {
    HTerm t{c, {}};
    for (auto& p : fs) {
      if (!p.first) return HTerm{0.0, {}};
      t.f.push_back(p.second);
    }
    return t;
  };
  DFac f0, f1;
  if (rank == 1) {
    ys.push_back({{}, {}});
    {
      const bool ok = fac1(holes[0], parts[0], f0);
      ys.back().e.push_back(mono(-1.0, {{ok, f0}}));
    }
    ys.push_back({{{1, pi[0]}, {0, hi[0]}}, {HTerm{1.0, {}}}});
  } else {
    Y y0{{}, {}};
    {
      DFac f2;
      const int s = fac2(holes[0], holes[1], parts[0], parts[1], f2);
      if (s) y0.e.push_back(HTerm{-1.0 * s, {f2}});
      bool a = fac1(holes[0], parts[0], f0), b = fac1(holes[1], parts[1], f1);
      y0.e.push_back(mono(1.0, {{a, f0}, {b, f1}}));
      a = fac1(holes[0], parts[1], f0);
      b = fac1(holes[1], parts[0], f1);
      y0.e.push_back(mono(-1.0, {{a, f0}, {b, f1}}));
    }
    ys.push_back(y0);
    // single y = (h -> p): -t(j->b) for (i->a), +t(i->b) for (j->a), +t(j->a) for (i->b), -t(i->a) for (j->b)
    const int yh[4] = {0, 1, 0, 1}, yp[4] = {0, 0, 1, 1};
    const double ys_sign[4] = {-1.0, 1.0, 1.0, -1.0};
    for (int q = 0; q < 4; ++q) {
      const int oh = 1 - yh[q], opp = 1 - yp[q];
      const bool ok = fac1(holes[oh], parts[opp], f0);
      ys.push_back({{{1, pi[yp[q]]}, {0, hi[yh[q]]}}, {mono(ys_sign[q], {{ok, f0}})}});
    }
    ys.push_back({{{1, pi[0]}, {1, pi[1]}, {0, hi[1]}, {0, hi[0]}}, {HTerm{1.0, {}}}});
  }

  std::vector<HTerm> terms;
  for (const Y& y : ys) {
    bool any = false;
    for (const HTerm& e : y.e) any = any || e.coef != 0.0;
    if (!any) continue;
    unsigned my = maskA;
    const int sy = apply_ops_host(my, y.ops);
    if (sy == 0) continue;
    const unsigned hb = maskB & ~my, pb = my & ~maskB;
    if (__builtin_popcount(hb) != __builtin_popcount(pb) || __builtin_popcount(hb) > 4) continue;
    std::vector<int> H, P;
    for (size_t k = 0; k < L.size(); ++k) {
      if (hb & (1u << k)) H.push_back((int)k);
      if (pb & (1u << k)) P.push_back((int)k);
    }
    std::vector<std::pair<int, int>> canon;
    for (int p : P) canon.push_back({1, p});
    for (int k = (int)H.size() - 1; k >= 0; --k) canon.push_back({0, H[k]});
    unsigned mc = maskB;
    const int sc = apply_ops_host(mc, canon);
    if (sc == 0 || mc != my) continue;
    const double pre = (double)(sy * sB * sc);
    for (const HTerm& c : expand_cluster(L, H, P))
      for (const HTerm& e : y.e) {
        if (e.coef == 0.0) continue;
        HTerm t{pre * c.coef * e.coef, e.f};
        t.f.insert(t.f.end(), c.f.begin(), c.f.end());
        terms.push_back(t);
      }
  }
  return terms;
}

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

// One pattern: thread -> (i, j, a, b) over the pattern's index ranges (core and
// virtual indices 0-based).  Equal-spin doubles with two core (virtual) indices
// are handled for i < j (a < b) and written to the four antisymmetric copies.
__global__ void coupling_pattern(const DTerm* __restrict__ terms, int nterms, PatternLaunch pl, Amp A,
                                 double* __restrict__ R, const double* __restrict__ Wp) {
  const int64_t tot = (int64_t)pl.cnt[0] * pl.cnt[1] * pl.cnt[2] * pl.cnt[3];
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= tot) return;
  int64_t r = id;
  const int bb = (int)(r % pl.cnt[3]); r /= pl.cnt[3];
  const int aa = (int)(r % pl.cnt[2]); r /= pl.cnt[2];
  const int jj = (int)(r % pl.cnt[1]);
  const int ii = (int)(r / pl.cnt[1]);
  const bool same = pl.block == 2 || pl.block == 3;
  if (same && pl.kind[0] == CORE && pl.kind[1] == CORE && ii >= jj) return;
  if (same && pl.kind[2] == VIRT && pl.kind[3] == VIRT && aa >= bb) return;
  double K = 0.0;
  for (int t = 0; t < nterms; ++t) {
    const DTerm& T = terms[t];
    double v = T.coef;
    for (int q = 0; q < T.nf; ++q) v *= factor(A, T.f[q], ii, jj, aa, bb);
    K += v;
  }
  const double KW = K * (*Wp);
  const int nc = A.nc, o = A.o, v = A.v;
  const int64_t ov = (int64_t)o * v, s2 = ov * ov;
  const int i = occ_pos(pl.kind[0], ii, nc), a = vir_pos(pl.kind[2], aa);
  if (pl.block < 2) {
    R[pl.block * ov + (int64_t)i * v + a] -= KW;
    return;
  }
  const int j = occ_pos(pl.kind[1], jj, nc), b = vir_pos(pl.kind[3], bb);
  double* Rb = R + 2 * ov + (int64_t)(pl.block - 2) * s2;
  auto at = [&](int p, int q, int c, int d) -> double& { return Rb[(((int64_t)p * o + q) * v + c) * v + d]; };
  at(i, j, a, b) -= KW;
  if (same) {
    at(j, i, a, b) += KW;
    at(i, j, b, a) += KW;
    at(j, i, b, a) -= KW;
  }
}

}  // namespace

namespace {
void add_patterns(std::vector<PatternLaunch>& pls, std::vector<DTerm>& all, int nc, int nv) {
  const int v = nv + 1;
  (void)v;
  auto choices_occ = [&](int spin, int slot) {
    std::vector<std::pair<Lo, int>> c;
    if (nc > 0) c.push_back({{spin, CORE, slot}, nc});
    c.push_back({{spin, spin == 0 ? KT : KU, -1}, 1});
    return c;
  };
  auto choices_vir = [&](int spin, int slot) {
    std::vector<std::pair<Lo, int>> c;
    c.push_back({{spin, VIRT, slot}, nv});
    c.push_back({{spin, spin == 0 ? KU : KT, -1}, 1});
    return c;
  };
  auto emit = [&](int block, const std::vector<Lo>& h, const std::vector<Lo>& p, const int cnt[4]) {
    PatternLaunch pl{};
    pl.block = block;
    pl.kind[0] = h[0].kind;
    pl.kind[2] = p[0].kind;
    pl.kind[1] = h.size() > 1 ? h[1].kind : CORE;
    pl.kind[3] = p.size() > 1 ? p[1].kind : CORE;
    for (int k = 0; k < 4; ++k) pl.cnt[k] = cnt[k];
    pl.term_off = (int)all.size();
    for (const HTerm& t : expand_pattern(h, p)) {
      if (t.coef == 0.0) continue;
      DTerm d{};
      d.coef = t.coef;
      d.nf = (int)t.f.size();
      if (d.nf > MAXF) throw std::runtime_error("coupling: too many factors");
      for (int q = 0; q < d.nf; ++q) d.f[q] = t.f[q];
      all.push_back(d);
    }
    pl.nterms = (int)all.size() - pl.term_off;
    pls.push_back(pl);
  };
  // singles
  for (int spin = 0; spin < 2; ++spin)
    for (auto& oc : choices_occ(spin, 0))
      for (auto& vc : choices_vir(spin, 2)) {
        const int cnt[4] = {oc.second, 1, vc.second, 1};
        emit(spin, {oc.first}, {vc.first}, cnt);
      }
  // doubles; equal spins: i < j and a < b (t is the last alpha-occupied, u the first alpha-virtual, etc.)
  for (int blk = 2; blk < 5; ++blk) {
    const int s1 = blk == 3 ? 1 : 0, s2 = blk == 2 ? 0 : 1;
    for (auto& oi : choices_occ(s1, 0))
      for (auto& oj : choices_occ(s2, 1))
        for (auto& va : choices_vir(s1, 2))
          for (auto& vb : choices_vir(s2, 3)) {
            if (blk < 4) {
              // equal spins: keep ordered pairs only (core < t, u-type virtual < virt)
              if (oi.first.kind != CORE && oj.first.kind != CORE) continue;  // t, t
              if (oi.first.kind != CORE && oj.first.kind == CORE) continue;  // (t, core): covered by (core, t)
              if (va.first.kind != VIRT && vb.first.kind != VIRT) continue;  // u, u
              if (va.first.kind == VIRT && vb.first.kind != VIRT) continue;  // (virt, u): covered by (u, virt)
            } else if (oi.first.kind != CORE && oj.first.kind != CORE && va.first.kind != VIRT &&
                       vb.first.kind != VIRT) {
              continue;  // the Phi_A -> Phi_B double (handled separately)
            }
            const int cnt[4] = {oi.second, oj.second, va.second, vb.second};
            emit(blk, {oi.first, oj.first}, {va.first, vb.first}, cnt);
          }
  }
}
}  // namespace

void coupling_prepare(int nc, int nv, std::vector<char>& launch_blob, std::vector<char>& term_blob) {
  std::vector<PatternLaunch> pls;
  std::vector<DTerm> all;
  add_patterns(pls, all, nc, nv);
  launch_blob.assign((const char*)pls.data(), (const char*)(pls.data() + pls.size()));
  term_blob.assign((const char*)all.data(), (const char*)(all.data() + all.size()));
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
// Every lane of a wave runs the same term loop (lanes past the end or outside
// the i < j, a < b half contribute zero), so that factors whose cotangent
// address is the same in all 64 lanes - every factor that does not depend on
// the fastest grid index, e.g. amplitudes with only t/u indices, which all
// elements of a pattern share - are summed in the wave first and added with
// one atomic instead of 64.
__global__ void coupling_pattern_adj(const DTerm* __restrict__ terms, int nterms, PatternLaunch pl, Amp A,
                                     double* Tbar, const double* __restrict__ Rbar, const double* __restrict__ Wp,
                                     double* Wbar) {
  const int64_t tot = (int64_t)pl.cnt[0] * pl.cnt[1] * pl.cnt[2] * pl.cnt[3];
  const int64_t id0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool inrange = id0 < tot;
  int64_t r = inrange ? id0 : tot - 1;
  const int bb = (int)(r % pl.cnt[3]); r /= pl.cnt[3];
  const int aa = (int)(r % pl.cnt[2]); r /= pl.cnt[2];
  const int jj = (int)(r % pl.cnt[1]);
  const int ii = (int)(r / pl.cnt[1]);
  const bool same = pl.block == 2 || pl.block == 3;
  const bool skip = (same && pl.kind[0] == CORE && pl.kind[1] == CORE && ii >= jj) ||
                    (same && pl.kind[2] == VIRT && pl.kind[3] == VIRT && aa >= bb);
  const int nc = A.nc, o = A.o, v = A.v;
  const int64_t ov = (int64_t)o * v, s2 = ov * ov;
  double rb = 0.0;
  if (inrange && !skip) {
    const int i = occ_pos(pl.kind[0], ii, nc), a = vir_pos(pl.kind[2], aa);
    if (pl.block < 2) {
      rb = Rbar[pl.block * ov + (int64_t)i * v + a];
    } else {
      const int j = occ_pos(pl.kind[1], jj, nc), b = vir_pos(pl.kind[3], bb);
      const double* Rb = Rbar + 2 * ov + (int64_t)(pl.block - 2) * s2;
      auto at = [&](int p, int q, int c, int d) { return Rb[(((int64_t)p * o + q) * v + c) * v + d]; };
      rb = at(i, j, a, b);
      if (same) rb += -at(j, i, a, b) - at(i, j, b, a) + at(j, i, b, a);
    }
  }
  const double g = -(*Wp) * rb;  // cotangent of K_x
  double K = 0.0;
  double* bars[5] = {Tbar, Tbar + ov, Tbar + 2 * ov, Tbar + 2 * ov + s2, Tbar + 2 * ov + 2 * s2};
  for (int t = 0; t < nterms; ++t) {
    const DTerm& T = terms[t];
    double fv[MAXF];
    for (int q = 0; q < T.nf; ++q) fv[q] = factor(A, T.f[q], ii, jj, aa, bb);
    double prod = T.coef;
    for (int q = 0; q < T.nf; ++q) prod *= fv[q];
    K += prod;
    for (int q = 0; q < T.nf; ++q) {
      double part = T.coef;
      for (int q2 = 0; q2 < T.nf; ++q2)
        if (q2 != q) part *= fv[q2];
      int arr;
      const int64_t off = factor_off(A, T.f[q], ii, jj, aa, bb, arr);
      const double val = g * part;
      const long long key = ((long long)arr << 40) | (long long)off;
      const long long k0 = __shfl(key, 0);
      if (__all(key == k0)) {
        const double sum = wave_sum(val);
        if (__lane_id() == 0 && sum != 0.0) atomicAdd(bars[arr] + off, sum);
      } else if (val != 0.0) {
        atomicAdd(bars[arr] + off, val);
      }
    }
  }
  const double w = wave_sum(-K * rb);
  if (__lane_id() == 0 && w != 0.0) atomicAdd(Wbar, w);
}

void coupling_apply_adj(const std::vector<char>& launch_blob, const void* d_terms, const double* T, double* Tbar,
                        const double* Rbar, const double* W_dev, double* Wbar, int nc, int nv, hipStream_t s) {
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
  const DTerm* terms = (const DTerm*)d_terms;
  for (size_t k = 0; k < np; ++k) {
    const PatternLaunch& pl = pls[k];
    const int64_t tot = (int64_t)pl.cnt[0] * pl.cnt[1] * pl.cnt[2] * pl.cnt[3];
    if (tot == 0 || pl.nterms == 0) continue;
    hipLaunchKernelGGL(coupling_pattern_adj, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       terms + pl.term_off, pl.nterms, pl, A, Tbar, Rbar, W_dev, Wbar);
    DCSD_CHECK_LAUNCH();
  }
}

void coupling_apply(const std::vector<char>& launch_blob, const void* d_terms, const double* T, double* R,
                    const double* W_dev, int nc, int nv, hipStream_t s) {
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
  const DTerm* terms = (const DTerm*)d_terms;
  for (size_t k = 0; k < np; ++k) {
    const PatternLaunch& pl = pls[k];
    const int64_t tot = (int64_t)pl.cnt[0] * pl.cnt[1] * pl.cnt[2] * pl.cnt[3];
    if (tot == 0 || pl.nterms == 0) continue;
    const int threads = 256;
    hipLaunchKernelGGL(coupling_pattern, dim3((unsigned)((tot + threads - 1) / threads)), dim3(threads), 0, s,
                       terms + pl.term_off, pl.nterms, pl, A, R, W_dev);
    DCSD_CHECK_LAUNCH();
  }
}

size_t coupling_term_size() { return sizeof(DTerm); }

}  // namespace dcsd
