// Symbolic expansion of the coupling coefficients K_x into per-pattern
// tables of amplitude products (host code).  Used by the library at context
// set-up and by the build-time generator of the compile-time tables
// (gen_coupling_tables.cpp); the derivation is described in coupling.hip.
#pragma once
#include <algorithm>
#include <cstring>
#include <stdexcept>
#include <utility>
#include <vector>

namespace dcsd {
namespace cpl {

enum Kind : int { CORE = 0, KT = 1, KU = 2, VIRT = 3 };

// A spin-orbital of a pattern: spin, kind and (for core/virtual) which index
// of x (0..3 = i, j, a, b) supplies its position.
struct Lo {
  int spin, kind, slot;
  bool operator==(const Lo& o) const { return spin == o.spin && kind == o.kind && slot == o.slot; }
};

inline bool occA(const Lo& d) { return d.kind == CORE || (d.kind == KT && d.spin == 0) || (d.kind == KU && d.spin == 1); }

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
  int fixed;       // index of the compile-time table of this pattern
};

// ---- host-side symbolic expansion -------------------------------------------
struct HTerm {
  double coef;
  std::vector<DFac> f;
};

inline int apply_ops_host(unsigned& mask, const std::vector<std::pair<int, int>>& ops) {
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
inline bool fac1(const Lo& h, const Lo& p, DFac& f) {
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
inline int fac2(Lo h1, Lo h2, Lo p1, Lo p2, DFac& f) {
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

inline Lo flip(Lo d) {
  d.spin ^= 1;
  return d;
}

inline constexpr int kMatch[5][10][4] = {
    {},
    {{-1}},
    {{-1, -1}, {1, 0}},
    {{-1, -1, -1}, {-1, 2, 1}, {1, 0, -1}, {2, -1, 0}},
    {{-1, -1, -1, -1}, {-1, -1, 3, 2}, {-1, 2, 1, -1}, {-1, 3, -1, 1}, {1, 0, -1, -1},
     {1, 0, 3, 2}, {2, -1, 0, -1}, {2, 3, 0, 1}, {3, -1, -1, 0}, {3, 2, 1, 0}}};
inline constexpr int kNMatch[5] = {1, 1, 2, 4, 10};

// Cluster expansion of the coefficient of a+_{P0}..a+_{P(r-1)} a_{H(r-1)}..a_{H0}|B>
// in e^{T_B}|B>, as a list of (coefficient, factors) with T_B = flipped T_A.
inline std::vector<HTerm> expand_cluster(const std::vector<Lo>& L, const std::vector<int>& H, const std::vector<int>& P) {
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
inline std::vector<HTerm> expand_pattern(const std::vector<Lo>& holes, const std::vector<Lo>& parts) {
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

// The patterns of every singles and doubles block, each with its expanded terms
// (exact zeros dropped), in a fixed order; cnt holds the index range sizes.
inline void add_patterns(std::vector<PatternLaunch>& pls, std::vector<DTerm>& all, int nc, int nv) {
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

// Fixed form of one pattern's terms: its distinct factors, in order of first
// appearance, and its terms as a coefficient times factors given by index,
// with the factor indices of a term sorted and terms with the same factors
// merged (coefficients summed, zero sums dropped).
struct FTerm {
  double coef;
  int nf;
  signed char idx[MAXF];
};
inline bool same_factor(const DFac& x, const DFac& y) { return std::memcmp(&x, &y, sizeof(DFac)) == 0; }
inline void fixed_form(const DTerm* terms, int nterms, std::vector<DFac>& fac, std::vector<FTerm>& out) {
  fac.clear();
  out.clear();
  for (int t = 0; t < nterms; ++t) {
    FTerm ft{};
    ft.coef = terms[t].coef;
    ft.nf = terms[t].nf;
    for (int q = 0; q < terms[t].nf; ++q) {
      int k = 0;
      while (k < (int)fac.size() && !same_factor(fac[k], terms[t].f[q])) ++k;
      if (k == (int)fac.size()) fac.push_back(terms[t].f[q]);
      ft.idx[q] = (signed char)k;
    }
    std::sort(ft.idx, ft.idx + ft.nf);
    bool merged = false;
    for (FTerm& o : out)
      if (o.nf == ft.nf && std::equal(o.idx, o.idx + o.nf, ft.idx)) {
        o.coef += ft.coef;
        merged = true;
        break;
      }
    if (!merged) out.push_back(ft);
  }
  out.erase(std::remove_if(out.begin(), out.end(), [](const FTerm& t) { return t.coef == 0.0; }), out.end());
}

}  // namespace cpl
}  // namespace dcsd
