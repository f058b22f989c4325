// Coupling between the two reference determinants: R_x -= K_x * W.
//
// K_x = <A^x| e^{-T_A} e^{T_B} |B>, T_B the spin flip of T_A (Theory
// section: the renormalisation term M_x W of the singles and doubles
// equations, with M_x = -K_x; the internal single products of the
// incomplete-active-space case are included and terms with a repeated
// spin-orbital cannot occur).  Each thread handles one amplitude x:
//
//   K_x = sum_{y subset of x} <A^x| e^{-T_A} |A^y> c_B(y),
//   c_B(y) = <A^y| e^{T_B} |B>,
//
// where the e^{-T_A} matrix elements are the closed forms of its single
// and double terms and every CI coefficient c_B is evaluated from the
// cluster expansion of e^{T_B} over the (at most four) holes and particles
// that separate A^y from B:  C = sum_{sigma} sgn(sigma) sum_{matchings}
// prod t1_B(h_k -> p_sigma(k)) prod 1/2 t2_B(h_k h_l -> p_sigma(k) p_sigma(l)).
// Fermion signs come from occupation bitmasks over the (<= 8) spin-orbitals
// involved, in a fixed local order.
#include "common.h"

namespace dcsd {
namespace {

// 1..4 element permutations with signs, and matchings into singletons and
// pairs (entry = partner position or -1).
__constant__ signed char kPerm1[1][1] = {{0}};
__constant__ signed char kPermSign1[1] = {1};
__constant__ signed char kPerm2[2][2] = {{0, 1}, {1, 0}};
__constant__ signed char kPermSign2[2] = {1, -1};
__constant__ signed char kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
__constant__ signed char kPermSign3[6] = {1, -1, -1, 1, 1, -1};
__constant__ signed char kPerm4[24][4] = {
    {0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 1, 3}, {0, 2, 3, 1}, {0, 3, 1, 2}, {0, 3, 2, 1},
    {1, 0, 2, 3}, {1, 0, 3, 2}, {1, 2, 0, 3}, {1, 2, 3, 0}, {1, 3, 0, 2}, {1, 3, 2, 0},
    {2, 0, 1, 3}, {2, 0, 3, 1}, {2, 1, 0, 3}, {2, 1, 3, 0}, {2, 3, 0, 1}, {2, 3, 1, 0},
    {3, 0, 1, 2}, {3, 0, 2, 1}, {3, 1, 0, 2}, {3, 1, 2, 0}, {3, 2, 0, 1}, {3, 2, 1, 0}};
__constant__ signed char kPermSign4[24] = {1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1,
                                           1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1};
__constant__ signed char kMatch1[1][1] = {{-1}};
__constant__ signed char kMatch2[2][2] = {{-1, -1}, {1, 0}};
__constant__ signed char kMatch3[4][3] = {{-1, -1, -1}, {-1, 2, 1}, {1, 0, -1}, {2, -1, 0}};
__constant__ signed char kMatch4[10][4] = {{-1, -1, -1, -1}, {-1, -1, 3, 2}, {-1, 2, 1, -1}, {-1, 3, -1, 1},
                                           {1, 0, -1, -1},   {1, 0, 3, 2},   {2, -1, 0, -1}, {2, 3, 0, 1},
                                           {3, -1, -1, 0},   {3, 2, 1, 0}};

enum Kind : signed char { CORE = 0, KT = 1, KU = 2, VIRT = 3 };

struct Orb {
  signed char spin, kind;
  int idx;
};

__device__ inline bool same(Orb a, Orb b) { return a.spin == b.spin && a.kind == b.kind && a.idx == b.idx; }

// Occupied in Phi_A = |core, t alpha, u beta>.
__device__ inline bool occA(Orb d) {
  return d.kind == CORE || (d.kind == KT && d.spin == 0) || (d.kind == KU && d.spin == 1);
}

struct Amp {
  const double* t1[2];
  const double* t2[3];  // aa, bb, ab
  int nc, o, v;

  __device__ int op(Orb d) const { return d.kind == CORE ? d.idx : nc; }
  __device__ int vp(Orb d) const { return d.kind == VIRT ? 1 + d.idx : 0; }
  __device__ int64_t i4(Orb a, Orb b, Orb c, Orb d) const {
    return (((int64_t)op(a) * o + op(b)) * v + vp(c)) * v + vp(d);
  }
  __device__ double t1A(Orb h, Orb p) const {
    if (h.spin != p.spin || !occA(h) || occA(p)) return 0.0;
    return t1[(int)h.spin][op(h) * v + vp(p)];
  }
  __device__ double t2A(Orb h1, Orb h2, Orb p1, Orb p2) const {
    if (!occA(h1) || !occA(h2) || occA(p1) || occA(p2)) return 0.0;
    const int s1 = h1.spin, s2 = h2.spin, s3 = p1.spin, s4 = p2.spin;
    if (s1 == 0 && s2 == 0) return (s3 == 0 && s4 == 0) ? t2[0][i4(h1, h2, p1, p2)] : 0.0;
    if (s1 == 1 && s2 == 1) return (s3 == 1 && s4 == 1) ? t2[1][i4(h1, h2, p1, p2)] : 0.0;
    if (s1 == 0) {  // h2 beta
      if (s3 == 0 && s4 == 1) return t2[2][i4(h1, h2, p1, p2)];
      if (s3 == 1 && s4 == 0) return -t2[2][i4(h1, h2, p2, p1)];
      return 0.0;
    }
    if (s3 == 0 && s4 == 1) return -t2[2][i4(h2, h1, p1, p2)];
    if (s3 == 1 && s4 == 0) return t2[2][i4(h2, h1, p2, p1)];
    return 0.0;
  }
  __device__ static Orb flip(Orb d) {
    d.spin ^= 1;
    return d;
  }
  __device__ double t1B(Orb h, Orb p) const { return t1A(flip(h), flip(p)); }
  __device__ double t2B(Orb h1, Orb h2, Orb p1, Orb p2) const {
    return t2A(flip(h1), flip(h2), flip(p1), flip(p2));
  }
};

// Apply an operator string (rightmost first) to a local bitmask; returns the
// sign (+1/-1) or 0 if the result vanishes.
__device__ int apply_ops(unsigned& mask, const signed char* create, const int* where, int nops) {
  int sign = 1;
  for (int q = nops - 1; q >= 0; --q) {
    const unsigned bit = 1u << where[q];
    if (__popc(mask & (bit - 1u)) & 1) sign = -sign;
    if (create[q]) {
      if (mask & bit) return 0;
      mask |= bit;
    } else {
      if (!(mask & bit)) return 0;
      mask ^= bit;
    }
  }
  return sign;
}

// Coefficient of a+_{P0}..a+_{P(r-1)} a_{H(r-1)}..a_{H0} |B> in e^{T_B}|B>.
__device__ double cluster_coef(const Amp& A, const Orb* L, const int* H, const int* P, int r) {
  if (r == 0) return 1.0;
  const signed char* perms;
  const signed char* signs;
  const signed char* match;
  int nperm, nmatch;
  switch (r) {
    case 1: perms = &kPerm1[0][0]; signs = kPermSign1; match = &kMatch1[0][0]; nperm = 1; nmatch = 1; break;
    case 2: perms = &kPerm2[0][0]; signs = kPermSign2; match = &kMatch2[0][0]; nperm = 2; nmatch = 2; break;
    case 3: perms = &kPerm3[0][0]; signs = kPermSign3; match = &kMatch3[0][0]; nperm = 6; nmatch = 4; break;
    default: perms = &kPerm4[0][0]; signs = kPermSign4; match = &kMatch4[0][0]; nperm = 24; nmatch = 10; break;
  }
  // spins of the holes and particles: a factor conserves spin, so most
  // (matching, permutation) pairs vanish and are skipped before any lookup
  int hs[4], ps[4];
  for (int k = 0; k < r; ++k) {
    hs[k] = L[H[k]].spin;
    ps[k] = L[P[k]].spin;
  }
  double sum = 0.0;
  for (int m = 0; m < nmatch; ++m) {
    const signed char* mt = match + m * r;
    for (int s = 0; s < nperm; ++s) {
      const signed char* pm = perms + s * r;
      bool ok = true;
      for (int k = 0; k < r && ok; ++k) {
        const int partner = mt[k];
        if (partner < 0) ok = hs[k] == ps[pm[k]];
        else if (partner > k) ok = hs[k] + hs[partner] == ps[pm[k]] + ps[pm[partner]];
      }
      if (!ok) continue;
      double prod = (double)signs[s];
      for (int k = 0; k < r && prod != 0.0; ++k) {
        const int partner = mt[k];
        if (partner < 0) {
          prod *= A.t1B(L[H[k]], L[P[pm[k]]]);
        } else if (partner > k) {
          prod *= 0.5 * A.t2B(L[H[k]], L[H[partner]], L[P[pm[k]]], L[P[pm[partner]]]);
        }
      }
      sum += prod;
    }
  }
  return sum;
}

struct Local {
  Orb L[8];
  int n = 0;
  __device__ int add(Orb d) {
    for (int k = 0; k < n; ++k)
      if (same(L[k], d)) return k;
    L[n] = d;
    return n++;
  }
};

// c_B(y) for the determinant A^y = (ops) |A>.
__device__ double cB(const Amp& A, const Local& loc, unsigned maskA, unsigned maskB, int sB,
                     const signed char* create, const int* where, int nops) {
  unsigned my = maskA;
  const int sy = apply_ops(my, create, where, nops);
  if (sy == 0) return 0.0;
  const unsigned hb = maskB & ~my, pb = my & ~maskB;
  const int r = __popc(hb);
  if (r != __popc(pb) || r > 4) return 0.0;
  int H[4], P[4], nh = 0, np = 0;
  for (int k = 0; k < loc.n; ++k) {
    if (hb & (1u << k)) H[nh++] = k;
    if (pb & (1u << k)) P[np++] = k;
  }
  // canonical string a+_{P0}..a+_{P(r-1)} a_{H(r-1)}..a_{H0} applied to |B>
  signed char cr[8];
  int wh[8];
  for (int k = 0; k < r; ++k) {
    cr[k] = 1;
    wh[k] = P[k];
    cr[r + k] = 0;
    wh[r + k] = H[r - 1 - k];
  }
  unsigned mc = maskB;
  const int sc = apply_ops(mc, cr, wh, 2 * r);
  if (sc == 0 || mc != my) return 0.0;
  return (double)(sy * sB * sc) * cluster_coef(A, loc.L, H, P, r);
}

__device__ Orb occ_orb(int spin, int i, int nc) {
  Orb d;
  d.spin = (signed char)spin;
  if (i < nc) { d.kind = CORE; d.idx = i; }
  else { d.kind = spin == 0 ? KT : KU; d.idx = 0; }
  return d;
}
__device__ Orb vir_orb(int spin, int a) {
  Orb d;
  d.spin = (signed char)spin;
  if (a > 0) { d.kind = VIRT; d.idx = a - 1; }
  else { d.kind = spin == 0 ? KU : KT; d.idx = 0; }
  return d;
}

__global__ void coupling_kernel(Amp A, double* R, const double* Wp, int64_t total) {
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= total) return;
  const int nc = A.nc, o = A.o, v = A.v;
  const int64_t ov = (int64_t)o * v, s2 = ov * ov;
  const double W = *Wp;

  Orb h[2], p[2];
  int rank;
  bool same_spin = false;
  if (x < 2 * ov) {
    const int spin = (int)(x / ov);
    const int64_t r = x % ov;
    h[0] = occ_orb(spin, (int)(r / v), nc);
    p[0] = vir_orb(spin, (int)(r % v));
    rank = 1;
  } else {
    const int64_t y = x - 2 * ov;
    const int blk = (int)(y / s2);
    int64_t r = y % s2;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o);
    const int i = (int)(r / o);
    const int si = blk == 1 ? 1 : 0, sj = blk == 0 ? 0 : 1;
    if (blk < 2) {
      same_spin = true;
      if (i == j || a == b) return;
    } else if (i == nc && j == nc && a == 0 && b == 0) {
      R[x] = 0.0;  // the Phi_A -> Phi_B double: its residual is W itself and is not solved for
      return;
    }
    h[0] = occ_orb(si, i, nc);
    h[1] = occ_orb(sj, j, nc);
    p[0] = vir_orb(si, a);
    p[1] = vir_orb(sj, b);
    rank = 2;
  }
  (void)same_spin;

  Local loc;
  Orb act[4] = {{0, KT, 0}, {1, KU, 0}, {0, KU, 0}, {1, KT, 0}};  // t a, u b, u a, t b
  for (int k = 0; k < 4; ++k) loc.add(act[k]);
  int hi[2], pi[2];
  for (int k = 0; k < rank; ++k) hi[k] = loc.add(h[k]);
  for (int k = 0; k < rank; ++k) pi[k] = loc.add(p[k]);
  unsigned maskA = 0;
  for (int k = 0; k < loc.n; ++k)
    if (occA(loc.L[k])) maskA |= 1u << k;
  // |B> = a+_{u a} a+_{t b} a_{u b} a_{t a} |A>
  unsigned maskB = maskA;
  const signed char cB_ops[4] = {1, 1, 0, 0};
  const int wB[4] = {2, 3, 1, 0};
  const int sB = apply_ops(maskB, cB_ops, wB, 4);

  double K;
  if (rank == 1) {
    const signed char c1[2] = {1, 0};
    const int w1[2] = {pi[0], hi[0]};
    K = cB(A, loc, maskA, maskB, sB, c1, w1, 2) - A.t1A(h[0], p[0]) * cB(A, loc, maskA, maskB, sB, c1, w1, 0);
  } else {
    const signed char c2[4] = {1, 1, 0, 0};
    const signed char c1[2] = {1, 0};
    const int wx[4] = {pi[0], pi[1], hi[1], hi[0]};
    K = cB(A, loc, maskA, maskB, sB, c2, wx, 4);
    // y = empty: <x| e^-T |A> = -t_ij^ab + t_i^a t_j^b - t_i^b t_j^a
    const double e0 = -A.t2A(h[0], h[1], p[0], p[1]) + A.t1A(h[0], p[0]) * A.t1A(h[1], p[1]) -
                      A.t1A(h[0], p[1]) * A.t1A(h[1], p[0]);
    if (e0 != 0.0) K += e0 * cB(A, loc, maskA, maskB, sB, c2, wx, 0);
    // single y = (k -> c): coefficients -t_j^b (i->a), +t_i^b (j->a), +t_j^a (i->b), -t_i^a (j->b)
    const int yh[4] = {hi[0], hi[1], hi[0], hi[1]};
    const int yp[4] = {pi[0], pi[0], pi[1], pi[1]};
    const double ey[4] = {-A.t1A(h[1], p[1]), A.t1A(h[0], p[1]), A.t1A(h[1], p[0]), -A.t1A(h[0], p[0])};
    for (int q = 0; q < 4; ++q) {
      if (ey[q] == 0.0) continue;
      const int w1[2] = {yp[q], yh[q]};
      K += ey[q] * cB(A, loc, maskA, maskB, sB, c1, w1, 2);
    }
  }
  R[x] -= K * W;
}

}  // namespace

void coupling_apply(const double* T, double* R, const double* W_dev, int nc, int nv, hipStream_t s) {
  Amp A;
  const int o = nc + 1, v = nv + 1;
  const int64_t ov = (int64_t)o * v, s2 = ov * ov;
  A.nc = nc; A.o = o; A.v = v;
  A.t1[0] = T;
  A.t1[1] = T + ov;
  A.t2[0] = T + 2 * ov;
  A.t2[1] = T + 2 * ov + s2;
  A.t2[2] = T + 2 * ov + 2 * s2;
  const int64_t total = 2 * ov + 3 * s2;
  const int threads = 128;
  hipLaunchKernelGGL(coupling_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, A,
                     R, W_dev, total);
  DCSD_CHECK_LAUNCH();
}

}  // namespace dcsd
