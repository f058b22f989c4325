// Context set-up and the 2D-DCSD / 2D-CCSD residual.
//
// Formulation (Theory section of the paper, implemented MI355X-first):
//  * Spin-blocked amplitudes of Phi_A (alpha and beta orbital orders differ
//    only by exchanging t and u).
//  * Singles enter through T1-dressed DF factors B~ = (1 - t1) B (1 + t1)
//    per spin and a dressed Fock matrix; the doubles residual is the CCD-like
//    expression of the dressed Hamiltonian plus the T2*T2 terms, in which the
//    distinguishable-cluster selection is applied (DCSD keeps the direct ring
//    and half of the two Fock-like terms, drops the rest).
//  * The particle-particle ladder is assembled from undressed spatial DF
//    factors in batches of orbital pairs, with the row index running over all
//    orbitals, so one assembly serves the alpha-alpha, beta-beta and
//    alpha-beta blocks and the T1 dressing of the ladder becomes a cheap back
//    transformation.
//  * Ring terms are particle-hole matrix products (spin-conserving 2ov x 2ov
//    and spin-flip ov x ov blocks).
//  * The coupling of the two determinants, R_x -= K_x W, is applied last.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>

#include "ops.h"

namespace dcsd {

// Ring GEMMs follow the precision and mode of the current evaluation
// (site: index of the call site; a_var / b_var: whether the operand changes
// with the amplitudes).  FP64: the MFMA GEMM; RECORD also stores the
// changing operands and the product P = A B at the refresh point.  Low
// precision: operands rounded into K-contiguous FP32/BF16 copies and
// multiplied on the low-precision MFMA with FP32 accumulation; DELTA uses
// A B = P_r + (A - A_r) B + A_r (B - B_r), rounding only the differences.
// The dressed-integral products (fp64_plain) take low precision only in that
// delta form and stay FP64 otherwise.  C must be a compact row-major M x N
// matrix.  Ring sites are timed as class 3.
void G::ring(Ctx& c, int site, bool a_var, bool b_var, bool fp64_plain) {
  hipEvent_t ev;
  const int rec = fp64_plain ? 0 : c.tbegin(&ev);  // the dressed-integral sites are not ring GEMMs
  if (a.ldc != a.N || !a.c_nc || a.batch != 1 || a.lda != (a.a_mc ? a.M : a.K) || a.ldb != (a.b_nc ? a.N : a.K))
    throw ArgError("ring GEMM site with a non-compact layout");
  Ctx::Site& st = c.site[site];
  const int64_t MN = a.M * a.N;
  if (c.prec_now == DCSD_PREC_FP64) {
    if (c.mode == Ctx::RECORD && st.Pr) {
      if (a_var) DCSD_HIP(hipMemcpyAsync(st.Ar, a.A, a.M * a.K * sizeof(double), hipMemcpyDeviceToDevice, c.s));
      if (b_var) DCSD_HIP(hipMemcpyAsync(st.Br, a.B, a.K * a.N * sizeof(double), hipMemcpyDeviceToDevice, c.s));
      G p(a.M, a.N, a.K);
      p.a = a;
      p.a.C = st.Pr;
      p.a.alpha = 1.0;
      p.a.beta = 0.0;
      p.run(c);
      axpby(a.C, st.Pr, a.alpha, a.beta, MN, c.s);
      st.valid = true;
    } else {
      run(c);
    }
  } else if (c.mode == Ctx::DELTA && st.valid) {
    axpby(a.C, st.Pr, a.alpha, a.beta, MN, c.s);
    if (a_var) lp_product(c, a.A, st.Ar, a.B, nullptr);
    if (b_var) lp_product(c, a_var ? st.Ar : a.A, nullptr, a.B, st.Br);
  } else if (fp64_plain) {
    run(c);  // the dressed integrals stay FP64 outside the delta form
  } else {
    lp_product(c, a.A, nullptr, a.B, nullptr, a.beta);
  }
  if (rec) c.tend(ev, 2.0 * (double)a.M * (double)a.N * (double)a.K, 3);
}
// C = alpha * lp(A - Asub) lp(B - Bsub) + beta * C (subtrahends may be NULL).
void G::lp_product(Ctx& c, const double* A, const double* Asub, const double* B, const double* Bsub, double beta) {
  const int pr = c.prec_now;
  const int64_t ld = lp_ld(a.K);
  if (a.M * ld > c.lp_cap || a.N * ld > c.lp_cap) throw ArgError("ring operand exceeds the low-precision buffer");
  // lpA[m][k] = A(m,k), lpB[n][k] = B(k,n)
  lp_convert(pr, c.lpA, ld, A, Asub, a.M, a.K, a.a_mc ? 1 : a.lda, a.a_mc ? a.lda : 1, c.s);
  lp_convert(pr, c.lpB, ld, B, Bsub, a.N, a.K, a.b_nc ? 1 : a.ldb, a.b_nc ? a.ldb : 1, c.s);
  LpGemm q;
  q.precision = pr;
  q.M = a.M; q.N = a.N; q.K = a.K;
  q.A = c.lpA; q.lda = ld; q.B = c.lpB; q.ldb = ld;
  q.C = a.C; q.ldc = a.ldc; q.c_nc = a.c_nc;
  q.alpha = a.alpha; q.beta = beta;
  const int64_t tiles = ((a.M + 127) / 128) * ((a.N + 127) / 128);
  int64_t ks = 1;
  if (tiles < 256 && a.K >= 2048) {
    ks = std::min<int64_t>(32, std::max<int64_t>(1, 1024 / tiles));
    while (ks > 1 && ks * a.M * a.N > c.lwork_cap) ks /= 2;
  }
  q.ks = (int)ks;
  q.work = c.lwork;
  q.k_padded = true;  // lp_convert zeroes the row padding of both operands
  lp_gemm(q, c.s);
}

namespace {

// Device operations of the residual and of the constants, recorded while a
// tape is active (the operation itself always runs).
void rfill(double* p, double v, int64_t n, hipStream_t s) {
  if (t_tape) tape_simple(OP_FILL, p, nullptr, n, v, 0.0);
  fill(p, v, n, s);
}
void raxpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s) {
  if (t_tape) tape_simple(OP_AXPBY, y, x, n, a, b);
  axpby(y, x, a, b, n, s);
}
void rcopy(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (t_tape) tape_simple(OP_MEMCPY, dst, src, n, 0.0, 0.0);
  DCSD_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
}
void rupload(double* dst, const double* host, int64_t n, hipStream_t s) {
  if (t_tape) tape_simple(OP_UPLOAD, dst, nullptr, n, 0.0, 0.0);
  DCSD_HIP(hipMemcpyAsync(dst, host, n * sizeof(double), hipMemcpyHostToDevice, s));
  DCSD_HIP(hipStreamSynchronize(s));  // the host source goes out of scope
}
void rswap(double* dst, const double* src, int64_t batch, int n, int nc, hipStream_t s) {
  if (t_tape) {
    TapeOp op;
    op.kind = OP_SWAPTU;
    op.dst = dst;
    op.src = src;
    op.n = batch;
    op.ints[0] = n;
    op.ints[1] = nc;
    tape_op(op);
  }
  swap_tu(dst, src, batch, n, nc, s);
}
void rjvec(double* J, const double* Ba, const double* Bb, int64_t naux, int n, int oa, int ob, hipStream_t s) {
  if (t_tape) {  // (the adjoint runs for Phi_A, oa == ob)
    TapeOp op;
    op.kind = OP_JVEC;
    op.dst = J;
    op.src = Ba;
    op.src2 = Bb;
    op.n = naux;
    op.ints[0] = n;
    op.ints[1] = oa;
    tape_op(op);
  }
  jvector(J, Ba, Bb, naux, n, oa, ob, s);
}
void rbreduce(double* dst, const double* src, int64_t nbat, int64_t bstride, int rows, int cols, int64_t ld,
              int64_t ldd, bool transpose, double alpha, hipStream_t s) {
  if (t_tape) {
    TapeOp op;
    op.kind = OP_BREDUCE;
    op.dst = dst;
    op.src = src;
    op.n = nbat;
    op.i64[0] = bstride;
    op.i64[1] = ld;
    op.i64[2] = ldd;
    op.ints[0] = rows;
    op.ints[1] = cols;
    op.ints[2] = transpose ? 1 : 0;
    op.alpha = alpha;
    tape_op(op);
  }
  batch_reduce(dst, src, nbat, bstride, rows, cols, ld, ldd, transpose, alpha, s);
}

}  // namespace

double* Ctx::alloc(int64_t count) {
  void* p = nullptr;
  const size_t b = (size_t)std::max<int64_t>(count, 1) * sizeof(double);
  if (hipMalloc(&p, b) != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  allocs.push_back(p);
  bytes += b;
  ++alloc_calls;
  reg((double*)p, std::max<int64_t>(count, 1), true);
  return (double*)p;
}

void* Ctx::alloc_raw(size_t b) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(b, 256)) != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  allocs.push_back(p);
  bytes += b;
  ++alloc_calls;
  return p;
}

int* Ctx::alloc_int(int64_t count) {
  void* p = nullptr;
  const size_t b = (size_t)std::max<int64_t>(count, 1) * sizeof(int);
  if (hipMalloc(&p, b) != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  allocs.push_back(p);
  bytes += b;
  ++alloc_calls;
  return (int*)p;
}

void Ctx::release() {
  tape_init.clear();
  tape_res.clear();
  for (void* p : allocs) (void)hipFree(p);
  allocs.clear();
}

// ---------------------------------------------------------------------------
// Fock matrix of Phi_A from (possibly dressed) factors:
//   f^s += sum_P J_P B^s[P] - sum_P sum_{k<o} B^s[P,:,k] B^s[P,k,:],
//   J_P = sum_{s'} sum_{k<o} B^{s'}[P,k,k].   fout must already hold h^s.
static void add_two_electron_fock(Ctx& c, double* const fout[2], double* const Bsrc[2]) {
  const int n = c.n;
  const int64_t naux = c.naux, n2 = c.n2;
  rjvec(c.Jv, Bsrc[0], Bsrc[1], naux, n, c.os[0], c.os[1], c.s);
  for (int sp = 0; sp < 2; ++sp) {
    const int o = c.os[sp];
    G(1, n2, naux).A(c.Jv, naux, false).B(Bsrc[sp], n2, true).C(fout[sp], n2).ab(1.0, 1.0).run(c);
    if (o == 0) continue;
    copyN(c.Xk, Bsrc[sp], {n, naux, o}, {naux * o, o, 1}, {n, n2, 1}, 1.0, 0.0, c.s);
    copyN(c.Yk, Bsrc[sp], {naux, o, n}, {(int64_t)o * n, n, 1}, {n2, n, 1}, 1.0, 0.0, c.s);
    G(n, n, naux * o).A(c.Xk, naux * o, false).B(c.Yk, n, true).C(fout[sp], n).ab(-1.0, 1.0).run(c);
  }
}

// X <- (1 - t1^T) X (1 + t1) for a batch of n x n matrices in the order of spin sp
// (t1 is o x v; rows/cols 0..o-1 occupied, o..n-1 virtual).
static void dress(Ctx& c, double* X, const double* t1, int64_t batch, int sp) {
  const int n = c.n, o = c.os[sp], v = c.vs[sp];
  const int64_t n2 = c.n2;
  if (o == 0) return;
  // X[:, 0:o] += X[:, o:n] t1^T
  G(n, o, v).A(X + o, n, false).B(t1, v, false).C(X, n).ab(1.0, 1.0).batch(batch, n2, 0, n2).run(c);
  // X[o:n, :] -= t1^T X[0:o, :]: a streaming kernel (under a tape, a recorded GEMM)
  if (!t_tape && dress_left(X, t1, n, o, v, n2, batch, c.s)) return;
  G(v, n, o).A(t1, v, true).B(X, n, true).C(X + (int64_t)o * n, n).ab(-1.0, 1.0).batch(batch, 0, n2, n2).run(c);
}

void Ctx::init(const dcsd_config& cf, const double* Bin, const double* Fin, hipStream_t stream) {
  cfg = cf;
  s = stream;
  if (cfg.nc < 0 || cfg.nv < 1 || cfg.naux < 1) throw ArgError("nc >= 0, nv >= 1 and naux >= 1 are required");
  if (!method_known(cfg.method)) throw ArgError("unknown method");
  if (cfg.precision != DCSD_PREC_FP64 && cfg.precision != DCSD_PREC_FP32 && cfg.precision != DCSD_PREC_BF16)
    throw ArgError("unknown precision");
  if (cfg.refresh_every < 0) throw ArgError("refresh_every must be >= 0");
  if (cfg.guard_iters < 0) throw ArgError("guard_iters must be >= 0");
  if (cfg.adjoint != 0 && cfg.adjoint != 1) throw ArgError("adjoint must be 0 or 1");
  if (cfg.ladder_cache < 0 || cfg.ladder_cache > 2) throw ArgError("ladder_cache must be 0, 1 or 2");
  if (cfg.diis_dim < 0 || cfg.diis_dim > 64) throw ArgError("diis_dim must be in [0, 64]");
  if (cfg.max_iter < 1) throw ArgError("max_iter must be >= 1");
  if (!(cfg.tol_residual > 0.0)) throw ArgError("tol_residual must be > 0");
  if (!(cfg.level_shift >= 0.0)) throw ArgError("level_shift must be >= 0");
  if (cfg.precond != DCSD_PRECOND_ORBITAL && cfg.precond != DCSD_PRECOND_EN) throw ArgError("unknown precond");
  const bool hs = method_hs(cfg.method);
  if (hs && cfg.nc < 1) throw ArgError("the high-spin methods need nc >= 1");
  if (hs && cfg.adjoint) throw ArgError("the adjoint is not available for the high-spin methods");
  if (!Bin || !Fin) throw ArgError("B and F must be device pointers");
  B = Bin;
  F = Fin;
  nc = cfg.nc;
  nv = cfg.nv;
  naux = cfg.naux;
  n = nc + 2 + nv;
  o = nc + 1;
  v = nv + 1;
  vu = nv + 2;
  npair = o * (o - 1) / 2;
  ov = (int64_t)o * v;
  s2 = ov * ov;
  n2 = (int64_t)n * n;
  // per-spin layout: Phi_A (t alpha, u beta) or the M_s = 1 determinant (t, u alpha)
  L.nc = nc;
  L.n = n;
  L.swap_tu = hs ? 0 : 1;
  L.o[0] = hs ? nc + 2 : o;
  L.o[1] = hs ? nc : o;
  L.v[0] = n - L.o[0];
  L.v[1] = n - L.o[1];
  for (int sp = 0; sp < 2; ++sp) {
    os[sp] = L.o[sp];
    vs[sp] = L.v[sp];
    ovs[sp] = L.ov(sp);
    oos[sp] = (int64_t)os[sp] * os[sp];
    npairs[sp] = os[sp] * (os[sp] - 1) / 2;
  }
  too2 = oos[0] + oos[1];
  tov = ovs[0] + ovs[1];
  sfr = (int64_t)os[0] * vs[1];
  sfc = (int64_t)os[1] * vs[0];
  total = L.total();
  wmax = std::max({ovs[0] * ovs[0], ovs[1] * ovs[1], ovs[0] * ovs[1], sfr * sfc, sfr * sfr, sfc * sfc});
  if ((int64_t)naux * n2 > (int64_t)1 << 40) throw ArgError("problem too large");
  DCSD_HIP(hipGetDevice(&device));

  const int64_t NA = naux;
  const int64_t o2 = (int64_t)o * o;
  // ---- allocations ------------------------------------------------------------
  (void)o2;
  Bs[0] = const_cast<double*>(B);
  // beta-order factors: Phi_A exchanges t and u; the high-spin determinant keeps the order
  Bs[1] = hs ? const_cast<double*>(B) : alloc(NA * n2);
  for (int sp = 0; sp < 2; ++sp) {
    h[sp] = alloc(n2);
    f[sp] = alloc(n2);
    Bt[sp] = alloc(NA * n2);
    ft[sp] = alloc(n2);
    Xv[sp] = alloc((int64_t)vs[sp] * vs[sp]);
    Fvv[sp] = alloc((int64_t)vs[sp] * vs[sp]);
    Yo[sp] = alloc(oos[sp]);
    Foo[sp] = alloc(oos[sp]);
    QX1[sp] = alloc(wmax);
    QX2[sp] = alloc(wmax);
    QY1[sp] = alloc(wmax);
    QY2[sp] = alloc(wmax);
    KJPQ[sp] = alloc(too2 * n2);
  }
  Bl = alloc(NA * n * vu);
  Jpq = alloc(n2);
  Kpq = alloc(n2);
  Isc = alloc(tov * tov);
  if (method_cc(cfg.method)) {
    Icc = alloc(tov * tov);
    Isf1 = alloc(sfr * sfc);
    Isf2 = alloc(sfr * sfc);
  }
  for (int k = 0; k < 3; ++k) Ikl[k] = alloc(wmax);
  Tw = alloc(total);
  Jv = alloc(NA);
  Xk = alloc((int64_t)n * NA * std::max(o, nc + 2));
  Yk = alloc((int64_t)n * NA * std::max(o, nc + 2));
  Bov = alloc(NA * tov);
  Bvo = alloc(NA * tov);
  Boo = alloc(NA * too2);
  Tsc = alloc(tov * tov);
  Tsf1 = alloc(sfr * sfc);
  Z = alloc(NA * tov);
  out1 = alloc(NA * std::max(ovs[0], ovs[1]));
  out2 = alloc(NA * std::max(ovs[0], ovs[1]));
  fvec = alloc(tov);
  KCBJ = alloc(tov * tov);
  Dvo = alloc(tov * tov);
  OOOO = alloc(too2 * too2);
  Ring = alloc(tov * tov);
  Wsf1 = alloc(sfc * sfc);
  Wsf2 = alloc(sfr * sfr);
  Rsf1 = alloc(sfr * sfc);
  Rsf2 = alloc(sfr * sfc);
  P1 = alloc(wmax);
  P2 = alloc(wmax);
  {
    const int64_t hh = std::max({oos[0], oos[1], (int64_t)os[0] * os[1]});
    Whh = alloc(hh * hh);
  }
  lb = cfg.ladder_block > 0 ? std::min(cfg.ladder_block, n) : std::min(32, n);
  const int64_t oab = (int64_t)os[0] * os[1];
  rows_main = oab + npairs[0] + npairs[1];
  rows_all = rows_main + oab;
  const int64_t vu2 = (int64_t)vu * vu;
  Tstack = alloc(rows_all * vu2);
  V2 = alloc((int64_t)lb * lb * vu2);
  Rb = alloc(rows_all * (int64_t)lb * lb);
  Rp = alloc(rows_main * n2);
  Smt = alloc(rows_main * (int64_t)n * std::max(vs[0], vs[1]));
  split_cap = 32;
  split = alloc(split_cap * rows_all * (int64_t)lb * lb);
  if (cfg.precision != DCSD_PREC_FP64) {
    const int64_t es = (int64_t)lp_size(cfg.precision);
    auto lp_alloc = [&](int64_t elems) { return (void*)alloc((elems * es + 7) / 8); };
    ldk = lp_ld(NA);
    kp = lp_ld(vu2);
    BlT = lp_alloc((int64_t)n * vu * ldk);
    TstackL = lp_alloc(rows_all * kp);
    V2L = lp_alloc((int64_t)lb * lb * kp);
    // the ladder contraction loads whole 16-byte chunks up to the end of K = vu^2: the row
    // padding of both operands is zeroed once here and nothing writes it afterwards
    fill((double*)TstackL, 0.0, (rows_all * kp * es + 7) / 8, s);
    fill((double*)V2L, 0.0, ((int64_t)lb * lb * kp * es + 7) / 8, s);
    // the ring operands (the rounding buffers lpA, lpB are allocated at the end of init,
    // sized also for the dressed-integral sites if those get their records)
    const int64_t lpm = std::max({tov, sfr, sfc});
    lp_cap = lpm * lp_ld(lpm);
    lwork_cap = std::max<int64_t>(split_cap * rows_all * (int64_t)lb * lb, (int64_t)1 << 22);
    lwork = (float*)alloc((lwork_cap + 1) / 2);
    TstackR = alloc(rows_all * vu2);
    RpR = alloc(rows_main * n2);
    // ring sites: 0 = I T_sc^T, 1 = T_sc W_sc (2ov x 2ov); 2, 3 = spin-flip I T (CCSD); 4, 5 = spin-flip
    // rings (the dressed-integral sites 6-10 are allocated at the end of init, when they fit)
    for (int k = 0; k < 6; ++k) {
      if ((k == 2 || k == 3) && !method_cc(cfg.method)) continue;
      if (site_size(k, 0)) site[k].Ar = alloc(site_size(k, 0));
      site[k].Br = alloc(site_size(k, 1));
      site[k].Pr = alloc(site_size(k, 2));
    }
  }
  gws_cap = std::max<int64_t>(1 << 22, 64 * (int64_t)v * v);
  gws = alloc(gws_cap);
  part = alloc(1024);
  scal = alloc(8 + 64);
  flag = alloc_int(4);
  Rw = alloc(total);
  if (cfg.diis_dim > 0) {
    histT = alloc((int64_t)cfg.diis_dim * total);
    histE = alloc((int64_t)cfg.diis_dim * total);
    coef = alloc(cfg.diis_dim);
  }
  Tn = alloc(total);
  Ev = alloc(total);
  Tbest = alloc(total);
  {
    // occupied pairs i < j: the alpha pairs, then the beta pairs
    std::vector<int> pi, pj;
    for (int sp = 0; sp < 2; ++sp)
      for (int i = 0; i < os[sp]; ++i)
        for (int j = i + 1; j < os[sp]; ++j) {
          pi.push_back(i);
          pj.push_back(j);
        }
    const int np = (int)pi.size();
    pair_i = alloc_int(std::max(np, 1));
    pair_j = alloc_int(std::max(np, 1));
    if (np > 0) {
      DCSD_HIP(hipMemcpyAsync(pair_i, pi.data(), np * sizeof(int), hipMemcpyHostToDevice, s));
      DCSD_HIP(hipMemcpyAsync(pair_j, pj.data(), np * sizeof(int), hipMemcpyHostToDevice, s));
      DCSD_HIP(hipStreamSynchronize(s));  // host sources go out of scope
    }
  }

  // ---- coupling patterns (checked against their compile-time tables) -----------
  if (!hs) coupling_prepare(nc, nv, coup_launch);
  // external inputs take part in the adjoint's buffer registry (not owned)
  reg(const_cast<double*>(B), NA * n2, false);
  reg(const_cast<double*>(F), n2, false);
  build_constants(true);
  if (cfg.adjoint) adj_reserve();
  alloc_optional();
}

// Optional memory, allocated after everything else and only where it leaves max(8 GiB, 5%)
// of the device memory free: in low precision the records of the dressed-integral delta
// sites (with the rounding buffers, which are allocated here in any case), then the ladder
// integral caches (cfg.ladder_cache): one slot per orbital-pair batch (p-block <= q-block),
// the low-precision slots of V2L's size with the row padding zeroed like V2L, the FP64
// slots of V2's size; then the FP64 GEMMs' padded operand workspace.
void Ctx::alloc_optional() {
  auto fits = [&](size_t b) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return fr > b && fr - b >= std::max<size_t>((size_t)8 << 30, tot / 20);
  };
  if (cfg.precision != DCSD_PREC_FP64) {
    // the dressed-integral delta sites 6-10 (records of their changing operands and FP64
    // products) and the rounding buffers, which those sites' operands enlarge; without the
    // records those products stay FP64 in every evaluation
    const int64_t es = (int64_t)lp_size(cfg.precision), NA = naux;
    const int64_t cap6 = std::max({lp_cap, tov * lp_ld(NA), n2 * lp_ld(NA), NA * lp_ld(tov), too2 * lp_ld(NA)});
    size_t rec = 0;
    for (int k = 6; k < kSites; ++k) rec += (size_t)(site_size(k, 0) + site_size(k, 1) + site_size(k, 2)) * 8;
    const bool with6 = fits(rec + (size_t)(2 * cap6 * es));
    if (with6) {
      lp_cap = cap6;
      for (int k = 6; k < kSites; ++k) {
        site[k].Ar = alloc(site_size(k, 0));
        site[k].Br = alloc(site_size(k, 1));
        site[k].Pr = alloc(site_size(k, 2));
      }
    }
    lpA = alloc((lp_cap * es + 7) / 8);
    lpB = alloc((lp_cap * es + 7) / 8);
  }
  // last, the padded operand copies of the FP64 GEMMs whose extents (o, v) are odd: the largest
  // products pad both operands of about o^2 v^2 elements each
  auto alloc_pad = [&]() {
    const int64_t om = std::max(L.o[0], L.o[1]), vm = std::max(L.v[0], L.v[1]) + 1;
    const int64_t cap = 2 * (om * om + 1) * vm * vm;
    if (fits((size_t)cap * sizeof(double))) {
      try {
        pws = (double*)alloc_raw((size_t)cap * sizeof(double));
        pws_cap = cap;
      } catch (const std::bad_alloc&) {
        pws = nullptr;
        pws_cap = 0;
      }
    }
  };
  if (!cfg.ladder_cache) {
    alloc_pad();
    DCSD_HIP(hipStreamSynchronize(s));
    return;
  }
  const int64_t nblk = (n + lb - 1) / lb, nbat = nblk * (nblk + 1) / 2;
  if (cfg.precision != DCSD_PREC_FP64) {
    const int64_t es = (int64_t)lp_size(cfg.precision);
    lcache_slot = (int64_t)lb * lb * kp;
    const size_t cbytes = (size_t)(nbat * lcache_slot * es);
    if (fits(cbytes)) {
      try {
        lcache = alloc_raw(cbytes);
        fill((double*)lcache, 0.0, (int64_t)((cbytes + 7) / 8), s);
      } catch (const std::bad_alloc&) {
        lcache = nullptr;
      }
    }
  }
  if (cfg.ladder_cache == 2) {
    lcache64_slot = (int64_t)lb * lb * vu * vu;
    const size_t cbytes = (size_t)(nbat * lcache64_slot) * sizeof(double);
    if (fits(cbytes)) {
      try {
        lcache64 = (double*)alloc_raw(cbytes);
      } catch (const std::bad_alloc&) {
        lcache64 = nullptr;
      }
    }
  }
  alloc_pad();
  DCSD_HIP(hipStreamSynchronize(s));
}

// Quantities of Phi_A built from (B, F) once per context; re-run under a tape
// by the adjoint (full = false skips the preconditioner matrices, the
// low-precision copy of the ladder factor and the reference energy, which
// carry no derivative).
void Ctx::build_constants(bool full) {
  const int64_t NA = naux;
  const bool hs = method_hs(cfg.method);
  // ---- beta-order factors: exchange t and u in both orbital indices (Phi_A) ---------
  if (!hs) rswap(Bs[1], Bs[0], NA, n, nc, s);

  // ---- one-electron Hamiltonian h = F - G_avg ---------------------------------------
  // G_avg = sum_core [2 J_k - K_k] + sum_{t,u} [J_x - K_x / 2]
  {
    const int K2 = nc + 2;
    // weighted Coulomb vector jw[P] = sum_{k<nc} 2 B[P,k,k] + B[P,t,t] + B[P,u,u]
    copyN(Xk, B, {NA, K2}, {K2, 1}, {n2, n + 1}, 1.0, 0.0, s);
    std::vector<double> w(K2, 1.0);
    for (int k = 0; k < nc; ++k) w[k] = 2.0;
    rupload(fvec, w.data(), K2, s);
    G(NA, 1, K2).A(Xk, K2, false).B(fvec, 1, true).C(Jv, 1).run(*this);
    rcopy(h[0], F, n2, s);
    G(1, n2, NA).A(Jv, NA, false).B(B, n2, true).C(h[0], n2).ab(-1.0, 1.0).run(*this);
    // exchange: X[p][(P,k)] = c_k B[P,p,k] (c = 1 core, 1/2 open), Y[(P,k)][q] = B[P,k,q]
    copyN(Xk, B, {n, NA, K2}, {NA * K2, K2, 1}, {n, n2, 1}, 1.0, 0.0, s);
    copyN(Xk + nc, B + nc, {n, NA, 2}, {NA * K2, K2, 1}, {n, n2, 1}, 0.5, 0.0, s);
    copyN(Yk, B, {NA, K2, n}, {(int64_t)K2 * n, n, 1}, {n2, n, 1}, 1.0, 0.0, s);
    G(n, n, NA * K2).A(Xk, NA * K2, false).B(Yk, n, true).C(h[0], n).ab(1.0, 1.0).run(*this);
    if (hs)
      rcopy(h[1], h[0], n2, s);
    else
      rswap(h[1], h[0], 1, n, nc, s);
  }
  // ---- Fock matrices of Phi_A (undressed) ------------------------------------------
  for (int sp = 0; sp < 2; ++sp)
    rcopy(f[sp], h[sp], n2, s);
  add_two_electron_fock(*this, f, Bs);

  // ---- (kc|ld) in the spin-conserving particle-hole layout --------------------------
  // Isc[(s,k,c),(s',l,d)], rows and columns [alpha (o0 v0) | beta (o1 v1)]
  for (int sp = 0; sp < 2; ++sp)
    copyN(Bov + L.t1_off(sp), Bs[sp] + os[sp], {NA, os[sp], vs[sp]}, {tov, vs[sp], 1}, {n2, n, 1}, 1.0, 0.0, s);
  G(tov, tov, NA).A(Bov, tov, true).B(Bov, tov, true).C(Isc, tov).run(*this);

  // Permuted copies used by the X, Y and hole-hole intermediates.
  const int oa = os[0], ob = os[1], va = vs[0], vb = vs[1];
  const int64_t ab_blk = ovs[0];  // Isc + ab_blk: the alpha-row, beta-column block
  for (int sp = 0; sp < 2; ++sp) {
    const int o_ = os[sp], v_ = vs[sp];
    const int64_t base = L.t1_off(sp) * (tov + 1), vt = (int64_t)v_ * tov;
    const std::initializer_list<int64_t> d4 = {o_ * (int64_t)v_ * v_, (int64_t)v_ * v_, v_, 1};
    // QX1[(k,l,c)][d] = (kc|ld)_ss
    copyN(QX1[sp], Isc + base, {o_, o_, v_, v_}, d4, {vt, v_, tov, 1}, 1.0, 0.0, s);
    // QY1[l][(k,c,d)] = (kc|ld)_ss
    copyN(QY1[sp], Isc + base, {o_, o_, v_, v_}, d4, {v_, vt, tov, 1}, 1.0, 0.0, s);
    // Ikl[(k,l),(c,d)] = (kc|ld)_ss
    copyN(Ikl[sp], Isc + base, {o_, o_, v_, v_}, d4, {vt, v_, tov, 1}, 1.0, 0.0, s);
  }
  const int64_t vta = (int64_t)va * tov;
  // QX2a[(k,L,C)][d] = (kd|LC)  (k, d alpha; L, C beta)
  copyN(QX2[0], Isc + ab_blk, {oa, ob, vb, va}, {ob * (int64_t)vb * va, (int64_t)vb * va, va, 1}, {vta, vb, 1, tov},
        1.0, 0.0, s);
  // QX2b[(l,K,c)][D] = (KD|lc)  (l, c alpha; K, D beta)
  copyN(QX2[1], Isc + ab_blk, {oa, ob, va, vb}, {ob * (int64_t)va * vb, (int64_t)va * vb, vb, 1}, {vta, vb, tov, 1},
        1.0, 0.0, s);
  // QY2a[l][(K,d,C)] = (KC|ld)  (l, d alpha; K, C beta)
  copyN(QY2[0], Isc + ab_blk, {oa, ob, va, vb}, {ob * (int64_t)va * vb, (int64_t)va * vb, vb, 1}, {vta, vb, tov, 1},
        1.0, 0.0, s);
  // QY2b[L][(k,c,D)] = (kc|LD)  (k, c alpha; L, D beta)
  copyN(QY2[1], Isc + ab_blk, {ob, oa, va, vb}, {oa * (int64_t)va * vb, (int64_t)va * vb, vb, 1}, {vb, vta, tov, 1},
        1.0, 0.0, s);
  // Ikl_ab[(k,L),(c,D)] = (kc|LD)
  copyN(Ikl[2], Isc + ab_blk, {oa, ob, va, vb}, {ob * (int64_t)va * vb, (int64_t)va * vb, vb, 1}, {vta, vb, tov, 1},
        1.0, 0.0, s);
  if (method_cc(cfg.method)) {
    // <kl||cd> = (kc|ld) - (kd|lc): exchange part on the equal-spin blocks
    rcopy(Icc, Isc, tov * tov, s);
    for (int sp = 0; sp < 2; ++sp) {
      const int o_ = os[sp], v_ = vs[sp];
      const int64_t base = L.t1_off(sp) * (tov + 1), vt = (int64_t)v_ * tov;
      copyN(Icc + base, Isc + base, {o_, v_, o_, v_}, {vt, tov, v_, 1}, {vt, 1, v_, tov}, -1.0, 1.0, s);
    }
    // spin-flip blocks: Isf1[(K,c),(l,D)] = -(KD|lc) (rows beta occ x alpha vir, columns alpha occ x
    // beta vir), Isf2[(k,C),(L,d)] = -(kd|LC) (rows alpha occ x beta vir, columns beta occ x alpha vir)
    const int64_t vtb = (int64_t)vb * tov;
    copyN(Isf1, Isc + ovs[0] * tov, {ob, va, oa, vb}, {va * sfr, sfr, vb, 1}, {vtb, 1, va, tov}, -1.0, 0.0, s);
    copyN(Isf2, Isc + ab_blk, {oa, vb, ob, va}, {vb * sfc, sfc, va, 1}, {vta, 1, vb, tov}, -1.0, 0.0, s);
  }
  // ---- ladder factor Bl[P][p][c] = B[P][p][nc + c], c over [t, u, virt] ------------
  copyN(Bl, B + nc, {NA, n, vu}, {(int64_t)n * vu, vu, 1}, {n2, n, 1}, 1.0, 0.0, s);
  if (!full) return;
  // ---- Coulomb/exchange matrices J_pq = (pp|qq), K_pq = (pq|qp) for the Epstein-Nesbet diagonal
  copyN(Xk, B, {NA, n}, {n, 1}, {n2, n + 1}, 1.0, 0.0, s);  // B[P][p][p]
  G(n, n, NA).A(Xk, n, true).B(Xk, n, true).C(Jpq, n).run(*this);
  sumsq_batch(Kpq, B, NA, n2, s);
  // low precision: BlT[(p,c)][P] = round(Bl[P][p][c])
  if (BlT) lp_convert(cfg.precision, BlT, ldk, Bl, nullptr, (int64_t)n * vu, NA, 1, (int64_t)n * vu, s);

  // ---- reference energy E_ref = 1/2 sum_s sum_{k<o} (h_kk + f_kk) --------------------
  {
    std::vector<double> hd(n2), fd(n2);
    double e = 0.0;
    for (int sp = 0; sp < 2; ++sp) {
      DCSD_HIP(hipMemcpyAsync(hd.data(), h[sp], n2 * sizeof(double), hipMemcpyDeviceToHost, s));
      DCSD_HIP(hipMemcpyAsync(fd.data(), f[sp], n2 * sizeof(double), hipMemcpyDeviceToHost, s));
      DCSD_HIP(hipStreamSynchronize(s));
      for (int k = 0; k < os[sp]; ++k) e += 0.5 * (hd[(int64_t)k * n + k] + fd[(int64_t)k * n + k]);
    }
    e_ref = e;
  }
  DCSD_HIP(hipStreamSynchronize(s));
}

// Doubles of a delta site's records: which = 0 the changing A operand (0: A constant),
// 1 the B operand, 2 the product.  Sites: 0 = I T_sc^T, 1 = T_sc W_sc (2ov x 2ov); 2, 3 =
// spin-flip I T (CCSD); 4, 5 = spin-flip rings; dressed integrals (delta form only): 6 =
// (ai|bj)~, 7 = (kc|bj)~, 8, 9 = (kj|pq)~ per spin, 10 = the singles intermediate Z.
int64_t Ctx::site_size(int k, int which) const {
  const int64_t NA = naux, sf2 = std::max(sfr, sfc) * std::max(sfr, sfc);
  const int64_t szA[kSites] = {0, tov * tov, 0, 0, sf2, sf2, NA * tov, NA * tov, NA * too2, NA * too2, NA * tov};
  const int64_t szB[kSites] = {tov * tov, tov * tov, sf2, sf2, sf2, sf2, NA * tov, NA * tov, NA * n2, NA * n2,
                               tov * tov};
  const int64_t szP[kSites] = {tov * tov, tov * tov, sf2, sf2, sf2, sf2, tov * tov, tov * tov, too2 * n2, too2 * n2,
                               NA * tov};
  return which == 0 ? szA[k] : (which == 1 ? szB[k] : szP[k]);
}

// ---------------------------------------------------------------------------
void Ctx::residual(const double* T, double* R, double* W_host, int prec, int md) {
  prec_now = prec < 0 ? cfg.precision : prec;
  if (prec_now != DCSD_PREC_FP64 && !BlT) throw ArgError("low precision was not configured at init");
  if ((md == RECORD && (prec_now != DCSD_PREC_FP64 || !BlT)) || (md == DELTA && prec_now == DCSD_PREC_FP64))
    throw ArgError("invalid evaluation mode");
  mode = md;
  if (mode == RECORD) {
    ladder_ref = false;
    for (auto& x : site) x.valid = false;
  }
  const uint32_t mask = cfg.term_mask;
  const int64_t NA = naux;
  const bool cc = method_cc(cfg.method);
  const double sdc = cc ? 1.0 : 0.5;  // weight of the Fock-like T2*T2 terms (Q_c, Q_d)
  const int oa = os[0], ob = os[1], va = vs[0], vb = vs[1];
  const int64_t oab = (int64_t)oa * ob;
  hipEvent_t ev_res;
  const int rec_res = tbegin(&ev_res);

  // amplitudes with the Phi_A -> Phi_B double set: zero in the two-determinant methods,
  // +1 or -1 in the fixed-reference ones (the high-spin methods have no such element)
  rcopy(Tw, T, total, s);
  const int64_t ab_pos = L.t2_off(2) + (((int64_t)nc * ob + nc) * va + 0) * vb + 0;
  if (method_ab(cfg.method)) rfill(Tw + ab_pos, ab_amplitude(cfg.method), 1, s);
  const double* t1[2] = {Tw + L.t1_off(0), Tw + L.t1_off(1)};
  const double* t2aa = Tw + L.t2_off(0);
  const double* t2bb = Tw + L.t2_off(1);
  const double* t2ab = Tw + L.t2_off(2);
  const double* t2ss[2] = {t2aa, t2bb};
  double* R1 = R;
  double* R2ss[2] = {R + L.t2_off(0), R + L.t2_off(1)};
  double* R2ab = R + L.t2_off(2);
  rfill(R, 0.0, total, s);

  // ---- T1 dressing of the DF factors and of the Fock matrix ------------------------
  for (int sp = 0; sp < 2; ++sp) {
    rcopy(Bt[sp], Bs[sp], NA * n2, s);
    dress(*this, Bt[sp], t1[sp], NA, sp);
    rcopy(ft[sp], h[sp], n2, s);
    dress(*this, ft[sp], t1[sp], 1, sp);
  }
  add_two_electron_fock(*this, ft, Bt);

  // ---- dressed factor blocks -----------------------------------------------------
  // Bov[P][(s,k,c)], Bvo[P][(s,k,c)] = B~[P][c][k], Boo[P][(s,k,i)] (rows [alpha | beta])
  for (int sp = 0; sp < 2; ++sp) {
    const int o_ = os[sp], v_ = vs[sp];
    copyN(Bov + L.t1_off(sp), Bt[sp] + o_, {NA, o_, v_}, {tov, v_, 1}, {n2, n, 1}, 1.0, 0.0, s);
    copyN(Bvo + L.t1_off(sp), Bt[sp] + (int64_t)o_ * n, {NA, o_, v_}, {tov, v_, 1}, {n2, 1, n}, 1.0, 0.0, s);
    copyN(Boo + (sp ? oos[0] : 0), Bt[sp], {NA, o_, o_}, {too2, o_, 1}, {n2, n, 1}, 1.0, 0.0, s);
  }

  // ---- particle-hole amplitude matrices ------------------------------------------
  // Tsc[(s,i,a),(s',k,c)] = t_ik^ac (spin-orbital), spin-conserving excitations
  const int64_t vta = (int64_t)va * tov, vtb = (int64_t)vb * tov;
  const int64_t aa2 = (int64_t)oa * va * va, bb2 = (int64_t)ob * vb * vb, ab2 = (int64_t)ob * va * vb;
  copyN(Tsc, t2aa, {oa, va, oa, va}, {vta, tov, va, 1}, {aa2, va, (int64_t)va * va, 1}, 1.0, 0.0, s);
  copyN(Tsc + ovs[0], t2ab, {oa, va, ob, vb}, {vta, tov, vb, 1}, {ab2, vb, (int64_t)va * vb, 1}, 1.0, 0.0, s);
  copyN(Tsc + ovs[0] * tov, t2ab, {ob, vb, oa, va}, {vtb, tov, va, 1}, {(int64_t)va * vb, 1, ab2, vb}, 1.0, 0.0, s);
  copyN(Tsc + ovs[0] * tov + ovs[0], t2bb, {ob, vb, ob, vb}, {vtb, tov, vb, 1}, {bb2, vb, (int64_t)vb * vb, 1}, 1.0,
        0.0, s);
  // Tsf1[(i,A),(K,c)] = t_{i K}^{A c} = -t2ab[i,K,c,A]  (sfr x sfc; Tsf2 = Tsf1^T)
  copyN(Tsf1, t2ab, {oa, vb, ob, va}, {vb * sfc, sfc, va, 1}, {ab2, 1, (int64_t)va * vb, vb}, -1.0, 0.0, s);

  // ---- singles residual -------------------------------------------------------------
  if (mask & DCSD_TERM_SINGLES) {
    for (int sp = 0; sp < 2; ++sp) {
      const int o_ = os[sp], v_ = vs[sp];
      copyN(R1 + L.t1_off(sp), ft[sp] + (int64_t)o_ * n, {o_, v_}, {v_, 1}, {1, n}, 1.0, 0.0, s);   // f~_ai
      copyN(fvec + L.t1_off(sp), ft[sp] + o_, {o_, v_}, {v_, 1}, {n, 1}, 1.0, 0.0, s);             // f~_kc
    }
    // sum_kc f~_kc t_ik^ac
    G(tov, 1, tov).A(Tsc, tov, false).B(fvec, 1, true).C(R1, 1).ab(1.0, 1.0).run(*this);
    // Z[P][(s,i,c)] = sum_{(s',k,d)} B~_ov[P][(s',k,d)] t_ik^cd
    G(NA, tov, tov).A(Bov, tov, false).B(Tsc, tov, true).C(Z, tov).ring(*this, 10, true, true, true);
    for (int sp = 0; sp < 2; ++sp) {
      const int o_ = os[sp], v_ = vs[sp];
      if (o_ == 0) continue;
      const int64_t off = L.t1_off(sp), ovx = ovs[sp];
      // + sum_P sum_c B~[P][a][c] Z[P][i][c]
      G(v_, o_, v_).A(Bt[sp] + (int64_t)o_ * n + o_, n, false).B(Z + off, v_, false).C(out1, o_)
          .batch(NA, n2, tov, ovx).run(*this);
      rbreduce(R1 + off, out1, NA, ovx, v_, o_, o_, v_, true, 1.0, s);
      // - sum_P sum_k B~[P][k][i] Z[P][k][a]
      G(o_, v_, o_).A(Bt[sp], n, true).B(Z + off, v_, true).C(out2, v_).batch(NA, n2, tov, ovx).run(*this);
      rbreduce(R1 + off, out2, NA, ovx, o_, v_, v_, v_, false, -1.0, s);
    }
  }

  // ---- driver and ring terms (particle-hole layout) -------------------------------
  // Dvo[(s,i,a),(s',j,b)] = (ai|bj)~
  if (mask & (DCSD_TERM_DRIVER | DCSD_TERM_RING))
    G(tov, tov, NA).A(Bvo, tov, true).B(Bvo, tov, true).C(Dvo, tov).ring(*this, 6, true, true, true);
  if (!(mask & DCSD_TERM_DRIVER)) rfill(Dvo, 0.0, tov * tov, s);
  if (mask & (DCSD_TERM_RING | DCSD_TERM_HH)) {
    // OOOO[(s,k,i),(s',l,j)] = (ki|lj)~
    G(too2, too2, NA).A(Boo, too2, true).B(Boo, too2, true).C(OOOO, too2).run(*this);
  }
  if (mask & DCSD_TERM_RING) {
    // KCBJ[(s,k,c),(s',j,b)] = (kc|bj)~ ; KJPQ[s'][(s,k,j)][(p,q)] = (kj|pq)~ (p, q in spin s' order)
    G(tov, tov, NA).A(Bov, tov, true).B(Bvo, tov, true).C(KCBJ, tov).ring(*this, 7, true, true, true);
    for (int sp = 0; sp < 2; ++sp)
      G(too2, n2, NA).A(Boo, too2, true).B(Bt[sp], n2, true).C(KJPQ[sp], n2).ring(*this, 8 + sp, true, true, true);
    // W_sc = <kb||cj>~ = (kc|bj)~ - (kj|bc)~ (equal spins)
    for (int sp = 0; sp < 2; ++sp) {
      const int o_ = os[sp], v_ = vs[sp];
      const int64_t base = L.t1_off(sp) * (tov + 1), vt = (int64_t)v_ * tov;
      copyN(KCBJ + base, KJPQ[sp] + (sp ? oos[0] : 0) * n2 + (int64_t)o_ * n + o_, {o_, v_, o_, v_},
            {vt, tov, v_, 1}, {o_ * n2, 1, n2, n}, -1.0, 1.0, s);
    }
    // + 1/2 <kl||cd> t_jl^bd  (DCSD: direct (kc|ld) only)
    G(tov, tov, tov).A(cc ? Icc : Isc, tov, false).B(Tsc, tov, true).C(KCBJ, tov).ab(0.5, 1.0).ring(*this, 0, false, true);
    // Ring_sc = T_sc W_sc
    G(tov, tov, tov).A(Tsc, tov, false).B(KCBJ, tov, true).C(Ring, tov).ring(*this, 1, true, true);
    // spin-flip: Wsf1[(K,c),(J,b)] = -(KJ|bc)~ (sfc x sfc), Wsf2[(k,C),(j,B)] = -(kj|BC)~ (sfr x sfr)
    copyN(Wsf1, KJPQ[0] + oos[0] * n2 + (int64_t)oa * n + oa, {ob, va, ob, va}, {va * sfc, sfc, va, 1},
          {ob * n2, 1, n2, n}, -1.0, 0.0, s);
    copyN(Wsf2, KJPQ[1] + (int64_t)ob * n + ob, {oa, vb, oa, vb}, {vb * sfr, sfr, vb, 1}, {oa * n2, 1, n2, n}, -1.0,
          0.0, s);
    if (cc) {
      // + 1/2 I_sf1 Tsf1 and + 1/2 I_sf2 Tsf1^T
      G(sfc, sfc, sfr).A(Isf1, sfr, false).B(Tsf1, sfc, true).C(Wsf1, sfc).ab(0.5, 1.0).ring(*this, 2, false, true);
      G(sfr, sfr, sfc).A(Isf2, sfc, false).B(Tsf1, sfc, false).C(Wsf2, sfr).ab(0.5, 1.0).ring(*this, 3, false, true);
    }
    G(sfr, sfc, sfc).A(Tsf1, sfc, false).B(Wsf1, sfc, true).C(Rsf1, sfc).ring(*this, 4, true, true);
    G(sfc, sfr, sfr).A(Tsf1, sfc, true).B(Wsf2, sfr, true).C(Rsf2, sfr).ring(*this, 5, true, true);
  } else {
    rfill(Ring, 0.0, tov * tov, s);
    rfill(Rsf1, 0.0, sfr * sfc, s);
    rfill(Rsf2, 0.0, sfr * sfc, s);
  }
  if (mask & (DCSD_TERM_DRIVER | DCSD_TERM_RING)) {
    // equal spins: R2 += P(ij)P(ab) [ 1/2 Dvo + Ring ]
    for (int sp = 0; sp < 2; ++sp) {
      const int o_ = os[sp], v_ = vs[sp];
      const int64_t base = L.t1_off(sp) * (tov + 1), vt = (int64_t)v_ * tov;
      const int64_t vv = (int64_t)v_ * v_;
      const double* src[2] = {Dvo + base, Ring + base};
      const double fac[2] = {0.5, 1.0};
      for (int q = 0; q < 2; ++q) {
        std::initializer_list<int64_t> dst = {o_ * vv, vv, v_, 1};
        copyN(R2ss[sp], src[q], {o_, o_, v_, v_}, dst, {vt, v_, tov, 1}, fac[q], 1.0, s);
        copyN(R2ss[sp], src[q], {o_, o_, v_, v_}, dst, {v_, vt, tov, 1}, -fac[q], 1.0, s);
        copyN(R2ss[sp], src[q], {o_, o_, v_, v_}, dst, {vt, v_, 1, tov}, -fac[q], 1.0, s);
        copyN(R2ss[sp], src[q], {o_, o_, v_, v_}, dst, {v_, vt, 1, tov}, fac[q], 1.0, s);
      }
    }
    // alpha-beta: D + Ring[(ia),(JB)] + Ring[(JB),(ia)] - Rsf2[(J,a),(i,B)] - Rsf1[(i,B),(J,a)]
    std::initializer_list<int64_t> dab = {ab2, (int64_t)va * vb, vb, 1};
    copyN(R2ab, Dvo + ovs[0], {oa, ob, va, vb}, dab, {vta, vb, tov, 1}, 1.0, 1.0, s);
    copyN(R2ab, Ring + ovs[0], {oa, ob, va, vb}, dab, {vta, vb, tov, 1}, 1.0, 1.0, s);
    copyN(R2ab, Ring + ovs[0] * tov, {oa, ob, va, vb}, dab, {va, vtb, 1, tov}, 1.0, 1.0, s);
    copyN(R2ab, Rsf2, {oa, ob, va, vb}, dab, {vb, va * sfr, sfr, 1}, -1.0, 1.0, s);
    copyN(R2ab, Rsf1, {oa, ob, va, vb}, dab, {vb * sfc, va, 1, sfc}, -1.0, 1.0, s);
  }

  // ---- Fock-like terms with the X (vv) and Y (oo) T2*T2 intermediates --------------
  if (mask & DCSD_TERM_FOCK) {
    for (int sp = 0; sp < 2; ++sp) {
      const int o_ = os[sp], v_ = vs[sp];
      const int64_t vv = (int64_t)v_ * v_, ov2 = o_ * vv, oo = oos[sp];
      // X[b][d] = sum (kc|ld)_ss t2ss[k,l,b,c] - sum (kd|L C) t2ab[k,L,b,C]   (alpha)
      copyN(P1, t2ss[sp], {v_, o_, o_, v_}, {oo * v_, o_ * (int64_t)v_, v_, 1}, {v_, ov2, vv, 1}, 1.0, 0.0, s);
      G(v_, v_, oo * v_).A(P1, oo * v_, false).B(QX1[sp], v_, true).C(Xv[sp], v_).run(*this);
      const int64_t kx = oab * vs[1 - sp];  // (k, L, C) for alpha, (l, K, c) for beta
      if (sp == 0)  // t2ab[k,L,b,C] -> [b][k][L][C]
        copyN(P2, t2ab, {va, oa, ob, vb}, {kx, (int64_t)ob * vb, vb, 1}, {vb, ab2, (int64_t)va * vb, 1}, 1.0, 0.0, s);
      else  // t2ab[l,K,c,B] -> [B][l][K][c]
        copyN(P2, t2ab, {vb, oa, ob, va}, {kx, (int64_t)ob * va, va, 1}, {1, ab2, (int64_t)va * vb, vb}, 1.0, 0.0, s);
      G(v_, v_, kx).A(P2, kx, false).B(QX2[sp], v_, true).C(Xv[sp], v_).ab(-1.0, 1.0).run(*this);
      // Y[l][j] = -sum (kc|ld) t2ss[j,k,c,d] + sum (KC|ld) t2ab[j,K,d,C]   (alpha)
      G(o_, o_, ov2).A(QY1[sp], ov2, false).B(t2ss[sp], ov2, false).C(Yo[sp], o_).ab(-1.0, 0.0).run(*this);
      if (sp == 0) {
        G(oa, oa, ab2).A(QY2[0], ab2, false).B(t2ab, ab2, false).C(Yo[0], oa).ab(1.0, 1.0).run(*this);
      } else {
        const int64_t ka = (int64_t)oa * va * vb;
        copyN(P2, t2ab, {ob, oa, va, vb}, {ka, (int64_t)va * vb, vb, 1}, {(int64_t)va * vb, ab2, vb, 1}, 1.0, 0.0,
              s);  // [J][k][c][D]
        G(ob, ob, ka).A(QY2[1], ka, false).B(P2, ka, false).C(Yo[1], ob).ab(1.0, 1.0).run(*this);
      }
      // F~vv = f~_vv + s X,  F~oo = f~_oo + s Y
      copyN(Fvv[sp], ft[sp] + (int64_t)o_ * n + o_, {v_, v_}, {v_, 1}, {n, 1}, 1.0, 0.0, s);
      raxpby(Fvv[sp], Xv[sp], sdc, 1.0, vv, s);
      copyN(Foo[sp], ft[sp], {o_, o_}, {o_, 1}, {n, 1}, 1.0, 0.0, s);
      raxpby(Foo[sp], Yo[sp], sdc, 1.0, oo, s);
    }
    for (int sp = 0; sp < 2; ++sp) {
      const int o_ = os[sp], v_ = vs[sp];
      const int64_t vv = (int64_t)v_ * v_, ov2 = o_ * vv;
      if (o_ == 0) continue;
      // P(ab) sum_d t_ij^ad F_bd
      G(oos[sp] * v_, v_, v_).A(t2ss[sp], v_, false).B(Fvv[sp], v_, false).C(P1, v_).run(*this);
      copyN(R2ss[sp], P1, {o_, o_, v_, v_}, {ov2, vv, v_, 1}, {ov2, vv, v_, 1}, 1.0, 1.0, s);
      copyN(R2ss[sp], P1, {o_, o_, v_, v_}, {ov2, vv, v_, 1}, {ov2, vv, 1, v_}, -1.0, 1.0, s);
      // -P(ij) sum_l t_il^ab F_lj
      G(o_, vv, o_).A(Foo[sp], o_, true).B(t2ss[sp], vv, true).C(P1, vv).batch(o_, 0, ov2, ov2).run(*this);
      copyN(R2ss[sp], P1, {o_, o_, v_, v_}, {ov2, vv, v_, 1}, {ov2, vv, v_, 1}, -1.0, 1.0, s);
      copyN(R2ss[sp], P1, {o_, o_, v_, v_}, {ov2, vv, v_, 1}, {vv, ov2, v_, 1}, 1.0, 1.0, s);
    }
    // alpha-beta
    const int64_t vab = (int64_t)va * vb;
    G(oab * va, vb, vb).A(t2ab, vb, false).B(Fvv[1], vb, false).C(R2ab, vb).ab(1.0, 1.0).run(*this);
    G(va, vb, va).A(Fvv[0], va, false).B(t2ab, vb, true).C(R2ab, vb).ab(1.0, 1.0).batch(oab, 0, vab, vab).run(*this);
    G(ob, vab, ob).A(Foo[1], ob, true).B(t2ab, vab, true).C(R2ab, vab).ab(-1.0, 1.0).batch(oa, 0, ab2, ab2).run(*this);
    G(oa, ab2, oa).A(Foo[0], oa, true).B(t2ab, ab2, true).C(R2ab, ab2).ab(-1.0, 1.0).run(*this);
  }

  // ---- hole-hole ladder -----------------------------------------------------------
  if (mask & DCSD_TERM_HH) {
    for (int blk = 0; blk < 3; ++blk) {
      const int s1 = blk == 1 ? 1 : 0, s3 = blk == 0 ? 0 : 1;
      const int o1 = os[s1], o3 = os[s3];
      const int64_t o13 = (int64_t)o1 * o3, v13 = (int64_t)vs[s1] * vs[s3];
      if (o13 == 0) continue;
      // Whh[(k,l),(i,j)] = (ki|lj)~  (k, i of spin s1; l, j of spin s3)
      copyN(Whh, OOOO + (s1 ? oos[0] : 0) * too2 + (s3 ? oos[0] : 0), {o1, o3, o1, o3},
            {o3 * o13, o13, o3, 1}, {o1 * too2, o3, too2, 1}, 1.0, 0.0, s);
      const double* t2b = blk == 0 ? t2aa : (blk == 1 ? t2bb : t2ab);
      double* Rb2 = blk == 0 ? R2ss[0] : (blk == 1 ? R2ss[1] : R2ab);
      if (cc)  // + 1/2 <kl||cd> t_ij^cd  ->  sum_cd (kc|ld) t_ij^cd (x 1/2 for equal spins)
        G(o13, o13, v13).A(Ikl[blk], v13, false).B(t2b, v13, false).C(Whh, o13).ab(blk == 2 ? 1.0 : 0.5, 1.0).run(*this);
      G(o13, v13, o13).A(Whh, o13, true).B(t2b, v13, true).C(Rb2, v13).ab(1.0, 1.0).run(*this);
    }
  }

  // ---- particle-particle ladder (DF-assembled, T1 back-transformed) -----------------
  if (mask & DCSD_TERM_PP) {
    const int64_t vu2 = (int64_t)vu * vu;
    const bool low = prec_now != DCSD_PREC_FP64;
    const bool delta = low && mode == DELTA && ladder_ref;  // contract lp(tau - tau_r), add L(tau_r)
    ladder_stack(Tstack, t2aa, t2bb, t2ab, pair_i, pair_j, L, vu, rows_all, s);
    // Under a tape the whole batch loop is one operation: its adjoint
    // recomputes each integral batch instead of storing it.
    Tape* const tape_here = t_tape;
    if (tape_here) {
      TapeOp op;
      op.kind = OP_STACK;
      op.dst = Tstack;
      op.src = t2aa;
      tape_op(op);
      if (low) throw ArgError("the adjoint runs in FP64 only");
      op = TapeOp();
      op.kind = OP_LADDER;
      op.dst = Rp;
      op.src = Tstack;
      op.src2 = Bl;
      op.val[0] = tape_value(Tstack, rows_all * vu2);
      tape_op(op);
      t_tape = nullptr;
    }
    if (low) lp_convert(prec_now, TstackL, kp, Tstack, delta ? TstackR : nullptr, rows_all, vu2, vu2, 1, s);
    int64_t batch = 0;
    for (int p0 = 0; p0 < n; p0 += lb) {
      const int np = std::min(lb, n - p0);
      for (int q0 = p0; q0 < n; q0 += lb, ++batch) {
        const int nq = std::min(lb, n - q0);
        const bool diag = q0 == p0;
        // low precision with the cache: the batch's slot, assembled on the first evaluation only
        void* const V2b = low && lcache ? (char*)lcache + batch * lcache_slot * lp_size(prec_now) : V2L;
        double* const V2d = !low && lcache64 ? lcache64 + batch * lcache64_slot : V2;
        if (low ? !lcache_valid : !lcache64_valid) {
          hipEvent_t ev0;
          const int rec = tbegin(&ev0);
          if (low)
            lp_pairs(prec_now, BlT, ldk, NA, vu, p0, np, q0, nq, kp, V2b, s);
          else
            gemm_f64_pairs(Bl, (int64_t)n * vu, vu, NA, p0, np, q0, nq, V2d, s);
          // algorithmic flops: a diagonal batch needs its np (np + 1) / 2 distinct pairs
          const double pairs = diag ? 0.5 * np * (np + 1.0) : (double)np * nq;
          if (rec) tend(ev0, 2.0 * pairs * vu * (double)vu * (double)NA, 0);
        }
        const int64_t M = diag ? rows_main : rows_all;
        const int64_t N = (int64_t)np * nq;
        const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
        int ks = (int)std::min<int64_t>(split_cap, std::max<int64_t>(1, 512 / std::max<int64_t>(tiles, 1)));
        ks = (int)std::min<int64_t>(ks, std::max<int64_t>(1, vu2 / 1024));
        hipEvent_t ev0;
        const int rec = tbegin(&ev0);
        if (low) {
          LpGemm q;
          q.precision = prec_now;
          q.M = M; q.N = N; q.K = vu2;
          q.A = TstackL; q.lda = kp; q.B = V2b; q.ldb = kp;
          q.C = Rb; q.ldc = N;
          q.ks = ks; q.work = lwork;
          q.k_padded = true;
          // BF16: 256 x 256 tiles, split about 256 ways (one workgroup per compute unit)
          if (prec_now == DCSD_PREC_BF16 && M >= 256 && N >= 256) {
            const int64_t t256 = ((M + 255) / 256) * ((N + 255) / 256);
            q.ks = (int)std::min<int64_t>(split_cap, std::max<int64_t>(1, 256 / t256));
            q.ks = (int)std::min<int64_t>(q.ks, std::max<int64_t>(1, vu2 / 1024));
            q.big_tiles = true;
          }
          lp_gemm(q, s);
        } else {
          G(M, N, vu2).A(Tstack, vu2, false).B(V2d, vu2, false).C(Rb, N).split(ks, split).run(*this);
        }
        if (rec) tend(ev0, 2.0 * (double)M * (double)N * (double)vu2, 1);
        ladder_scatter(Rp, Rb, M, rows_main, oab, n, p0, np, q0, nq, diag, s);
      }
    }
    if (low && lcache) lcache_valid = true;
    if (!low && lcache64) lcache64_valid = true;
    if (mode == RECORD) {
      rcopy(TstackR, Tstack, rows_all * vu2, s);
      rcopy(RpR, Rp, rows_main * n2, s);
      ladder_ref = true;
    } else if (delta) {
      raxpby(Rp, RpR, 1.0, 1.0, rows_main * n2, s);
    }
    t_tape = tape_here;
    if (t_tape) {
      TapeOp op;
      op.kind = OP_MTRANS;
      op.dst = R;
      op.src = Rp;
      op.src2 = Tw;
      op.val[0] = tape_value(Rp, rows_main * n2);
      op.val[1] = tape_value(Tw, 2 * ov);
      tape_op(op);
    }
    ladder_mtransform(R2ss[0], R2ss[1], R2ab, Smt, Rp, t1[0], t1[1], pair_i, pair_j, rows_main, L, s);
  }

  // ---- coupling of the two determinants (2D methods only) ---------------------------
  const bool two_det = method_ab(cfg.method) && !method_fr(cfg.method);
  if (two_det)
    rcopy(scal, R + ab_pos, 1, s);  // W
  else
    rfill(scal, 0.0, 1, s);  // W = 0: fixed-reference and high-spin methods
  if (two_det && (mask & DCSD_TERM_COUPLING)) {
    if (t_tape) {
      TapeOp op;
      op.kind = OP_COUPLING;
      op.dst = R;
      op.src = Tw;
      op.src2 = scal;
      op.val[0] = tape_value(Tw, total);
      op.val[1] = tape_value(scal, 1);
      tape_op(op);
    }
    coupling_apply(coup_launch, Tw, R, scal, nc, nv, s);
  }
  // the Phi_A -> Phi_B double is not solved for (its residual is W in the two-determinant
  // methods; the fixed-reference methods hold the amplitude fixed)
  if (method_ab(cfg.method)) rfill(R + ab_pos, 0.0, 1, s);
  if (rec_res) tend(ev_res, 0.0, 2);
  if (W_host) {
    DCSD_HIP(hipMemcpyAsync(W_host, scal, sizeof(double), hipMemcpyDeviceToHost, s));
    DCSD_HIP(hipStreamSynchronize(s));
  }
}

int Ctx::tbegin(hipEvent_t* ev) {
  if (!timing) return 0;
  if (pool_next + 2 > pool.size()) {  // grow the pool: no interval is dropped
    const size_t old = pool.size(), grown = std::max<size_t>(1024, 2 * old);
    pool.resize(grown);
    for (size_t k = old; k < grown; ++k) DCSD_HIP(hipEventCreate(&pool[k]));
  }
  *ev = pool[pool_next++];
  DCSD_HIP(hipEventRecord(*ev, s));
  return 1;
}

void Ctx::tend(hipEvent_t a, double flops, int cls) {
  hipEvent_t b = pool[pool_next++];
  DCSD_HIP(hipEventRecord(b, s));
  recs.push_back({a, b, flops, cls});
}

// dE_A and W of amplitudes T: W from an FP64 residual into the solver's work
// vector (the fixed-reference methods have W = 0 and need none).
void Ctx::energies(const double* T, dcsd_energies* out) {
  double W = 0.0;
  if (method_ab(cfg.method) && !method_fr(cfg.method)) residual(T, Rw, &W, DCSD_PREC_FP64, PLAIN);
  const double e = energy_A(T);
  out->dE_A = e;
  out->W = W;
  state_energies(cfg.method, e, W, out->E_S, out->E_T);
  out->E_ref_A = e_ref;
}

double Ctx::energy_A(const double* T) {
  rcopy(Tw, T, total, s);
  if (method_ab(cfg.method)) {
    const int64_t ab_pos = L.t2_off(2) + (((int64_t)nc * os[1] + nc) * vs[0] + 0) * vs[1] + 0;
    rfill(Tw + ab_pos, ab_amplitude(cfg.method), 1, s);
  }
  energy(Tw, Isc, f[0], f[1], L, scal + 2, part, s);
  double e = 0.0;
  DCSD_HIP(hipMemcpyAsync(&e, scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  DCSD_HIP(hipStreamSynchronize(s));
  return e;
}

}  // namespace dcsd
