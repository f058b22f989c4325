// Recording-aware helpers shared by the residual and its adjoint (internal):
// the FP64 GEMM builder and the strided copy.  While a tape is active every
// call is recorded before it is executed.
#pragma once

#include <algorithm>
#include <initializer_list>

#include "ctx.h"
#include "tape.h"

namespace dcsd {

inline void copyN(double* dst, const double* src, std::initializer_list<int64_t> dims,
                  std::initializer_list<int64_t> ds, std::initializer_list<int64_t> ss, double alpha, double beta,
                  hipStream_t s) {
  Strided st;
  st.nd = (int)dims.size();
  int d = 0;
  for (auto x : dims) st.dims[d++] = x;
  d = 0;
  for (auto x : ds) st.ds[d++] = x;
  d = 0;
  for (auto x : ss) st.ss[d++] = x;
  if (t_tape) tape_copy(dst, src, st, alpha, beta);
  strided_copy(dst, src, st, alpha, beta, s);
}

struct G {
  GemmArgs a;
  G(int64_t M, int64_t N, int64_t K) {
    a.M = M;
    a.N = N;
    a.K = K;
  }
  G& A(const double* p, int64_t ld, bool mc) { a.A = p; a.lda = ld; a.a_mc = mc; return *this; }
  G& B(const double* p, int64_t ld, bool nc) { a.B = p; a.ldb = ld; a.b_nc = nc; return *this; }
  G& C(double* p, int64_t ld, bool nc = true) { a.C = p; a.ldc = ld; a.c_nc = nc; return *this; }
  G& ab(double al, double be) { a.alpha = al; a.beta = be; return *this; }
  G& batch(int64_t b, int64_t sA, int64_t sB, int64_t sC) { a.batch = b; a.sA = sA; a.sB = sB; a.sC = sC; return *this; }
  G& split(int k, double* w) { a.ksplit = k; a.work = w; return *this; }
  // Few output tiles and a long K: split K across workgroups into the context's
  // workspace (fixed-order reduction, deterministic), aiming at about 1024
  // workgroups of the tile size that will run (128 when both M and N reach it;
  // the 64-wide kernel is capped at 256 splits, beyond which it ran slower).
  void run(Ctx& c) {
    // a small output over a long K: dot products streamed over K (outside a tape, whose
    // adjoint replays the recorded GEMMs)
    if (!t_tape && a.ksplit == 1 && gemm_f64_small(a, c.gws, c.gws_cap, c.s)) return;
    const double* g_ws = c.gws;
    const int64_t g_ws_cap = c.gws_cap;
    if (a.ksplit == 1 && g_ws && a.K >= 2048) {
      const int64_t T = a.M >= 128 && a.N >= 128 ? 128 : 64;
      const int64_t tiles = ((a.M + T - 1) / T) * ((a.N + T - 1) / T) * a.batch;
      if (tiles < 256) {
        int64_t ks = std::min<int64_t>(T == 128 ? 1024 : 256, std::max<int64_t>(1, 1024 / tiles));
        ks = std::min<int64_t>(ks, a.K / 512);
        const int64_t span = (a.batch - 1) * a.sC + (a.c_nc ? (a.M - 1) * a.ldc + a.N : (a.N - 1) * a.ldc + a.M);
        while (ks > 1 && ks * span > g_ws_cap) ks /= 2;
        if (ks > 1) {
          a.ksplit = (int)ks;
          a.work = c.gws;
        }
      }
    }
    a.pad = c.pws;
    a.pad_cap = c.pws_cap;
    if (t_tape) tape_gemm(a);
    gemm_f64(a, c.s);
  }
  // fp64_plain: FP64 outside the delta form (low precision only for the changes since a
  // refresh point)
  void ring(Ctx& c, int site, bool a_var, bool b_var, bool fp64_plain = false);
  void lp_product(Ctx& c, const double* A, const double* Asub, const double* B, const double* Bsub,
                  double beta = 1.0);
};

}  // namespace dcsd
