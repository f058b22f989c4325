// Reverse mode through the residual, the energy and the constants built from
// (B, F): tape recording, the backward sweep with one hand-written adjoint
// per recorded operation, and the lambda equations of the energy Lagrangian.
//
// With E = eS E_S + eT E_T = a dE_A + b W (a = eS + eT, b = eS - eT) and the
// amplitude equations R(T; B, F) = 0 (the A->B element excluded), the
// Lagrangian L = a dE_A + b W + lambda . R is stationary in T when
//   (dR/dT)^T lambda + a d(dE_A)/dT + b dW/dT = 0,
// solved by the same Jacobi/DIIS iteration as the amplitudes (one backward
// sweep per iteration).  The equal-spin amplitudes are stored in full but only
// their antisymmetric combinations are unknowns: the equations are the
// projections of the cotangent on those, and lambda is kept antisymmetric
// (then lambda . dR/dB over all stored elements is the multiplier sum over the
// independent equations, R being antisymmetric).  dE/dB and dE/dF are then dL/dB and dL/dF at the
// converged lambda: one more sweep that also runs through the constants.
#include <algorithm>
#include <cmath>

#include "ops.h"

namespace dcsd {

// ---- tape -------------------------------------------------------------------------
void Tape::clear() {
  for (double* p : scratch) (void)hipFree(p);
  scratch.clear();
  snaps.clear();
  ops.clear();
  temp_need = 0;
  arena_used = 0;
  need = 0;
}

namespace {
Ctx& tctx() { return *t_ctx; }

int buf_of(const void* p) {
  const int id = tctx().find_buf(p);
  if (id < 0) throw ArgError("tape: operand outside the registered device arrays");
  tctx().bufs[id].used = true;
  return id;
}
void bump(const void* p) { tctx().bufs[buf_of(p)].version++; }

int64_t span_a(const GemmArgs& g) {
  return (g.batch - 1) * g.sA + (g.a_mc ? (g.M - 1) + (g.K - 1) * g.lda : (g.M - 1) * g.lda + (g.K - 1)) + 1;
}
int64_t span_b(const GemmArgs& g) {
  return (g.batch - 1) * g.sB + (g.b_nc ? (g.N - 1) + (g.K - 1) * g.ldb : (g.N - 1) * g.ldb + (g.K - 1)) + 1;
}
}  // namespace

const double* tape_value(const double* p, int64_t count) {
  Ctx& c = tctx();
  Tape& t = *t_tape;
  const int id = buf_of(p);
  Ctx::Buf& b = c.bufs[id];
  if (b.constant) return p;
  const double* hi = p + count;
  if (p < b.p || hi > b.p + b.n) throw ArgError("tape: operand range outside its array");
  for (const Snapshot& sn : t.snaps)
    if (sn.buf == id && sn.version == b.version && sn.lo <= p && hi <= sn.hi) return sn.copy + (p - sn.lo);
  double* cp = nullptr;
  const int64_t padded = (count + 31) / 32 * 32;  // 256-byte granules
  t.need += padded;
  if (t.arena) {
    if (t.arena_used + padded > t.arena_cap)
      throw ArgError("adjoint: the tape needs more snapshot memory than dcsd_init reserved");
    cp = t.arena + t.arena_used;
    t.arena_used += padded;
  } else {
    // only while dcsd_init sizes the reservation
    ++c.alloc_calls;
    if (hipMalloc((void**)&cp, (size_t)count * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    t.scratch.push_back(cp);
  }
  DCSD_HIP(hipMemcpyAsync(cp, p, (size_t)count * sizeof(double), hipMemcpyDeviceToDevice, c.s));
  t.snaps.push_back({id, b.version, p, hi, cp});
  return cp;
}

void tape_gemm(const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  TapeOp op;
  op.kind = OP_GEMM;
  op.g = g;
  op.g.ksplit = 1;
  op.g.work = nullptr;
  if (g.K > 0) {
    op.Aval = tape_value(g.A, span_a(g));
    op.Bval = tape_value(g.B, span_b(g));
  }
  if (g.batch > 1 && g.sA == 0) t_tape->temp_need = std::max(t_tape->temp_need, g.batch * g.M * g.K);
  if (g.batch > 1 && g.sB == 0) t_tape->temp_need = std::max(t_tape->temp_need, g.batch * g.K * g.N);
  buf_of(g.C);
  t_tape->ops.push_back(op);
  bump(g.C);
}

void tape_copy(double* dst, const double* src, const Strided& st, double alpha, double beta) {
  TapeOp op;
  op.kind = OP_COPY;
  op.dst = dst;
  op.src = src;
  op.st = st;
  op.alpha = alpha;
  op.beta = beta;
  buf_of(src);
  t_tape->ops.push_back(op);
  bump(dst);
}

void tape_simple(int kind, double* dst, const double* src, int64_t n, double a, double b) {
  TapeOp op;
  op.kind = kind;
  op.dst = dst;
  op.src = src;
  op.n = n;
  op.alpha = a;
  op.beta = b;
  if (src) buf_of(src);
  t_tape->ops.push_back(op);
  bump(dst);
}

void tape_op(const TapeOp& op) {
  if (op.src) buf_of(op.src);
  if (op.src2) buf_of(op.src2);
  t_tape->ops.push_back(op);
  bump(op.dst);
}

// ---- buffer registry ------------------------------------------------------------------
void Ctx::reg(double* p, int64_t count, bool /*owned*/) {
  Buf b;
  b.p = p;
  b.n = count;
  auto it = std::upper_bound(bufs.begin(), bufs.end(), p, [](const double* x, const Buf& y) { return x < y.p; });
  bufs.insert(it, b);
}

int Ctx::find_buf(const void* p) const {
  const double* q = (const double*)p;
  auto it = std::upper_bound(bufs.begin(), bufs.end(), q, [](const double* x, const Buf& y) { return x < y.p; });
  if (it == bufs.begin()) return -1;
  --it;
  if (q >= it->p + it->n) return -1;
  return (int)(it - bufs.begin());
}

double* Ctx::bar(const void* p) {
  const int id = find_buf(p);
  if (id < 0 || !bufs[id].bar) throw ArgError("adjoint: no cotangent array for an operand");
  return bufs[id].bar + ((const double*)p - bufs[id].p);
}

bool Ctx::wants(const void* p, bool params) {
  const int id = find_buf(p);
  return id >= 0 && bufs[id].bar && (params || !bufs[id].constant);
}

// ---- set-up and recording ---------------------------------------------------------
void Ctx::adj_setup() {
  if (Tin) return;
  Tin = alloc(total);
  Rt = alloc(total);
  lam = alloc(total);
}

// Reserves everything the adjoint calls need (called by dcsd_init): one
// recording at T = 0 allocates the cotangent arrays and the sweep's work space
// and measures the operand snapshots of each tape, which then move into one
// arena per tape.  The tapes' operation sequence and snapshot sizes depend only
// on the sizes, the method and the term mask, not on the amplitude values.
void Ctx::adj_reserve() {
  adj_setup();
  fill(Tin, 0.0, total, s);
  record(Tin);
  for (Tape* t : {&tape_init, &tape_res}) {
    const int64_t need = t->need;
    t->clear();
    t->arena = (double*)alloc_raw((size_t)std::max<int64_t>(need, 32) * sizeof(double));
    t->arena_cap = std::max<int64_t>(need, 32);
  }
  adj_ready = true;
  DCSD_HIP(hipStreamSynchronize(s));
}

void Ctx::record(const double* T) {
  if (!Tin) throw ArgError("adjoint memory was not reserved (set cfg.adjoint at dcsd_init)");
  if (T != Tin) DCSD_HIP(hipMemcpyAsync(Tin, T, total * sizeof(double), hipMemcpyDeviceToDevice, s));
  tape_init.clear();
  tape_res.clear();
  for (auto& b : bufs) {
    b.constant = false;
    b.version = 0;
  }
  const int iB = find_buf(B), iF = find_buf(F);
  t_ctx = this;
  // constants from (B, F): only the inputs are fixed while they are rebuilt
  bufs[iB].constant = bufs[iF].constant = true;
  t_tape = &tape_init;
  try {
    build_constants(false);
  } catch (...) {
    t_tape = nullptr;
    throw;
  }
  // the residual at T with everything built from (B, F) held fixed
  const double* consts[] = {Bs[1], h[0], h[1], f[0], f[1], Isc, QX1[0], QX1[1], QX2[0], QX2[1], QY1[0], QY1[1],
                            QY2[0], QY2[1], Ikl[0], Ikl[1], Ikl[2], Icc, Isf1, Isf2, Bl, Jpq, Kpq};
  for (const double* p : consts)
    if (p) bufs[find_buf(p)].constant = true;
  t_tape = &tape_res;
  try {
    residual(Tin, Rt, nullptr, DCSD_PREC_FP64, PLAIN);
    TapeOp op;
    op.kind = OP_ENERGY;
    op.dst = scal + 2;
    op.src = Tw;
    op.val[0] = tape_value(Tw, total);
    tape_op(op);
    energy(Tw, Isc, f[0], f[1], L, scal + 2, part, s);
    for (const double* p : {(const double*)Isc, (const double*)f[0], (const double*)f[1]}) buf_of(p);
  } catch (...) {
    t_tape = nullptr;
    throw;
  }
  t_tape = nullptr;
  // cotangent arrays of everything the tapes touch, and the sweep's work space
  std::vector<std::pair<double*, int64_t>> need_bar;
  for (const auto& b : bufs)
    if (b.used && !b.bar) need_bar.push_back({b.p, b.n});
  const int64_t vu2 = (int64_t)vu * vu;
  int64_t need = std::max<int64_t>(2 * (int64_t)lb * lb * vu2, rows_main * ((int64_t)v * v + (int64_t)n * v));
  need = std::max(need, std::max(tape_init.temp_need, tape_res.temp_need));
  if (adj_ready) {  // after dcsd_init nothing may be allocated
    if (!need_bar.empty() || need > temp_cap)
      throw ArgError("adjoint: the tape needs memory that dcsd_init did not reserve (term_mask changed?)");
    return;
  }
  for (const auto& x : need_bar) {
    double* q = alloc(x.second);  // registers q: find the owner afterwards
    bufs[find_buf(x.first)].bar = q;
  }
  if (need > temp_cap) {
    temp = alloc(need);
    temp_cap = need;
  }
  DCSD_HIP(hipStreamSynchronize(s));
}

// ---- the sweep ------------------------------------------------------------------------
void Ctx::sweep(const double* Rbar, double Wbar, double Ebar, bool params) {
  for (auto& b : bufs)
    if (b.bar) fill(b.bar, 0.0, b.n, s);
  axpby(bar(Rt), Rbar, 1.0, 0.0, total, s);
  fill(bar(scal), Wbar, 1, s);
  fill(bar(scal) + 2, Ebar, 1, s);
  for (auto it = tape_res.ops.rbegin(); it != tape_res.ops.rend(); ++it) adjoint_op(*it, params);
  if (params)
    for (auto it = tape_init.ops.rbegin(); it != tape_init.ops.rend(); ++it) adjoint_op(*it, true);
}

namespace {
// Abar += alpha Cbar B^T and Bbar += alpha A^T Cbar for the product C = alpha A B (+ beta C)
// described by g (cotangents in the layouts of A, B, C).  Batches that share one
// operand (stride 0) go through `work` (per-batch products, then summed).
void gemm_vjp(Ctx& c, const GemmArgs& g, const double* Aval, const double* Bval, const double* Cbar, double* Abar,
              double* Bbar, double* work) {
  if (Abar) {
    G h(g.M, g.K, g.N);
    h.A(Cbar, g.ldc, !g.c_nc).B(Bval, g.ldb, !g.b_nc).ab(g.alpha, 1.0);
    if (g.batch > 1 && g.sA == 0) {
      h.C(work, g.K, true).ab(g.alpha, 0.0).batch(g.batch, g.sC, g.sB, g.M * g.K);
      h.run(c);
      batch_reduce(Abar, work, g.batch, g.M * g.K, (int)g.M, (int)g.K, g.K, g.lda, g.a_mc, 1.0, c.s);
    } else {
      h.C(Abar, g.lda, !g.a_mc).batch(g.batch, g.sC, g.sB, g.sA);
      h.run(c);
    }
  }
  if (Bbar) {
    G h(g.K, g.N, g.M);
    h.A(Aval, g.lda, !g.a_mc).B(Cbar, g.ldc, g.c_nc).ab(g.alpha, 1.0);
    if (g.batch > 1 && g.sB == 0) {
      h.C(work, g.N, true).ab(g.alpha, 0.0).batch(g.batch, g.sA, g.sC, g.K * g.N);
      h.run(c);
      batch_reduce(Bbar, work, g.batch, g.K * g.N, (int)g.K, (int)g.N, g.N, g.ldb, !g.b_nc, 1.0, c.s);
    } else {
      h.C(Bbar, g.ldb, g.b_nc).batch(g.batch, g.sA, g.sC, g.sB);
      h.run(c);
    }
  }
}
// dst[pattern] *= factor over a strided pattern (in place)
void scale_pattern(double* p, const Strided& st_in, double factor, hipStream_t s) {
  Strided st = st_in;
  for (int d = 0; d < 6; ++d) st.ss[d] = st.ds[d];
  strided_copy(p, p, st, factor, 0.0, s);
}
}  // namespace

void Ctx::gemm_adjoint(const TapeOp& op, bool params) {
  const GemmArgs& g = op.g;
  double* Cb = bar(g.C);
  if (g.K > 0) {
    double* Ab = wants(g.A, params) ? bar(g.A) : nullptr;
    double* Bb = wants(g.B, params) ? bar(g.B) : nullptr;
    if (temp_cap < std::max(tape_init.temp_need, tape_res.temp_need)) throw ArgError("adjoint: work space too small");
    gemm_vjp(*this, g, op.Aval, op.Bval, Cb, Ab, Bb, temp);
  }
  if (g.beta != 1.0) {
    Strided st;
    st.nd = 3;
    st.dims[0] = g.batch;
    st.dims[1] = g.M;
    st.dims[2] = g.N;
    st.ds[0] = g.sC;
    st.ds[1] = g.c_nc ? g.ldc : 1;
    st.ds[2] = g.c_nc ? 1 : g.ldc;
    scale_pattern(Cb, st, g.beta, s);
  }
}

void Ctx::ladder_adjoint(const TapeOp& op, bool params) {
  const int64_t NA = naux, vu2 = (int64_t)vu * vu, o2 = (int64_t)o * o;
  const double* Tst = op.val[0];
  double* Tst_bar = bar(Tstack);
  const double* Rp_bar = bar(Rp);
  double* Bl_bar = params && wants(Bl, true) ? bar(Bl) : nullptr;
  double* V2bar = temp;
  double* V2plain = temp + (int64_t)lb * lb * vu2;
  for (int p0 = 0; p0 < n; p0 += lb) {
    const int np = std::min(lb, n - p0);
    for (int q0 = p0; q0 < n; q0 += lb) {
      const int nq = std::min(lb, n - q0);
      const bool diag = q0 == p0;
      const int64_t M = diag ? rows_main : rows_all;
      const int64_t N = (int64_t)np * nq;
      gemm_f64_pairs(Bl, (int64_t)n * vu, vu, NA, p0, np, q0, nq, V2, s);  // recomputed integrals
      ladder_scatter_adj(Rb, Rp_bar, M, rows_main, o2, n, p0, np, q0, nq, diag, s);
      // forward: Rb = Tstack[0:M] V2^T
      GemmArgs fg;
      fg.M = M; fg.N = N; fg.K = vu2;
      fg.A = Tstack; fg.lda = vu2; fg.a_mc = false;
      fg.B = V2; fg.ldb = vu2; fg.b_nc = false;
      fg.C = Rb; fg.ldc = N; fg.c_nc = true;
      if (Bl_bar) fill(V2bar, 0.0, N * vu2, s);
      gemm_vjp(*this, fg, Tst, V2, Rb, Tst_bar, Bl_bar ? V2bar : nullptr, nullptr);
      if (Bl_bar) {
        // V2bar[(p,q)][c][d] -> plain [(p,c)][(q,d)]
        Strided st;
        st.nd = 4;
        const int64_t dims[4] = {np, vu, nq, vu};
        const int64_t ds[4] = {(int64_t)vu * nq * vu, (int64_t)nq * vu, vu, 1};
        const int64_t ss[4] = {(int64_t)nq * vu2, vu, vu2, 1};
        for (int d = 0; d < 4; ++d) {
          st.dims[d] = dims[d];
          st.ds[d] = ds[d];
          st.ss[d] = ss[d];
        }
        strided_copy(V2plain, V2bar, st, 1.0, 0.0, s);
        // forward: V2[(p,c),(q,d)] = sum_P Bl[P][p0+p][c] Bl[P][q0+q][d]
        GemmArgs ag;
        ag.M = (int64_t)np * vu; ag.N = (int64_t)nq * vu; ag.K = NA;
        ag.A = Bl + (int64_t)p0 * vu; ag.lda = (int64_t)n * vu; ag.a_mc = true;
        ag.B = Bl + (int64_t)q0 * vu; ag.ldb = (int64_t)n * vu; ag.b_nc = true;
        ag.C = V2plain; ag.ldc = (int64_t)nq * vu; ag.c_nc = true;
        gemm_vjp(*this, ag, ag.A, ag.B, V2plain, Bl_bar + (int64_t)p0 * vu, nullptr, nullptr);
        gemm_vjp(*this, ag, ag.A, ag.B, V2plain, nullptr, Bl_bar + (int64_t)q0 * vu, nullptr);
      }
    }
  }
  fill(bar(Rp), 0.0, rows_main * n2, s);  // Rp was overwritten by the forward operation
}

void Ctx::adjoint_op(const TapeOp& op, bool params) {
  switch (op.kind) {
    case OP_GEMM:
      gemm_adjoint(op, params);
      break;
    case OP_COPY: {
      if (wants(op.src, params)) {
        Strided st = op.st;
        for (int d = 0; d < 6; ++d) std::swap(st.ds[d], st.ss[d]);
        strided_copy(bar(op.src), bar(op.dst), st, op.alpha, 1.0, s);
      }
      if (op.beta != 1.0) scale_pattern(bar(op.dst), op.st, op.beta, s);
      break;
    }
    case OP_FILL:
    case OP_UPLOAD:
      fill(bar(op.dst), 0.0, op.n, s);
      break;
    case OP_AXPBY:
      if (wants(op.src, params)) axpby(bar(op.src), bar(op.dst), op.alpha, 1.0, op.n, s);
      if (op.beta != 1.0) axpby(bar(op.dst), bar(op.dst), op.beta, 0.0, op.n, s);
      break;
    case OP_MEMCPY:
      if (wants(op.src, params)) axpby(bar(op.src), bar(op.dst), 1.0, 1.0, op.n, s);
      fill(bar(op.dst), 0.0, op.n, s);
      break;
    case OP_SWAPTU:
      if (wants(op.src, params)) swap_tu_adj(bar(op.src), bar(op.dst), op.n, op.ints[0], op.ints[1], s);
      fill(bar(op.dst), 0.0, op.n * (int64_t)op.ints[0] * op.ints[0], s);
      break;
    case OP_JVEC:
      if (wants(op.src, params)) jvector_adj(bar(op.src), bar(op.src2), bar(op.dst), op.n, op.ints[0], op.ints[1], s);
      fill(bar(op.dst), 0.0, op.n, s);
      break;
    case OP_BREDUCE:
      if (wants(op.src, params))
        batch_reduce_adj(bar(op.src), bar(op.dst), op.n, op.i64[0], op.ints[0], op.ints[1], op.i64[1], op.i64[2],
                         op.ints[2] != 0, op.alpha, s);
      break;
    case OP_STACK: {
      const int64_t s2l = ov * ov;
      double* t2b = bar(op.src);  // t2aa inside the amplitude copy
      ladder_stack_adj(t2b, t2b + s2l, t2b + 2 * s2l, bar(op.dst), o, v, vu, npair, s);
      fill(bar(op.dst), 0.0, rows_all * (int64_t)vu * vu, s);
      break;
    }
    case OP_LADDER:
      ladder_adjoint(op, params);
      break;
    case OP_MTRANS: {
      const int64_t s2l = ov * ov, o2 = (int64_t)o * o;
      const double* Rb = bar(op.dst);
      ladder_mtransform_adj(bar(op.src), bar(op.src2), Rb + 2 * ov, Rb + 2 * ov + s2l, Rb + 2 * ov + 2 * s2l,
                            op.val[0], op.val[1], op.val[1] + ov, pair_i, pair_j, rows_main, o2, npair, n, nc, o, v,
                            temp, Smt, temp + rows_main * (int64_t)v * v, s);
      break;
    }
    case OP_COUPLING:
      coupling_apply_adj(coup_launch, op.val[0], bar(op.src), bar(op.dst), op.val[1], bar(op.src2), nc, nv, s);
      break;
    case OP_ENERGY:
      energy_adj(bar(op.src), params ? bar(Isc) : nullptr, params ? bar(f[0]) : nullptr,
                 params ? bar(f[1]) : nullptr, op.val[0], Isc, f[0], f[1], bar(op.dst), o, v, n, s);
      fill(bar(op.dst), 0.0, 1, s);
      break;
    default:
      throw ArgError("adjoint: unknown tape operation");
  }
}

// ---- lambda equations -------------------------------------------------------------
int Ctx::lambda_solve(double a, double b, double* L, dcsd_report* rep) {
  const int m = cfg.diis_dim;
  std::vector<double> gram((size_t)std::max(m, 1) * std::max(m, 1), 0.0);
  std::vector<int> order;
  int count = 0;
  dcsd_report r{};
  for (int it = 0; it < cfg.max_iter; ++it) {
    sweep(L, b, a, false);
    // the residual of the lambda equations: the amplitude cotangent projected
    // on the independent (antisymmetric) amplitudes; lambda stays antisymmetric
    antisym_copy(Rw, bar(Tin), o, v, s);
    int zero = 0, bad = 0;
    DCSD_HIP(hipMemcpyAsync(flag, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    maxabs(Rw, total, scal + 1, flag, part, s);
    dot(Rw, Rw, total, scal + 3, part, s);
    double rmax = 0.0, ss = 0.0;
    DCSD_HIP(hipMemcpyAsync(&rmax, scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    DCSD_HIP(hipMemcpyAsync(&ss, scal + 3, sizeof(double), hipMemcpyDeviceToHost, s));
    DCSD_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    DCSD_HIP(hipStreamSynchronize(s));
    r.iterations = it + 1;
    r.res_max = rmax;
    r.res_rms = std::sqrt(std::max(ss, 0.0) / (double)total);
    r.fp64 = 1;
    r.converged = (!bad && rmax <= cfg.tol_residual) ? 1 : 0;
    if (bad || !std::isfinite(rmax)) {
      if (rep) *rep = r;
      return DCSD_ERR_NONFINITE;
    }
    if (r.converged) {
      if (rep) *rep = r;
      return DCSD_OK;
    }
    jacobi_diis(it, L, Rw, gram, order, count);
  }
  if (rep) *rep = r;
  return DCSD_ERR_NOCONV;
}

}  // namespace dcsd
