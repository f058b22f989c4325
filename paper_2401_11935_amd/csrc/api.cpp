// C ABI of libdcsd: argument checks, status codes and error messages.  No
// exception crosses this boundary.
#include <new>
#include <string>

#include "ctx.h"

struct dcsd_ctx {
  dcsd::Ctx c;
};

namespace {
thread_local std::string g_init_error;  // last failed dcsd_init or context-free call of this thread

template <class Fn>
dcsd_status guarded(dcsd_ctx* h, Fn&& fn) {
  if (!h) return DCSD_ERR_ARG;
  if (h->c.sticky) return DCSD_ERR_STATE;
  try {
    h->c.err.clear();
    return fn();
  } catch (const dcsd::ArgError& e) {
    h->c.err = e.what();
    return DCSD_ERR_ARG;
  } catch (const dcsd::HipError& e) {
    h->c.err = e.what();
    h->c.sticky = true;
    return DCSD_ERR_HIP;
  } catch (const std::bad_alloc&) {
    h->c.err = "allocation failed";
    return DCSD_ERR_OOM;
  } catch (const std::exception& e) {
    h->c.err = e.what();
    h->c.sticky = true;
    return DCSD_ERR_HIP;
  }
}
}  // namespace

namespace dcsd {
void set_call_error(const char* msg) { g_init_error = msg; }
}  // namespace dcsd

extern "C" {

int64_t dcsd_amplitude_count(int32_t nc, int32_t nv) {
  if (nc < 0 || nv < 1) return -1;
  const int64_t o = nc + 1, v = nv + 1;
  return 2 * o * v + 3 * o * o * v * v;
}

int64_t dcsd_method_amplitude_count(int32_t nc, int32_t nv, int32_t method) {
  if (!dcsd::method_known(method)) return -1;
  if (!dcsd::method_hs(method)) return dcsd_amplitude_count(nc, nv);
  if (nc < 1 || nv < 1) return -1;
  dcsd::SpinLayout L;
  L.nc = nc;
  L.n = nc + 2 + nv;
  L.swap_tu = 0;
  L.o[0] = nc + 2;
  L.o[1] = nc;
  L.v[0] = nv;
  L.v[1] = nv + 2;
  return L.total();
}

void dcsd_default_config(dcsd_config* c) {
  if (!c) return;
  *c = dcsd_config{};
  c->method = DCSD_METHOD_DCSD;
  c->precision = DCSD_PREC_FP64;
  c->diis_dim = 8;
  c->diis_start = 2;
  c->max_iter = 200;
  c->tol_residual = 1e-10;
  c->level_shift = 0.0;
  c->ladder_block = 0;
  c->term_mask = DCSD_TERM_ALL;
  c->precond = DCSD_PRECOND_ORBITAL;
  c->refresh_every = 0;
  c->adjoint = 0;
  c->guard_iters = 10;
  c->ladder_cache = 1;
}

dcsd_status dcsd_init(const dcsd_config* cfg, const double* B_dev, const double* F_dev, void* hip_stream,
                      dcsd_ctx** out) {
  if (!out) return DCSD_ERR_ARG;
  *out = nullptr;
  if (!cfg) {
    g_init_error = "cfg is NULL";
    return DCSD_ERR_ARG;
  }
  dcsd_ctx* h = new (std::nothrow) dcsd_ctx;
  if (!h) return DCSD_ERR_OOM;
  dcsd_status st = DCSD_OK;
  try {
    h->c.init(*cfg, B_dev, F_dev, (hipStream_t)hip_stream);
  } catch (const dcsd::ArgError& e) {
    g_init_error = e.what();
    st = DCSD_ERR_ARG;
  } catch (const std::bad_alloc&) {
    g_init_error = "device allocation failed";
    st = DCSD_ERR_OOM;
  } catch (const std::exception& e) {
    g_init_error = e.what();
    st = DCSD_ERR_HIP;
  }
  if (st != DCSD_OK) {
    if (!h->c.allocs.empty()) (void)hipStreamSynchronize((hipStream_t)hip_stream);
    h->c.release();
    delete h;
    return st;
  }
  g_init_error.clear();
  *out = h;
  return DCSD_OK;
}

dcsd_status dcsd_residual(dcsd_ctx* ctx, const double* T_dev, double* R_dev, double* W_host) {
  return guarded(ctx, [&] {
    if (!T_dev || !R_dev || T_dev == R_dev) throw dcsd::ArgError("T and R must be distinct device pointers");
    ctx->c.residual(T_dev, R_dev, W_host);
    return DCSD_OK;
  });
}

dcsd_status dcsd_energy(dcsd_ctx* ctx, const double* T_dev, dcsd_energies* out) {
  return guarded(ctx, [&] {
    if (!T_dev || !out) throw dcsd::ArgError("T and out are required");
    ctx->c.energies(T_dev, out);
    return DCSD_OK;
  });
}

dcsd_status dcsd_triples(dcsd_ctx* ctx, const double* T_dev, dcsd_triples_energy* out, double* contrib_dev) {
  return guarded(ctx, [&] {
    if (!T_dev || !out) throw dcsd::ArgError("T and out are required");
    ctx->c.triples(T_dev, out, contrib_dev);
    return DCSD_OK;
  });
}

dcsd_status dcsd_solve(dcsd_ctx* ctx, double* T_inout, dcsd_report* out, dcsd_iter_cb cb, void* user) {
  return guarded(ctx, [&] {
    if (!T_inout) throw dcsd::ArgError("T_inout is required");
    const int rc = ctx->c.solve(T_inout, out, cb, user);
    if (rc == DCSD_ERR_NOCONV) ctx->c.err = "not converged within max_iter";
    if (rc == DCSD_ERR_NONFINITE) ctx->c.err = "non-finite residual";
    return (dcsd_status)rc;
  });
}

dcsd_status dcsd_residual_vjp(dcsd_ctx* ctx, const double* T_dev, const double* Rbar_dev, double Wbar, double EAbar,
                              double* Tbar_dev, double* Bbar_dev, double* Fbar_dev) {
  return guarded(ctx, [&] {
    if (!T_dev || !Rbar_dev) throw dcsd::ArgError("T and Rbar are required");
    dcsd::Ctx& c = ctx->c;
    if (!c.adj_ready) {
      c.err = "the adjoint needs a context built with cfg.adjoint = 1";
      return DCSD_ERR_STATE;
    }
    c.record(T_dev);
    c.sweep(Rbar_dev, Wbar, EAbar, Bbar_dev || Fbar_dev);
    if (Tbar_dev) DCSD_HIP(hipMemcpyAsync(Tbar_dev, c.bar(c.Tin), c.total * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    if (Bbar_dev)
      DCSD_HIP(hipMemcpyAsync(Bbar_dev, c.bar(c.B), (size_t)c.naux * c.n2 * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    if (Fbar_dev) DCSD_HIP(hipMemcpyAsync(Fbar_dev, c.bar(c.F), c.n2 * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    DCSD_HIP(hipStreamSynchronize(c.s));
    return DCSD_OK;
  });
}

dcsd_status dcsd_backward(dcsd_ctx* ctx, const double* T_dev, double ebar_S, double ebar_T, double* Bbar_dev,
                          double* Fbar_dev, double* lambda_dev, dcsd_report* out) {
  return guarded(ctx, [&] {
    if (!T_dev || !Bbar_dev || !Fbar_dev) throw dcsd::ArgError("T, Bbar and Fbar are required");
    dcsd::Ctx& c = ctx->c;
    if (!c.adj_ready) {
      c.err = "the adjoint needs a context built with cfg.adjoint = 1";
      return DCSD_ERR_STATE;
    }
    c.record(T_dev);
    if (lambda_dev)
      DCSD_HIP(hipMemcpyAsync(c.lam, lambda_dev, c.total * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    else
      dcsd::fill(c.lam, 0.0, c.total, c.s);
    // E = a dE_A + b W; a fixed-reference run has one state, with energy dE_A and W = 0
    double a = ebar_S + ebar_T, b = ebar_S - ebar_T;
    if (dcsd::method_fr(c.cfg.method)) {
      a = dcsd::ab_amplitude(c.cfg.method) > 0.0 ? ebar_S : ebar_T;
      b = 0.0;
    }
    dcsd_report rep{};
    const int rc = c.lambda_solve(a, b, c.lam, &rep);
    if (out) *out = rep;
    if (rc == DCSD_ERR_NONFINITE) {
      c.err = "non-finite lambda residual";
      return (dcsd_status)rc;
    }
    c.sweep(c.lam, b, a, true);
    dcsd::symmetrize(Bbar_dev, c.bar(c.B), c.naux, c.n, c.s);
    dcsd::symmetrize(Fbar_dev, c.bar(c.F), 1, c.n, c.s);
    if (lambda_dev)
      DCSD_HIP(hipMemcpyAsync(lambda_dev, c.lam, c.total * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    DCSD_HIP(hipStreamSynchronize(c.s));
    if (rc == DCSD_ERR_NOCONV) c.err = "lambda equations not converged within max_iter";
    return (dcsd_status)rc;
  });
}

dcsd_status dcsd_update_config(dcsd_ctx* ctx, const dcsd_config* cfg) {
  return guarded(ctx, [&] {
    if (!cfg) throw dcsd::ArgError("cfg is NULL");
    const dcsd_config& c = ctx->c.cfg;
    if (cfg->nc != c.nc || cfg->nv != c.nv || cfg->naux != c.naux || cfg->method != c.method ||
        cfg->precision != c.precision || cfg->diis_dim != c.diis_dim || cfg->ladder_block != c.ladder_block)
      throw dcsd::ArgError("only solver settings may change after dcsd_init");
    if (cfg->adjoint != c.adjoint) throw dcsd::ArgError("adjoint is fixed at dcsd_init");
    if (cfg->ladder_cache != c.ladder_cache) throw dcsd::ArgError("ladder_cache is fixed at dcsd_init");
    if (cfg->max_iter < 1 || !(cfg->tol_residual > 0.0) || !(cfg->level_shift >= 0.0) || cfg->refresh_every < 0 ||
        cfg->guard_iters < 0 ||
        (cfg->precond != DCSD_PRECOND_ORBITAL && cfg->precond != DCSD_PRECOND_EN))
      throw dcsd::ArgError("invalid solver settings");
    ctx->c.cfg = *cfg;
    return DCSD_OK;
  });
}

dcsd_status dcsd_timing_start(dcsd_ctx* ctx) {
  return guarded(ctx, [&] {
    dcsd::Ctx& c = ctx->c;
    if (c.pool.empty()) {
      c.pool.resize(4096);
      for (auto& e : c.pool) DCSD_HIP(hipEventCreate(&e));
    }
    DCSD_HIP(hipStreamSynchronize(c.s));
    c.recs.clear();
    c.pool_next = 0;
    c.timing = true;
    return DCSD_OK;
  });
}

dcsd_status dcsd_timing_stop(dcsd_ctx* ctx, dcsd_timing* out) {
  return guarded(ctx, [&] {
    dcsd::Ctx& c = ctx->c;
    DCSD_HIP(hipStreamSynchronize(c.s));
    c.timing = false;
    dcsd_timing t{};
    dcsd_kernel_time* k[4] = {&t.assembly, &t.contraction, &t.residual, &t.ring};
    for (const auto& r : c.recs) {
      float ms = 0.f;
      DCSD_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      k[r.cls]->ms += ms;
      k[r.cls]->launches += 1;
      k[r.cls]->flops += r.flops;
    }
    c.recs.clear();
    c.pool_next = 0;
    if (out) *out = t;
    return DCSD_OK;
  });
}

dcsd_status dcsd_device_memory(const dcsd_ctx* ctx, int64_t* bytes, int64_t* allocations) {
  if (!ctx) return DCSD_ERR_ARG;
  if (bytes) *bytes = (int64_t)ctx->c.bytes;
  if (allocations) *allocations = ctx->c.alloc_calls;
  return DCSD_OK;
}

const char* dcsd_last_error(const dcsd_ctx* ctx) {
  if (!ctx) return g_init_error.c_str();
  return ctx->c.err.c_str();
}

void dcsd_destroy(dcsd_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->c.s);
  for (auto& e : ctx->c.pool) (void)hipEventDestroy(e);
  ctx->c.release();
  delete ctx;
}

dcsd_status dcsd_selftest_gemm(int32_t precision, int64_t M, int64_t N, int64_t K, const double* A_dev,
                               const double* B_dev, double* C_dev, void* hip_stream) {
  if (M <= 0 || N <= 0 || K <= 0 || !A_dev || !B_dev || !C_dev) return DCSD_ERR_ARG;
  if (precision != DCSD_PREC_FP64 && precision != DCSD_PREC_FP32 && precision != DCSD_PREC_BF16) return DCSD_ERR_ARG;
  const hipStream_t st = (hipStream_t)hip_stream;
  if (precision == DCSD_PREC_FP64) {
    try {
      dcsd::GemmArgs g;
      g.M = M; g.N = N; g.K = K;
      g.A = A_dev; g.lda = K; g.a_mc = false;
      g.B = B_dev; g.ldb = N; g.b_nc = true;
      g.C = C_dev; g.ldc = N; g.c_nc = true;
      dcsd::gemm_f64(g, st);
      if (hipStreamSynchronize(st) != hipSuccess) return DCSD_ERR_HIP;
    } catch (...) {
      return DCSD_ERR_HIP;
    }
    return DCSD_OK;
  }
  const int64_t ld = dcsd::lp_ld(K);
  const size_t es = dcsd::lp_size(precision);
  void *a = nullptr, *b = nullptr;
  float* w = nullptr;
  const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
  const int ks = (tiles < 16 && K >= 256) ? 4 : 1;  // exercises the split-K path on small outputs
  dcsd_status st_out = DCSD_OK;
  try {
    if (hipMalloc(&a, M * ld * es) != hipSuccess || hipMalloc(&b, N * ld * es) != hipSuccess ||
        (ks > 1 && hipMalloc((void**)&w, ks * M * N * sizeof(float)) != hipSuccess))
      throw dcsd::HipError("allocation failed");
    dcsd::lp_convert(precision, a, ld, A_dev, nullptr, M, K, K, 1, st);  // a[m][k] = A[m][k]
    dcsd::lp_convert(precision, b, ld, B_dev, nullptr, N, K, 1, N, st);  // b[n][k] = B[k][n]
    dcsd::LpGemm q;
    q.precision = precision;
    q.M = M; q.N = N; q.K = K;
    q.A = a; q.lda = ld; q.B = b; q.ldb = ld;
    q.C = C_dev; q.ldc = N;
    q.ks = ks; q.work = w;
    dcsd::lp_gemm(q, st);
    if (hipStreamSynchronize(st) != hipSuccess) st_out = DCSD_ERR_HIP;
  } catch (...) {
    st_out = DCSD_ERR_HIP;
  }
  (void)hipStreamSynchronize(st);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (w) (void)hipFree(w);
  return st_out;
}

dcsd_status dcsd_selftest_gemm_layout(int64_t M, int64_t N, int64_t K, const double* A_dev, int64_t lda,
                                      int32_t a_mc, const double* B_dev, int64_t ldb, int32_t b_nc, double* C_dev,
                                      int64_t ldc, double alpha, double beta, int32_t ksplit, void* hip_stream) {
  if (M <= 0 || N <= 0 || K <= 0 || !A_dev || !B_dev || !C_dev || ksplit < 1) return DCSD_ERR_ARG;
  if (lda < (a_mc ? M : K) || ldb < (b_nc ? N : K) || ldc < N) return DCSD_ERR_ARG;
  const hipStream_t st = (hipStream_t)hip_stream;
  double *w = nullptr, *pw = nullptr;
  dcsd_status st_out = DCSD_OK;
  try {
    dcsd::GemmArgs g;
    g.M = M; g.N = N; g.K = K;
    g.A = A_dev; g.lda = lda; g.a_mc = a_mc != 0;
    g.B = B_dev; g.ldb = ldb; g.b_nc = b_nc != 0;
    g.C = C_dev; g.ldc = ldc; g.c_nc = true;
    g.alpha = alpha; g.beta = beta;
    g.ksplit = ksplit;
    // the library's dispatch: small outputs over a long K take the split dot products
    const int64_t small = ksplit == 1 ? dcsd::gemm_f64_small_work(g) : 0;
    if (small > 0) {
      if (hipMalloc((void**)&w, (size_t)small * sizeof(double)) != hipSuccess) throw dcsd::HipError("allocation failed");
      if (!dcsd::gemm_f64_small(g, w, small, st)) throw dcsd::HipError("small-output product refused");
    } else {
      if (ksplit > 1) {
        if (hipMalloc((void**)&w, (size_t)ksplit * M * ldc * sizeof(double)) != hipSuccess)
          throw dcsd::HipError("allocation failed");
        g.work = w;
      }
      // operands the direct-to-LDS kernel cannot stream are copied, zero-padded, as in the method
      const int64_t padw = dcsd::gemm_f64_pad_work(g);
      if (padw > 0) {
        if (hipMalloc((void**)&pw, (size_t)padw * sizeof(double)) != hipSuccess)
          throw dcsd::HipError("allocation failed");
        g.pad = pw;
        g.pad_cap = padw;
      }
      dcsd::gemm_f64(g, st);
    }
    if (hipStreamSynchronize(st) != hipSuccess) st_out = DCSD_ERR_HIP;
  } catch (const dcsd::ArgError&) {
    st_out = DCSD_ERR_ARG;
  } catch (...) {
    st_out = DCSD_ERR_HIP;
  }
  (void)hipStreamSynchronize(st);
  if (w) (void)hipFree(w);
  if (pw) (void)hipFree(pw);
  return st_out;
}

}  // extern "C"
