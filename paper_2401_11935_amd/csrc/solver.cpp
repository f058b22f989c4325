// Amplitude solver: Jacobi steps with orbital-energy denominators and Pulay
// DIIS.  All vectors stay on the device in FP64; only the (m+1)^2 DIIS system,
// the residual max-norm and the energies cross to the host (one
// synchronisation per iteration).  In low precision the iterations run the
// low-precision residual, after the first refresh point in delta form (FP64
// products at the refresh point plus low-precision products of the operand
// changes); refreshes are FP64 evaluations and convergence is only accepted
// on one of them.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.h"

namespace dcsd {

namespace {
// Solves A x = b (dense, partial pivoting); A is overwritten.
bool solve_dense(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * b[k];
    b[r] = s / A[r * n + r];
  }
  return true;
}
}  // namespace

// One Jacobi step from residual R at X (Tn = X + R/(D - s - shift)) followed by
// the DIIS extrapolation over the stored (Tn, Tn - X) pairs; X receives the
// new vector.
void Ctx::jacobi_diis(int it, double* X, const double* R, std::vector<double>& gram, std::vector<int>& order,
                      int& count) {
  const int m = cfg.diis_dim;
  const bool en = cfg.precond == DCSD_PRECOND_EN;
  jacobi(Tn, Ev, X, R, f[0], f[1], en ? Jpq : nullptr, en ? Kpq : nullptr, L, cfg.level_shift, s);
  if (m > 0) {
    const int slot = count % m;
    ++count;
    DCSD_HIP(hipMemcpyAsync(histT + (int64_t)slot * total, Tn, total * sizeof(double), hipMemcpyDeviceToDevice, s));
    DCSD_HIP(hipMemcpyAsync(histE + (int64_t)slot * total, Ev, total * sizeof(double), hipMemcpyDeviceToDevice, s));
    for (size_t k = 0; k < order.size(); ++k)
      if (order[k] == slot) {
        order.erase(order.begin() + k);
        break;
      }
    order.push_back(slot);
    const int nh = (int)order.size();
    for (int j = 0; j < nh; ++j)
      dot(histE + (int64_t)slot * total, histE + (int64_t)order[j] * total, total, scal + 4 + j, part, s);
    std::vector<double> d(nh);
    DCSD_HIP(hipMemcpyAsync(d.data(), scal + 4, nh * sizeof(double), hipMemcpyDeviceToHost, s));
    DCSD_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < nh; ++j) {
      gram[slot * m + order[j]] = d[j];
      gram[order[j] * m + slot] = d[j];
    }
    if (it >= cfg.diis_start && nh >= 2) {
      const int N = nh + 1;
      std::vector<double> A((size_t)N * N, 0.0), b(N, 0.0);
      for (int i = 0; i < nh; ++i)
        for (int j = 0; j < nh; ++j) A[i * N + j] = gram[order[i] * m + order[j]];
      for (int i = 0; i < nh; ++i) {
        A[i * N + nh] = -1.0;
        A[nh * N + i] = -1.0;
      }
      b[nh] = -1.0;
      if (solve_dense(A, b, N)) {
        // coefficients in slot order for the device combination
        std::vector<double> c(m, 0.0);
        for (int i = 0; i < nh; ++i) c[order[i]] = b[i];
        DCSD_HIP(hipMemcpyAsync(coef, c.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
        DCSD_HIP(hipStreamSynchronize(s));
        combine(X, histT, total, coef, std::min(count, m), total, s);
        return;
      }
    }
  }
  DCSD_HIP(hipMemcpyAsync(X, Tn, total * sizeof(double), hipMemcpyDeviceToDevice, s));
}

int Ctx::solve(double* T, dcsd_report* rep, dcsd_iter_cb cb, void* user) {
  const int m = cfg.diis_dim;
  const bool low = cfg.precision != DCSD_PREC_FP64;
  std::vector<double> gram((size_t)std::max(m, 1) * std::max(m, 1), 0.0);
  std::vector<int> order;  // slots from oldest to newest
  int count = 0;
  dcsd_report r{};
  bool have_ref = false;  // a refresh point has been recorded
  int since = 0;          // low-precision iterations since the last refresh
  double ref_res = 0.0;   // FP64 max |R| at the last refresh
  double best = 0.0;      // smallest corrected max |R| since the last refresh, and its iteration
  int best_it = -1;
  // Best amplitudes of the solve (returned without convergence): smallest max |R|
  // among FP64 evaluations, or among all evaluations while none was FP64.
  dcsd_report best_rep{};
  bool have_best = false;
  // Divergence guard: consecutive growths of max |R|, and how often it has acted.
  // The raised level shift lasts for this solve only.
  struct ShiftRestore {
    dcsd_config& c;
    double v;
    ~ShiftRestore() { c.level_shift = v; }
  } restore{cfg, cfg.level_shift};
  double prev_res = -1.0;
  int growths = 0, guard_events = 0;
  // max |Rw|, sum Rw^2, energies of Tw and W; one synchronisation
  auto measure = [&](double host[4], int& bad) {
    int zero = 0;
    DCSD_HIP(hipMemcpyAsync(flag, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    DCSD_HIP(hipStreamSynchronize(s));
    maxabs(Rw, total, scal + 1, flag, part, s);
    energy(Tw, Isc, f[0], f[1], L, scal + 2, part, s);
    dot(Rw, Rw, total, scal + 3, part, s);
    DCSD_HIP(hipMemcpyAsync(host, scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    DCSD_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    DCSD_HIP(hipStreamSynchronize(s));
  };
  // without convergence: hand back the best amplitudes and the report that describes them
  auto give_up = [&](int status) {
    if (have_best) {
      DCSD_HIP(hipMemcpyAsync(T, Tbest, total * sizeof(double), hipMemcpyDeviceToDevice, s));
      DCSD_HIP(hipStreamSynchronize(s));
      best_rep.iterations = r.iterations;
      best_rep.converged = 0;
      if (rep) *rep = best_rep;
    } else if (rep) {
      *rep = r;
    }
    return status;
  };
  // Refreshes.  A low-precision residual that meets the tolerance, has dropped
  // by kDrop since the last refresh or completes refresh_every iterations still
  // takes its step, and the next iteration is the refresh.  One that has set no
  // new minimum for kStall iterations sits on its noise floor: it is replaced at
  // once by the FP64 residual at the same amplitudes, which takes the step.
  constexpr int kStall = 3;
  const double kDrop = cfg.precision == DCSD_PREC_BF16 ? 1e-2 : 1e-5;
  bool refresh_next = false;
  for (int it = 0; it < cfg.max_iter; ++it) {
    bool exact = !low || refresh_next;
    if (low && refresh_next)
      residual(T, Rw, nullptr, DCSD_PREC_FP64, RECORD);
    else
      residual(T, Rw, nullptr, -1, low && have_ref ? DELTA : PLAIN);
    double host[4];
    int bad = 0;
    measure(host, bad);
    if (low && !exact) {
      ++since;
      if (best_it < 0 || host[1] < best) {
        best = host[1];
        best_it = it;
      }
      if (it == 0) ref_res = host[1];
      if (!bad && it - best_it >= kStall) {
        residual(T, Rw, nullptr, DCSD_PREC_FP64, RECORD);
        measure(host, bad);
        exact = true;
      }
    }
    if (low && exact) {  // a refresh: the new reference point
      have_ref = true;
      since = 0;
      best = host[1];
      best_it = it;
      ref_res = host[1];
    }
    refresh_next = low && !bad &&
                   (exact ? cfg.refresh_every == 1
                          : (host[1] <= cfg.tol_residual || host[1] <= kDrop * ref_res ||
                             (cfg.refresh_every > 0 && since + 1 >= cfg.refresh_every)));
    r.iterations = it + 1;
    r.res_max = host[1];
    r.res_rms = std::sqrt(std::max(host[3], 0.0) / (double)total);
    r.e.W = host[0];
    r.e.dE_A = host[2];
    state_energies(cfg.method, host[2], host[0], r.e.E_S, r.e.E_T);
    r.e.E_ref_A = e_ref;
    r.fp64 = exact ? 1 : 0;
    r.converged = (!bad && exact && host[1] <= cfg.tol_residual) ? 1 : 0;
    if (cb) cb(&r, user);
    if (bad || !std::isfinite(host[0]) || !std::isfinite(host[2])) return give_up(DCSD_ERR_NONFINITE);
    if (r.converged) {
      if (rep) *rep = r;
      return DCSD_OK;
    }
    if (!have_best || (r.fp64 && !best_rep.fp64) || (r.fp64 == best_rep.fp64 && r.res_max < best_rep.res_max)) {
      DCSD_HIP(hipMemcpyAsync(Tbest, T, total * sizeof(double), hipMemcpyDeviceToDevice, s));
      best_rep = r;
      have_best = true;
    }
    if (cfg.guard_iters > 0) {
      growths = (prev_res >= 0.0 && host[1] > prev_res) ? growths + 1 : 0;
      prev_res = host[1];
      if (growths >= cfg.guard_iters) {
        if (++guard_events > 2) return give_up(DCSD_ERR_NOCONV);
        // restart from the best amplitudes with a fresh DIIS history and a larger shift
        order.clear();
        count = 0;
        std::fill(gram.begin(), gram.end(), 0.0);
        cfg.level_shift = 2.0 * cfg.level_shift + 1.0;
        DCSD_HIP(hipMemcpyAsync(T, Tbest, total * sizeof(double), hipMemcpyDeviceToDevice, s));
        growths = 0;
        prev_res = -1.0;
        continue;
      }
    }
    jacobi_diis(it, T, Rw, gram, order, count);
  }
  return give_up(DCSD_ERR_NOCONV);
}

}  // namespace dcsd
