// libdcsd context (internal).
#pragma once

#include <string>
#include <vector>

#include "../../include/libdcsd.h"
#include "kernels.h"

namespace dcsd {

// Device memory owned by the context; every buffer is allocated in dcsd_init.
struct DevBuf {
  double* p = nullptr;
  int64_t n = 0;
};

struct Ctx {
  dcsd_config cfg{};
  std::string err;
  bool sticky = false;
  hipStream_t s = nullptr;
  int device = 0;

  // sizes
  int nc = 0, nv = 0, naux = 0, n = 0, o = 0, v = 0, vu = 0, npair = 0;
  int64_t ov = 0, tov = 0, s2 = 0, n2 = 0, total = 0;

  // borrowed inputs
  const double* B = nullptr;
  const double* F = nullptr;

  // constants (built at init)
  double* Bs[2] = {nullptr, nullptr};  // B in alpha order (== input) and beta order
  double* h[2] = {nullptr, nullptr};   // one-electron Hamiltonian in spin order
  double* f[2] = {nullptr, nullptr};   // reference Fock matrices of Phi_A in spin order
  double* Bl = nullptr;                // ladder factor [P][p][c], c over [t,u,virt]
  double* Jpq = nullptr;               // (pp|qq), spatial
  double* Kpq = nullptr;               // (pq|qp), spatial
  double* gws = nullptr;               // split-K workspace
  int64_t gws_cap = 0;
  double* Isc = nullptr;               // undressed (kc|ld), spin-conserving ph matrix (2ov x 2ov)
  double* Icc = nullptr;               // antisymmetrised <kl||cd> ph matrix (CCSD only)
  double* Isf1 = nullptr;              // spin-flip <kl||cd> blocks (CCSD only)
  double* Isf2 = nullptr;
  double* QX1[2] = {nullptr, nullptr}, *QX2[2] = {nullptr, nullptr};
  double* QY1[2] = {nullptr, nullptr}, *QY2[2] = {nullptr, nullptr};
  double* Ikl[3] = {nullptr, nullptr, nullptr};  // aa, bb, ab: [(k,l),(c,d)]
  std::vector<char> coup_launch;       // coupling pattern launches (host)
  double* coup_terms = nullptr;        // coupling term tables (device)
  int* pair_i = nullptr;
  int* pair_j = nullptr;
  double e_ref = 0.0;

  // per-evaluation work buffers
  double *Tw = nullptr, *Bt[2] = {nullptr, nullptr}, *ft[2] = {nullptr, nullptr}, *Jv = nullptr;
  double *Xk = nullptr, *Yk = nullptr;
  double *Bov = nullptr, *Bvo = nullptr, *Boo = nullptr;
  double *Tsc = nullptr, *Tsf1 = nullptr, *Z = nullptr, *out1 = nullptr, *out2 = nullptr, *fvec = nullptr;
  double *KCBJ = nullptr, *Dvo = nullptr, *KJPQ[2] = {nullptr, nullptr}, *OOOO = nullptr;
  double *Tmp = nullptr, *Ring = nullptr;
  double *Wsf1 = nullptr, *Wsf2 = nullptr, *Rsf1 = nullptr, *Rsf2 = nullptr;
  double *P1 = nullptr, *P2 = nullptr;
  double *Xv[2] = {nullptr, nullptr}, *Yo[2] = {nullptr, nullptr}, *Fvv[2] = {nullptr, nullptr},
         *Foo[2] = {nullptr, nullptr};
  double* Whh = nullptr;
  // ladder
  int lb = 0;  // block of spatial orbitals per ladder batch side
  int64_t rows_main = 0, rows_all = 0;
  double *Tstack = nullptr, *V2 = nullptr, *Rb = nullptr, *Rp = nullptr, *Smt = nullptr, *split = nullptr;
  int64_t split_cap = 0;
  // scalars and reductions
  double* part = nullptr;
  double* scal = nullptr;  // [0] W, [1] res max, [2] dE_A, [3] dot, ...
  int* flag = nullptr;
  // solver
  double *Tn = nullptr, *Ev = nullptr, *histT = nullptr, *histE = nullptr, *coef = nullptr, *Rw = nullptr;

  // timing (HIP events on the context's stream)
  bool timing = false;
  std::vector<hipEvent_t> pool;
  size_t pool_next = 0;
  struct Rec {
    hipEvent_t a, b;
    double flops;
    int cls;
  };
  std::vector<Rec> recs;
  int tbegin(hipEvent_t* ev);  // returns 1 if an interval is being recorded
  void tend(hipEvent_t a, double flops, int cls);

  std::vector<void*> allocs;
  size_t bytes = 0;

  double* alloc(int64_t count);
  int* alloc_int(int64_t count);
  void release();

  void init(const dcsd_config& c, const double* B, const double* F, hipStream_t stream);
  void residual(const double* T, double* R, double* W_host);
  double energy_A(const double* T);
  int solve(double* T, dcsd_report* rep, dcsd_iter_cb cb, void* user);
};

}  // namespace dcsd
