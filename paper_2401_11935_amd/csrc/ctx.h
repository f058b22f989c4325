// libdcsd context (internal).
#pragma once

#include <string>
#include <vector>

#include "../../include/libdcsd.h"
#include "kernels.h"
#include "tape.h"

namespace dcsd {

// Method families: CCSD keeps all T2*T2 terms, DCSD drops the distinguishable-cluster set;
// the fixed-reference methods hold the Phi_A -> Phi_B double at +1 (singlet) or -1
// (M_s = 0 triplet) and have no coupling terms.
// The high-spin methods solve the single-reference equations of the M_s = 1 determinant.
inline bool method_known(int m) { return m >= DCSD_METHOD_DCSD && m <= DCSD_METHOD_HS_CCSD; }
inline bool method_cc(int m) {
  return m == DCSD_METHOD_CCSD || m == DCSD_METHOD_FR_CCSD_SINGLET || m == DCSD_METHOD_FR_CCSD_TRIPLET ||
         m == DCSD_METHOD_HS_CCSD;
}
inline bool method_fr(int m) { return m >= DCSD_METHOD_FR_DCSD_SINGLET && m <= DCSD_METHOD_FR_CCSD_TRIPLET; }
inline bool method_hs(int m) { return m == DCSD_METHOD_HS_DCSD || m == DCSD_METHOD_HS_CCSD; }
// the methods whose residual has a Phi_A -> Phi_B element (held at 0 or +-1)
inline bool method_ab(int m) { return !method_hs(m); }
// value of the Phi_A -> Phi_B double in the residual and energy
inline double ab_amplitude(int m) {
  if (!method_fr(m)) return 0.0;
  return (m == DCSD_METHOD_FR_DCSD_SINGLET || m == DCSD_METHOD_FR_CCSD_SINGLET) ? 1.0 : -1.0;
}
// singlet and triplet correlation energies from dE_A and W
inline void state_energies(int m, double dEA, double W, double& ES, double& ET) {
  if (method_hs(m)) {
    ES = __builtin_nan("");
    ET = dEA;
    return;
  }
  if (!method_fr(m)) {
    ES = dEA + W;
    ET = dEA - W;
    return;
  }
  const double nan = __builtin_nan("");
  const bool singlet = ab_amplitude(m) > 0.0;
  ES = singlet ? dEA : nan;
  ET = singlet ? nan : dEA;
}

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

  // sizes.  o, v, ov, s2 and npair describe Phi_A (both spins alike, as the adjoint and
  // the coupling use them); the residual runs on the per-spin layout L, whose spins
  // differ for the high-spin methods.
  int nc = 0, nv = 0, naux = 0, n = 0, o = 0, v = 0, vu = 0, npair = 0;
  int64_t ov = 0, tov = 0, s2 = 0, n2 = 0, total = 0;
  SpinLayout L;
  int os[2] = {0, 0}, vs[2] = {0, 0};   // per-spin occupied / virtual counts (= L.o, L.v)
  int64_t ovs[2] = {0, 0};              // o v per spin (ph block widths)
  int64_t oos[2] = {0, 0};              // o^2 per spin, and too2 = oos[0] + oos[1]
  int64_t too2 = 0;
  int npairs[2] = {0, 0};               // same-spin occupied pairs i < j per spin
  int64_t sfr = 0, sfc = 0;             // spin-flip ph dimensions: (alpha occ, beta vir), (beta occ, alpha vir)
  int64_t wmax = 0;                     // largest of the per-block ph and doubles sizes

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
  double* pws = nullptr;               // padded operand copies of the FP64 GEMMs (optional)
  int64_t pws_cap = 0;
  double* Isc = nullptr;               // undressed (kc|ld), spin-conserving ph matrix (2ov x 2ov)
  double* Icc = nullptr;               // antisymmetrised <kl||cd> ph matrix (CCSD only)
  double* Isf1 = nullptr;              // spin-flip <kl||cd> blocks (CCSD only)
  double* Isf2 = nullptr;
  double* QX1[2] = {nullptr, nullptr}, *QX2[2] = {nullptr, nullptr};
  double* QY1[2] = {nullptr, nullptr}, *QY2[2] = {nullptr, nullptr};
  double* Ikl[3] = {nullptr, nullptr, nullptr};  // aa, bb, ab: [(k,l),(c,d)]
  std::vector<char> coup_launch;       // coupling pattern launches (host)
  int* pair_i = nullptr;
  int* pair_j = nullptr;
  double e_ref = 0.0;

  // per-evaluation work buffers
  double *Tw = nullptr, *Bt[2] = {nullptr, nullptr}, *ft[2] = {nullptr, nullptr}, *Jv = nullptr;
  double *Xk = nullptr, *Yk = nullptr;
  double *Bov = nullptr, *Bvo = nullptr, *Boo = nullptr;
  double *Tsc = nullptr, *Tsf1 = nullptr, *Z = nullptr, *out1 = nullptr, *out2 = nullptr, *fvec = nullptr;
  double *KCBJ = nullptr, *Dvo = nullptr, *KJPQ[2] = {nullptr, nullptr}, *OOOO = nullptr;
  double* Ring = nullptr;
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
  // low precision (allocated only when cfg.precision != FP64)
  int prec_now = DCSD_PREC_FP64;      // precision of the ladder and ring GEMMs of the current evaluation
  // How the low-precision GEMMs of an evaluation relate to the last refresh
  // point T_r: PLAIN rounds the operands themselves; RECORD (an FP64
  // evaluation) stores the FP64 operands and products at T_r; DELTA adds the
  // stored FP64 products to low-precision products of the operand changes.
  enum Mode { PLAIN = 0, RECORD = 1, DELTA = 2 };
  int mode = PLAIN;
  void* BlT = nullptr;                 // Bl transposed to [(p,c)][P], row stride ldk
  void *TstackL = nullptr, *V2L = nullptr;  // rows of stride kp
  // low-precision ladder integrals of every batch (cfg.ladder_cache), filled by the first
  // low-precision evaluation; slot = lb * lb * kp elements
  void* lcache = nullptr;
  int64_t lcache_slot = 0;
  bool lcache_valid = false;
  // FP64 ladder integrals of every batch (cfg.ladder_cache = 2), filled by the first FP64 evaluation
  double* lcache64 = nullptr;
  int64_t lcache64_slot = 0;
  bool lcache64_valid = false;
  void *lpA = nullptr, *lpB = nullptr; // rounded ring operands, lp_cap elements each
  float* lwork = nullptr;              // FP32 split-K partials, lwork_cap floats
  int64_t ldk = 0, kp = 0, lp_cap = 0, lwork_cap = 0;
  double *TstackR = nullptr, *RpR = nullptr;  // ladder amplitudes and spatial ladder result at T_r
  bool ladder_ref = false;
  // ring GEMM sites: FP64 operands (those that change with T) and product at T_r
  struct Site {
    double *Ar = nullptr, *Br = nullptr, *Pr = nullptr;
    bool valid = false;
  };
  static constexpr int kSites = 11;
  Site site[kSites];
  // scalars and reductions
  double* part = nullptr;
  double* scal = nullptr;  // [0] W, [1] res max, [2] dE_A, [3] dot, ...
  int* flag = nullptr;
  // solver
  double *Tn = nullptr, *Ev = nullptr, *histT = nullptr, *histE = nullptr, *coef = nullptr, *Rw = nullptr;
  double* Tbest = nullptr;  // best amplitudes of a solve (smallest max |R|)

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
  size_t bytes = 0;         // device bytes allocated by the context (kept until dcsd_destroy)
  int64_t alloc_calls = 0;  // device allocation calls made, including the adjoint's sizing pass

  // Registry of the FP64 device arrays (context buffers and the borrowed B, F)
  // for the adjoint: tape bookkeeping (constant flag, write version) and the
  // shadow array holding each one's cotangent.
  struct Buf {
    double* p;
    int64_t n;
    bool constant = false;
    int version = 0;
    bool used = false;
    double* bar = nullptr;
  };
  std::vector<Buf> bufs;
  void reg(double* p, int64_t n, bool owned);
  int find_buf(const void* p) const;
  double* bar(const void* p);             // shadow address of p
  bool wants(const void* p, bool params);  // cotangent needed in this sweep?

  // adjoint state (reserved by dcsd_init when cfg.adjoint is set)
  Tape tape_init, tape_res;
  double *Tin = nullptr, *Rt = nullptr, *temp = nullptr, *lam = nullptr;
  int64_t temp_cap = 0;
  bool adj_ready = false;
  void adj_setup();
  void adj_reserve();
  void record(const double* T);
  void sweep(const double* Rbar, double Wbar, double Ebar, bool params);
  void adjoint_op(const TapeOp& op, bool params);
  void gemm_adjoint(const TapeOp& op, bool params);
  void ladder_adjoint(const TapeOp& op, bool params);
  int lambda_solve(double a, double b, double* lam_io, dcsd_report* rep);
  void build_constants(bool full);

  double* alloc(int64_t count);
  int* alloc_int(int64_t count);
  void* alloc_raw(size_t bytes);  // owned, not in the adjoint's array registry
  void release();

  void init(const dcsd_config& c, const double* B, const double* F, hipStream_t stream);
  void alloc_optional();
  int64_t site_size(int k, int which) const;
  // prec < 0: the configured precision; DCSD_PREC_FP64 forces an FP64 evaluation.
  // mode: PLAIN, RECORD (FP64 only) or DELTA (low precision with a recorded reference).
  void residual(const double* T, double* R, double* W_host, int prec = -1, int mode = PLAIN);
  double energy_A(const double* T);
  int solve(double* T, dcsd_report* rep, dcsd_iter_cb cb, void* user);
  void energies(const double* T, dcsd_energies* out);
  // perturbative triples of the M_s = 1 determinant (device memory allocated on first use)
  struct TriBuf {
    bool ready = false;
    double *t1so = nullptr, *t2so = nullptr, *fo = nullptr, *fv = nullptr, *fov = nullptr;
    double *I = nullptr, *oovv = nullptr, *Q = nullptr, *Zt = nullptr;
    double *part = nullptr, *out = nullptr, *Aop = nullptr;
  } tri;
  void triples(const double* T, dcsd_triples_energy* out, double* contrib);
  void jacobi_diis(int it, double* X, const double* R, std::vector<double>& gram, std::vector<int>& order,
                   int& count);
};

}  // namespace dcsd
