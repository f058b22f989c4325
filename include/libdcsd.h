/*
 * libdcsd -- two-determinant distinguishable-cluster (2D-DCSD) and 2D-CCSD
 * amplitude residual, energies and solver on one AMD Instinct MI355X (gfx950).
 *
 * Method: Schraivogel & Kats, "Two Determinant Distinguishable Cluster",
 * Theory section.  An open-shell singlet (or M_s = 0 triplet) is described by
 * two determinants Phi_A = |core, t alpha, u beta> and Phi_B = |core, u alpha,
 * t beta> (Fig. 1) whose amplitudes are spin flips of each other.  The
 * amplitude equations are the single-reference CCSD (or DCSD) equations of
 * Phi_A plus the renormalisation terms M_x W; the Phi_A -> Phi_B double is
 * fixed at zero and its residual element is W; the 2x2 effective Hamiltonian
 * gives the singlet dE_A + W and the triplet dE_A - W.
 *
 * Inputs (all FP64, row-major, device memory):
 *   B[P][p][q]  (naux x n x n) DF factors defining (pq|rs) = sum_P B[P,p,q] B[P,r,s];
 *               must be symmetric in p,q.
 *   F[p][q]     (n x n) spin-averaged Fock matrix of the open-shell reference;
 *               the one-electron Hamiltonian is h = F - G_avg[B] with
 *               G_avg = sum_core [2 J_k - K_k] + sum_{x = t,u} [J_x - K_x / 2].
 *   Orbital order [core 0..nc-1 | t = nc | u = nc+1 | virtuals], n = nc+2+nv.
 *
 * Packed amplitude / residual vector (length dcsd_amplitude_count), with
 * o = nc+1 and v = nv+1 per spin:
 *   [ t1a (o,v) | t1b (o,v) | t2aa (o,o,v,v) | t2bb (o,o,v,v) | t2ab (o,o,v,v) ]
 * alpha-occ = [core, t], alpha-vir = [u, virt], beta-occ = [core, u],
 * beta-vir = [t, virt].  Same-spin doubles are stored in full and must be
 * antisymmetric.  t2ab[nc][nc][0][0] (Phi_A -> Phi_B) is ignored on input and
 * is zero in every residual.
 *
 * Ownership: every pointer argument is owned by the caller.  B and F are
 * borrowed and must stay alive and unchanged until dcsd_destroy.  The library
 * allocates all of its device memory in dcsd_init and frees it in
 * dcsd_destroy; no other call allocates.
 *
 * Streams: all device work is enqueued on the HIP stream given to dcsd_init.
 * Calls that return host values synchronise that stream before returning.
 *
 * Errors: functions return a dcsd_status and never throw; dcsd_last_error
 * gives a message.  After DCSD_ERR_HIP the context is unusable (sticky).
 */
#ifndef LIBDCSD_H
#define LIBDCSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dcsd_ctx dcsd_ctx;

typedef enum {
  DCSD_OK = 0,
  DCSD_ERR_ARG = 1,        /* invalid argument or configuration            */
  DCSD_ERR_OOM = 2,        /* device allocation failed in dcsd_init        */
  DCSD_ERR_HIP = 3,        /* HIP runtime error (context becomes unusable) */
  DCSD_ERR_NOCONV = 4,     /* not converged (max_iter or divergence guard) */
  DCSD_ERR_NONFINITE = 5,  /* a residual contained Inf/NaN                 */
  DCSD_ERR_STATE = 6       /* context in an error state, or adjoint call
                              on a context built without cfg.adjoint     */
} dcsd_status;

/* Methods.  2D-DCSD and 2D-CCSD solve the two-determinant equations (Theory
 * section): the Phi_A -> Phi_B double is held at zero, the coupling -K_x W
 * enters every residual, and one solve gives both the open-shell singlet
 * E_S = dE_A + W and the M_s = 0 triplet E_T = dE_A - W.
 * The fixed-reference methods (introduction; the FR approach) solve the
 * single-reference DCSD or CCSD equations of Phi_A with the Phi_A -> Phi_B
 * double fixed at +1 (singlet: Phi_A + Phi_B) or -1 (M_s = 0 triplet:
 * Phi_A - Phi_B) and no coupling terms.  One solve gives one state: its
 * correlation energy dE_A (which includes the fixed amplitude) is reported in
 * E_S (singlet) or E_T (triplet), the other is NaN, and W is 0. */
/* The high-spin methods solve the single-reference DCSD or CCSD equations of
 * the M_s = 1 triplet determinant Phi_T = |core, t alpha, u alpha> (the
 * component the paper's single-reference triplets use for singlet-triplet
 * gaps; Computational Details and Results): no coupling, no fixed amplitude;
 * the triplet's correlation energy dE (the CC energy expression of Phi_T) is
 * reported in E_T and in dE_A, E_S is NaN, W is 0, and E_ref_A is <T|H|T>.
 * Their packed amplitudes use per-spin orders alpha-occ = [core, t, u],
 * beta-occ = [core], alpha-vir = [virt], beta-vir = [t, u, virt]:
 *   [ t1a (nc+2, nv) | t1b (nc, nv+2) | t2aa (nc+2, nc+2, nv, nv) |
 *     t2bb (nc, nc, nv+2, nv+2) | t2ab (nc+2, nc, nv, nv+2) ]
 * of length dcsd_method_amplitude_count(nc, nv, method).  They need nc >= 1
 * and run in every precision; the adjoint (cfg.adjoint) is not available for
 * them (DCSD_ERR_ARG). */
enum {
  DCSD_METHOD_DCSD = 0,
  DCSD_METHOD_CCSD = 1,
  DCSD_METHOD_FR_DCSD_SINGLET = 2,
  DCSD_METHOD_FR_DCSD_TRIPLET = 3,
  DCSD_METHOD_FR_CCSD_SINGLET = 4,
  DCSD_METHOD_FR_CCSD_TRIPLET = 5,
  DCSD_METHOD_HS_DCSD = 6,
  DCSD_METHOD_HS_CCSD = 7
};
/* Arithmetic of the particle-particle ladder and ring GEMMs (everything else
 * is FP64 in every mode): FP64 MFMA, or FP32 / BF16 MFMA inputs (rounded to
 * nearest even through FP32) with FP32 accumulation, added into FP64. */
enum { DCSD_PREC_FP64 = 0, DCSD_PREC_FP32 = 1, DCSD_PREC_BF16 = 2 };
/* Jacobi preconditioner: orbital-energy denominators D, or D minus the
 * two-electron (Epstein-Nesbet) part of the diagonal of dR/dT at T = 0. */
enum { DCSD_PRECOND_ORBITAL = 0, DCSD_PRECOND_EN = 1 };

/* Residual term selection (all bits set in production). */
enum {
  DCSD_TERM_DRIVER = 1u << 0,   /* <ab||ij>~                              */
  DCSD_TERM_FOCK = 1u << 1,     /* f_vv, f_oo terms with X, Y intermediates */
  DCSD_TERM_HH = 1u << 2,       /* hole-hole ladder                         */
  DCSD_TERM_PP = 1u << 3,       /* particle-particle ladder (DF-assembled)  */
  DCSD_TERM_RING = 1u << 4,     /* ring terms (linear and quadratic)        */
  DCSD_TERM_SINGLES = 1u << 5,  /* singles residual                         */
  DCSD_TERM_COUPLING = 1u << 6, /* -K_x W coupling of the two determinants  */
  DCSD_TERM_ALL = 0x7fu
};

typedef struct {
  int32_t nc, nv, naux;   /* core (doubly occupied) orbitals, virtuals, DF rank;
                             nc >= 0, nv >= 1, naux >= 1 (else DCSD_ERR_ARG) */
  int32_t method;         /* DCSD_METHOD_*                                      */
  int32_t precision;      /* DCSD_PREC_FP64, DCSD_PREC_FP32 or DCSD_PREC_BF16   */
  int32_t diis_dim;       /* DIIS subspace size (0 = plain Jacobi)              */
  int32_t diis_start;     /* first iteration that extrapolates                  */
  int32_t max_iter;
  double tol_residual;    /* convergence: max |R| <= tol                        */
  double level_shift;     /* Jacobi step R/(D - shift), shift >= 0              */
  int32_t ladder_block;   /* orbitals per ladder batch side (0 = automatic)    */
  uint32_t term_mask;     /* DCSD_TERM_* bits                                   */
  int32_t precond;        /* DCSD_PRECOND_ORBITAL or DCSD_PRECOND_EN            */
  int32_t refresh_every;  /* low precision only: FP64 residual at least every k-th
                             iteration of dcsd_solve (0 = only by the rules of
                             dcsd_solve)                                         */
  int32_t adjoint;        /* 1: dcsd_init also reserves the memory of
                             dcsd_residual_vjp and dcsd_backward (tape operand
                             snapshots, cotangent arrays, sweep work space), so
                             that those calls allocate nothing; 0: those calls
                             return DCSD_ERR_STATE                               */
  int32_t guard_iters;    /* divergence guard of dcsd_solve: after this many
                             consecutive growths of max |R| the DIIS history is
                             cleared, the level shift raised to 2 shift + 1 and
                             the iterations restart from the best amplitudes;
                             the third such event ends the solve with
                             DCSD_ERR_NOCONV (0 = off)                           */
  int32_t ladder_cache;   /* 1 (default): keep the FP32/BF16 particle-particle
                             ladder integrals (pc|qd) of every orbital-pair batch
                             in device memory after the first low-precision
                             evaluation, so that later ones skip their assembly
                             (they depend on B only, not on T; nc=12 nv=400:
                             32 GB in BF16, 65 GB in FP32).  2: the same, and
                             also the FP64 integrals after the first FP64
                             evaluation (129 GB at nc=12 nv=400), which serves
                             FP64 solves and the FP64 refreshes of the mixed
                             solver.  dcsd_init allocates the caches after all
                             other memory and leaves a cache off when it would
                             leave less than max(8 GiB, 5%) of the device free
                             (the records of the dressed-integral delta products,
                             allocated just before them, follow the same rule).
                             0: assemble every time                              */
} dcsd_config;

typedef struct {
  double dE_A;    /* single-reference correlation energy expression of Phi_A */
  double W;       /* effective coupling <B| H_N e^T_A |A> (residual element);
                     0 for the fixed-reference methods                        */
  double E_S;     /* open-shell singlet correlation energy dE_A + W (fixed
                     reference: dE_A of a singlet run, NaN otherwise)          */
  double E_T;     /* M_s = 0 triplet correlation energy dE_A - W (fixed
                     reference: dE_A of a triplet run, NaN otherwise)          */
  double E_ref_A; /* <A|H|A>                                                 */
} dcsd_energies;

typedef struct {
  int32_t iterations; /* residual evaluations performed                      */
  int32_t converged;  /* 1 if max |R| <= tol_residual                        */
  double res_max;     /* max |R| of the residual the report describes        */
  double res_rms;     /* root mean square of that residual over the packed
                         vector (sqrt(sum R^2 / dcsd_amplitude_count))       */
  dcsd_energies e;    /* energies of the amplitudes the report describes     */
  int32_t fp64;       /* 1 if res_max and e come from an FP64 residual (every
                         record in FP64 mode; refresh records otherwise)     */
} dcsd_report;

typedef void (*dcsd_iter_cb)(const dcsd_report* it, void* user);

/* Length of the packed amplitude vector of the two-determinant and
 * fixed-reference methods: 2 o v + 3 o^2 v^2. */
int64_t dcsd_amplitude_count(int32_t nc, int32_t nv);

/* Length of the packed amplitude vector of a method (the high-spin methods
 * have their own layout, see DCSD_METHOD_HS_*); -1 on invalid arguments. */
int64_t dcsd_method_amplitude_count(int32_t nc, int32_t nv, int32_t method);

/* Fills *cfg with defaults (DCSD, FP64, DIIS 8 from iteration 2, max_iter 200,
 * tol 1e-10, no shift, all terms, no adjoint reservation, guard_iters 10,
 * ladder_cache 1). */
void dcsd_default_config(dcsd_config* cfg);

/* Builds a context for the reference determinant Phi_A of the open-shell
 * singlet (Theory section, the two determinants of Fig. 1, with the
 * Hamiltonian given by the DF factors and the spin-averaged Fock matrix):
 * validates sizes, allocates all device work memory (with cfg->adjoint, also
 * that of the adjoint, sized by recording one residual at T = 0), and forms
 * the constant quantities of Phi_A (one-electron Hamiltonian, spin Fock
 * matrices, (ov|ov) integrals, reference energy <A|H|A>).  B_dev and F_dev are
 * borrowed, not copied: they must stay allocated and unchanged until
 * dcsd_destroy.  hip_stream may be NULL (default stream).  Returns
 * DCSD_ERR_ARG on invalid sizes or settings, DCSD_ERR_OOM when device memory
 * runs out; on failure *out is NULL and dcsd_last_error(NULL) gives the
 * reason. */
dcsd_status dcsd_init(const dcsd_config* cfg, const double* B_dev, const double* F_dev, void* hip_stream,
                      dcsd_ctx** out);

/* Residual of the 2D equations (Theory section, singles and doubles
 * equations): R = <x| e^-T H e^T |A> - [DC dropped terms] - K_x W, with
 * R at the Phi_A -> Phi_B double set to zero.  Fixed-reference methods: the
 * same first two terms with the Phi_A -> Phi_B double of T taken as +1 or -1
 * (whatever T_dev holds there), no coupling, W = 0.  T_dev and R_dev are packed
 * vectors (may not alias).  If W_host is not NULL it receives W and the call
 * synchronises; otherwise it is asynchronous. */
dcsd_status dcsd_residual(dcsd_ctx* ctx, const double* T_dev, double* R_dev, double* W_host);

/* Energies of amplitudes T (Theory section: the single-reference energy
 * expression dE_A of Phi_A, the effective coupling W = the Phi_A -> Phi_B
 * element of the doubles residual at T, and the 2x2 effective Hamiltonian
 * [[dE_A, W], [W, dE_A]] whose roots are E_S = dE_A + W and E_T = dE_A - W),
 * plus E_ref_A = <A|H|A>.  W is computed from T itself by one FP64 residual
 * evaluation into the context's work memory (whatever the precision
 * setting), so the call costs about one FP64 dcsd_residual; the
 * fixed-reference methods (W = 0, see DCSD_METHOD_*) need no residual.
 * T_dev is a packed device vector.  Synchronises.  DCSD_ERR_ARG on NULL
 * arguments. */
dcsd_status dcsd_energy(dcsd_ctx* ctx, const double* T_dev, dcsd_energies* out);

typedef struct {
  double e_t4;     /* E[4]_T: sum of N^c N^c / D                               */
  double e_st5;    /* E[5]_ST: N^c times the t1 <jk||bc> disconnected term / D */
  double e_dt;     /* N^c times the f_ia t_jk^bc disconnected term / D         */
  double e_t;      /* E_(T) = e_t4 + e_st5 + e_dt                              */
  int64_t triples; /* occupied spin-orbital triples i < j < k summed           */
} dcsd_triples_energy;

/* Perturbative triples correction E_(T) of the M_s = 1 high-spin methods
 * (DCSD_METHOD_HS_DCSD / HS_CCSD) at amplitudes T, normally the converged
 * ones.  The paper names perturbative-triples extensions of 2D-CCSD only as
 * other work (Introduction) and defines none; this is the standard
 * single-reference (T) expression applied to the single determinant Phi_T:
 * in spin orbitals
 *   N^c_ijk^abc = P(i/jk) P(a/bc) [sum_e t_jk^ae <ei||bc> - sum_m t_im^bc <ma||jk>],
 *   N^d_ijk^abc = P(i/jk) P(a/bc) [t_i^a <jk||bc> + f_ia t_jk^bc],
 *   D = f_ii + f_jj + f_kk - f_aa - f_bb - f_cc (Fock diagonal of Phi_T),
 *   E_(T) = 1/36 sum N^c (N^c + N^d) / D,
 * with P(i/jk) g = g(ijk) - g(jik) - g(kji) and P(a/bc) alike; DCSD(T) takes
 * the same expression with DCSD amplitudes.  Spin orbitals: occupied [alpha
 * core, t, u | beta core], virtual [alpha virt | beta t, u, virt].  FP64.
 * If contrib_dev is not NULL it receives, on the device, the contribution of
 * each occupied triple i < j < k (summed over all a, b, c), in lexicographic
 * order of (i, j, k): C(2 nc + 2, 3) doubles.  The first call allocates the
 * device memory of the correction and keeps it until dcsd_destroy: the
 * integrals <ei||bc> of every occupied spin orbital next to the amplitude
 * rows t_im^bc (n_occ (n_vir + n_occ) n_vir^2 doubles, n_occ = 2 nc + 2,
 * n_vir = 2 nv + 2), <jk||bc>, the spin-orbital amplitudes and one n_vir^3
 * work array.  Synchronises.  DCSD_ERR_ARG on NULL out or T
 * and for the two-determinant and fixed-reference methods, whose triples
 * correction is not defined here. */
dcsd_status dcsd_triples(dcsd_ctx* ctx, const double* T_dev, dcsd_triples_energy* out, double* contrib_dev);

/* Solves the amplitude equations starting from T_inout (zeros = the usual
 * start): Jacobi steps with orbital-energy denominators plus Pulay DIIS, all
 * vectors in FP64 on the device, until max |R| <= tol_residual.  T_inout
 * receives the converged amplitudes and *out their report; cb (may be NULL)
 * is called after every residual evaluation.  Without convergence (max_iter
 * evaluations, or the divergence guard of cfg.guard_iters giving up) the call
 * returns DCSD_ERR_NOCONV with the best amplitudes seen in T_inout (smallest
 * max |R| among FP64 evaluations, or among all evaluations if none was FP64)
 * and *out describing exactly those amplitudes (iterations = evaluations
 * performed).  DCSD_ERR_NONFINITE on Inf/NaN (T_inout then holds the best
 * amplitudes too).  Checkpoint/resume: T is the whole solver state apart from
 * the DIIS history, which a new call starts afresh.
 *
 * With precision FP32 or BF16 the iterations use the low-precision residual.
 * A refresh evaluates the FP64 residual at the current amplitudes T_r, takes
 * the step with it and records T_r: the amplitudes of the ladder with the
 * FP64 ladder result, and the changing operands of each ring GEMM with its
 * FP64 product.  After the first refresh, low-precision iterations evaluate
 * L(tau) = L(tau_r) + L_low(tau - tau_r) and A B = (A B)_r + (A - A_r) B +
 * A_r (B - B_r) with only the differences rounded, so their error shrinks
 * with |T - T_r|.  The iteration after a low-precision residual that
 * reaches tol_residual or has dropped 100-fold (BF16; 10^5-fold in FP32)
 * below the last refresh is a refresh (one FP64 evaluation), and with
 * refresh_every = k > 0 at least every k-th iteration is one.  A
 * low-precision residual that has set no new minimum for 3 iterations sits
 * on its noise floor: the FP64 residual at the same amplitudes replaces it
 * (that iteration costs one low-precision and one FP64 evaluation).
 * Convergence is declared only on a refresh whose FP64 residual meets
 * tol_residual, so the converged amplitudes solve the FP64 equations to the
 * same tolerance. */
dcsd_status dcsd_solve(dcsd_ctx* ctx, double* T_inout, dcsd_report* out, dcsd_iter_cb cb, void* user);

/* Vector-Jacobian product of one residual evaluation (hand-written reverse
 * mode through every step of dcsd_residual and of the quantities dcsd_init
 * builds from B and F).  The map is (T, B, F) -> (R, W, dE_A), R as returned by
 * dcsd_residual and dE_A the energy expression of Phi_A at T (dcsd_energy);
 * given the cotangents Rbar_dev (packed, like R), Wbar and EAbar it writes
 *   Tbar = Rbar.dR/dT + Wbar dW/dT + EAbar ddE_A/dT   (packed; 0 at the A->B double),
 *   Bbar = the same with respect to every entry of B[naux][n][n] as stored,
 *   Fbar = the same with respect to F[n][n],
 * each output optional (NULL: not computed; Bbar and Fbar NULL skips the pass
 * through the constants).  T, B and F are differentiated entry by entry as
 * stored: the packed same-spin doubles hold both t_ij^ab and t_ji^ab (and both
 * orders of a, b), so Tbar.dT is the derivative along an amplitude change only
 * for dT with that antisymmetry, and B and F are not treated as symmetric
 * matrices.  Always FP64.  Needs a context built with cfg.adjoint = 1
 * (DCSD_ERR_STATE otherwise); allocates nothing: the tape's snapshots,
 * cotangent arrays and work space were reserved by dcsd_init (about the
 * context's work memory again, plus the snapshots).  A term_mask changed
 * after init whose tape needs more snapshot memory than was reserved gives
 * DCSD_ERR_ARG. */
dcsd_status dcsd_residual_vjp(dcsd_ctx* ctx, const double* T_dev, const double* Rbar_dev, double Wbar, double EAbar,
                              double* Tbar_dev, double* Bbar_dev, double* Fbar_dev);

/* Gradient of E = ebar_S E_S + ebar_T E_T (correlation energies, E_ref
 * excluded) at converged amplitudes T_dev with respect to B and F, through the
 * Lagrangian L = E + lambda . R (Theory section: the 2D amplitude equations
 * hold at T, so dE/dB = dL/dB at the lambda solving
 * (dR/dT)^T lambda = -dE/dT, the A->B element excluded).  The lambda
 * equations are iterated like the amplitudes (Jacobi with the configured
 * denominators, DIIS, tol_residual, max_iter), starting from lambda_dev if not
 * NULL (which then receives the solution) or from zero.  Bbar_dev [naux][n][n]
 * and Fbar_dev [n][n] receive the gradient with respect to symmetric B[P] and F:
 * (G_pq + G_qp)/2, where moving both mirrored entries by h/2 changes E by
 * h (G_pq + G_qp)/2.  *out (may be NULL) reports the lambda iterations.
 * Returns DCSD_ERR_NOCONV (gradient from the last lambda) or
 * DCSD_ERR_NONFINITE like dcsd_solve.  FP64 in every precision setting;
 * needs cfg.adjoint = 1 and allocates nothing, like dcsd_residual_vjp.  A fixed-reference run has one state:
 * E = ebar_S dE_A for a singlet method, ebar_T dE_A for a triplet method (the
 * other weight is ignored). */
dcsd_status dcsd_backward(dcsd_ctx* ctx, const double* T_dev, double ebar_S, double ebar_T, double* Bbar_dev,
                          double* Fbar_dev, double* lambda_dev, dcsd_report* out);

/* Changes the solver settings of an existing context (max_iter,
 * tol_residual, level_shift, diis_start, term_mask, precond).  Sizes, method,
 * precision, diis_dim and ladder_block must equal those given to dcsd_init;
 * otherwise DCSD_ERR_ARG and nothing changes. */
dcsd_status dcsd_update_config(dcsd_ctx* ctx, const dcsd_config* cfg);

/* Kernel timing, measured with HIP events recorded on the context's stream
 * around every launch of the ladder integral assembly (DF GEMM building
 * (pc|qd) for a batch of orbital pairs), of the ladder contraction with the
 * amplitudes, of the ring GEMMs (with their operand rounding in low
 * precision), and around each whole residual evaluation.  `flops` is the
 * algorithmic count (2 per multiply-add) of the launches recorded. */
typedef struct {
  double ms;        /* summed event-to-event duration */
  int64_t launches; /* launches recorded              */
  double flops;     /* summed algorithmic flops       */
} dcsd_kernel_time;

typedef struct {
  dcsd_kernel_time assembly;    /* ladder integral assembly (MFMA, K = naux)   */
  dcsd_kernel_time contraction; /* ladder contraction (MFMA, K = (nv+2)^2)     */
  dcsd_kernel_time residual;    /* whole dcsd_residual evaluations             */
  dcsd_kernel_time ring;        /* ring GEMMs (2ov x 2ov and ov x ov blocks)   */
} dcsd_timing;

/* Starts recording (clears earlier records).  Events come from a pool of
 * host-side HIP events (no device memory) that grows when a recording needs
 * more, so no interval is dropped. */
dcsd_status dcsd_timing_start(dcsd_ctx* ctx);

/* Synchronises the stream, stops recording and sums the recorded intervals. */
dcsd_status dcsd_timing_stop(dcsd_ctx* ctx, dcsd_timing* out);

/* Device memory held by the context: *bytes (may be NULL) receives the bytes
 * it has allocated, *allocations (may be NULL) the number of device
 * allocation calls it has made since dcsd_init began.  Both stay constant
 * after dcsd_init returns (no call allocates), which is what this reports. */
dcsd_status dcsd_device_memory(const dcsd_ctx* ctx, int64_t* bytes, int64_t* allocations);

/* Message of the last error on this context ("" if none); with ctx NULL, the
 * reason the calling thread's last failed dcsd_init or
 * dcsd_selftest_gemm_layout_noalloc gave. */
const char* dcsd_last_error(const dcsd_ctx* ctx);

/* Releases all device memory of the context (NULL is allowed). */
void dcsd_destroy(dcsd_ctx* ctx);

/* Diagnostic (not part of the method): C = A * B through the library's
 * MFMA GEMM of the given precision (DCSD_PREC_*; FP32 and BF16 round A and B
 * and accumulate in FP32, splitting K when the output has few tiles), with A
 * (M x K) and B (K x N) row-major FP64 device arrays and C (M x N) row-major
 * FP64.  Returns DCSD_ERR_ARG on non-positive sizes or an unknown precision;
 * low precision allocates (and frees) temporary device memory. */
dcsd_status dcsd_selftest_gemm(int32_t precision, int64_t M, int64_t N, int64_t K, const double* A_dev,
                               const double* B_dev, double* C_dev, void* hip_stream);

/* Diagnostic (not part of the method): C = alpha * A * B + beta * C through
 * the library's FP64 GEMM with explicit operand layouts, as the method's
 * contractions call it.  A is M x K, stored m-contiguous when a_mc != 0
 * (element (m, k) at A_dev[m + k*lda]) or k-contiguous otherwise
 * (A_dev[m*lda + k]); B is K x N, stored n-contiguous when b_nc != 0
 * (B_dev[n + k*ldb]) or k-contiguous otherwise (B_dev[n*ldb + k]); C is M x N
 * row-major with leading dimension ldc and is read when beta != 0.  ksplit > 1
 * splits K into that many chunks summed by a second kernel (the library
 * allocates and frees the partial sums).  With ksplit = 1, outputs of at most
 * 16 x 16 over K >= 65536 with both operands k-contiguous take the split dot
 * product kernels, as in the method's products.  As there too, an operand
 * with an odd contiguous extent or leading dimension or a base that is not
 * 16-byte aligned is first copied, zero-padded to an even leading dimension,
 * into memory the library allocates and frees, when the output has at least
 * 128 tiles of 128 x 128 and the product at least 256 flops per copied
 * element (the direct-to-LDS kernel streams 16-byte chunks of aligned rows);
 * the other such products take the register-staged kernel.  Returns DCSD_ERR_ARG on
 * non-positive sizes, ksplit < 1 or leading dimensions smaller than the
 * stored extents. */
dcsd_status dcsd_selftest_gemm_layout(int64_t M, int64_t N, int64_t K, const double* A_dev, int64_t lda,
                                      int32_t a_mc, const double* B_dev, int64_t ldb, int32_t b_nc, double* C_dev,
                                      int64_t ldc, double alpha, double beta, int32_t ksplit, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as dcsd_selftest_gemm_layout, with the same arguments, kernels and
 * results, allocating nothing.  The scratch that call allocates (ksplit > 1:
 * ksplit * M * ldc partial sums; small outputs over a long K: one partial per
 * 2048-long K chunk and output element; the zero-padded operand copies)
 * comes from a per-GPU device array of
 * 4194304 doubles (32 MiB) that the library holds on each GPU it has run this
 * call on until the process ends; a call needing more returns DCSD_ERR_ARG
 * (dcsd_last_error(NULL) says why) without launching anything.  Every call on
 * one GPU uses that GPU's one array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.  The
 * array needs no clearing: each call writes every partial it reads. */
dcsd_status dcsd_selftest_gemm_layout_noalloc(int64_t M, int64_t N, int64_t K, const double* A_dev, int64_t lda,
                                              int32_t a_mc, const double* B_dev, int64_t ldb, int32_t b_nc,
                                              double* C_dev, int64_t ldc, double alpha, double beta, int32_t ksplit,
                                              void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LIBDCSD_H */
