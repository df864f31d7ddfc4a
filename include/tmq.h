/*
 * tmq.h -- C ABI of the MI355X (gfx950) twisted-mass Dirac operator and CG library.
 *
 * The library applies the even/odd preconditioned Wilson twisted-mass operator
 * and solves the normal equations with it, as stated in the paper by Jansen and
 * Urbach ("tmLQCD", Comput. Phys. Commun. 180 (2009)), Appendix B:
 *
 *   M^{+-}      = (1 +- i mut gamma_5) - kappa H                 eq. (eo0), mut = 2 kappa mu
 *   (H psi)(x)  = sum_mu [ e^{ i theta_mu pi/L_mu} U(x,mu)      (1 + gamma_mu) psi(x+mu)
 *                        + e^{-i theta_mu pi/L_mu} U(x-mu,mu)^+ (1 - gamma_mu) psi(x-mu) ]
 *                (hopping term; boundary phase spread over every hop, Sec. 4.1.2)
 *   Q^{+-}      = gamma_5 M^{+-}                                 eq. (eo1)
 *   Qhat^{+-}   = gamma_5 [ (1 +- i mut g5) - kappa^2/(1+mut^2) H_oe (1 -+ i mut g5) H_eo ]
 *                on the odd sites                                 eqs. (eo3), (eo4)
 *   solve         Qhat^+ Qhat^- x = b  (Qhat^- applied first) by CG, Sec. 4.4
 *
 * Around that path: batches of right-hand sides and a solve server (many
 * inversions per gauge field, Sec. 3.2), the full-lattice M^{+-} inversion
 * through the even/odd factorisation (App. B), BiCGstab on Qhat^{+-} (Sec. 4.4),
 * the mass non-degenerate flavour doublet (eq. (Dh)), the HMC force solves
 * (eq. (eo6)) and the one-end-trick correlators of the online measurements.
 *
 * Gamma matrices are those of Appendix A (gamma_5 = diag(1,1,-1,-1)); mu = 0:t,
 * 1:x, 2:y, 3:z.  theta_mu = 1 is antiperiodic, psi(x + L_mu) = e^{i theta_mu pi} psi(x)
 * (Sec. 2.4).
 *
 * ---------------------------------------------------------------- layouts
 * All fields crossing this boundary are little-endian complex128 (pairs of
 * double: real, imaginary), C order, in the canonical site order
 *   site = ((t*LZ + z)*LY + y)*LX + x,  dims[4] = {T, LZ, LY, LX}, all even,
 * which is the index order of the paper's propagator files (Sec. 4.7):
 *   gauge field      [site][mu][row][col]        4*9*V complex
 *   full spinor      [site][spin][colour]        12*V complex
 *   odd-site spinor  [k][spin][colour]           12*V/2 complex, k-th odd site
 *                                                 ((t+x+y+z) odd) in site order
 * Functions ending in _dev take DEVICE pointers (e.g. torch tensors' data_ptr()
 * on the lattice's device) and a hipStream_t passed as void* (NULL = the
 * default stream); work is ordered on that stream and the call returns once it
 * is enqueued unless stated otherwise.  The other functions take HOST pointers
 * and return when the result is in host memory.
 *
 * ------------------------------------------------------------- ownership
 * The caller owns every buffer it passes; the library only reads inputs and
 * writes outputs for the duration of the call (for _dev calls: until the work
 * enqueued on the stream has run).  tmq_load_gauge* copies the field: the
 * caller may free it afterwards.  A tmq_lattice owns its resident gauge copies
 * and solver work space; tmq_lattice_destroy frees them.  One lattice object
 * must not be used from two host threads at once.
 *
 * ---------------------------------------------------------------- errors
 * Every int-returning call returns TMQ_OK (0) or a negative tmq_status
 * (tmq_server_poll and tmq_server_wait also TMQ_PENDING); it never throws or
 * aborts.  tmq_last_error() returns a message for the last
 * failure on the calling thread.
 */
#ifndef TMQ_H
#define TMQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tmq_lattice tmq_lattice;

typedef enum {
    TMQ_OK = 0,
    TMQ_EINVAL = -1,  /* bad argument: odd or non-positive extent, NULL pointer, bad enum */
    TMQ_ENOMEM = -2,  /* device allocation failed, or footprint above a server budget */
    TMQ_ENOCONV = -3, /* max_iter reached; x holds the last iterate, info the true residual */
    TMQ_EDEVICE = -4, /* a HIP runtime call failed */
    TMQ_ENAN = -5,    /* a non-finite value appeared in the solver */
    TMQ_ESTATE = -6,  /* call out of order, e.g. apply before any gauge field was loaded */
    TMQ_PENDING = 1   /* tmq_server_poll / tmq_server_wait: the request has not finished yet */
} tmq_status;

/* storage precision of spinors / links on the device; arithmetic is FP64 for
 * TMQ_FP64 and FP32 otherwise.  FP16/BF16 spinors carry one FP32 scale per
 * site (scale = largest |real or imaginary part| of the site's 24 reals). */
typedef enum { TMQ_FP64 = 0, TMQ_FP32 = 1, TMQ_FP16 = 2, TMQ_BF16 = 3 } tmq_prec;

typedef struct {
    double kappa;    /* hopping parameter */
    double mu_tilde; /* mut = 2 kappa mu */
    double theta[4]; /* boundary phases along t, x, y, z (1 = antiperiodic) */
} tmq_params;

typedef struct {
    double tol;          /* stop when ||b - A x|| <= tol * ||b|| (relative) or <= tol (absolute),
                            judged on the FP64 true residual (Sec. 4.4) */
    int relative;        /* 1: relative criterion, 0: absolute */
    int max_iter;        /* bound on CG iterations (all precisions together); <= 0: 10000 */
    tmq_prec sloppy;     /* TMQ_FP64: plain FP64 CG.  FP32/FP16/BF16: mixed precision, the
                            inner CG runs FP32 arithmetic on this spinor storage */
    tmq_prec sloppy_link;/* inner link storage, TMQ_FP32 or TMQ_FP16 (two-row); ignored for FP64 */
    double delta;        /* mixed precision: recompute the FP64 true residual whenever the
                            iterated residual fell by this factor (0 < delta < 1); <= 0: default
                            (1e-4 for FP32 spinors and links, 0.01 for FP32 spinors with FP16
                            links, 0.005 for FP16 and 0.05 for BF16 spinors) */
    int mode;            /* TMQ_MODE_RELIABLE (0, default): the inner CG runs entirely in the
                            reduced precision with FP64 reliable updates (above).
                            TMQ_MODE_SWITCH (1): the paper's reduced-precision CG (Sec. 4.4):
                            FP64 vectors throughout, the FP64 operator until the relative
                            residual is below sqrt(tol), the reduced-precision operator (storage
                            `sloppy`, links `sloppy_link`) after that; convergence is still
                            declared on the FP64 true residual */
} tmq_solver_opts;

#define TMQ_MODE_RELIABLE 0
#define TMQ_MODE_SWITCH 1
#define TMQ_MODE_BICGSTAB 2 /* tmq_solve_M only: the odd-site system Qhat^{sign} psi_o = g5 phi'_o by
                               BiCGstab on Qhat itself (FP64, sloppy = TMQ_FP64) instead of CG on
                               the normal equations; the CG calls refuse it */

typedef struct {
    int status;               /* same value the call returned */
    int iters;                /* CG iterations (inner iterations for mixed precision) */
    int reliable_updates;     /* FP64 true-residual recomputations inside the solve */
    double true_rel_residual; /* ||b - A x|| / ||b|| in FP64 at exit */
    double seconds;           /* wall time of the call (host clock, includes waiting) */
} tmq_solve_info;

/* ---------------------------------------------------------------- setup */

/* Create a lattice of extents dims = {T, LZ, LY, LX} (each even, >= 2) on HIP
 * device `device`.  *out receives the handle.  TMQ_EINVAL for bad extents,
 * TMQ_EDEVICE if the device cannot be used. */
int tmq_lattice_create(const int dims[4], int device, tmq_lattice **out);

/* Free every device allocation of the lattice.  NULL is allowed. */
void tmq_lattice_destroy(tmq_lattice *lat);

/* Load a gauge field (canonical complex128 [site][mu][3][3], periodic in every
 * direction, Sec. 2.4) and build the device copies sorted for the operator:
 * per (parity, direction) structure-of-arrays, FP64 full links, and two-row
 * FP64/FP32/FP16 copies (the third row is rebuilt as conj(row0 x row1) in the
 * kernels), which every operator uses when the links are SU(3) to within 1e-12.
 * A field that fails that check (eq. (eo0) holds for any U) gets a full 3x3
 * FP32 copy as well, and then every operator keeps all three rows: FP64 full
 * links for the FP64 operator, FP32 full links for every reduced precision
 * (whatever sloppy_link asks for).  This is the paper's "double copy of the
 * gauge field sorted in access order" (Sec. 4.1).  The boundary phases are
 * never folded into the links. */
int tmq_load_gauge(tmq_lattice *lat, const double *U_host);
int tmq_load_gauge_dev(tmq_lattice *lat, const double *U_dev, void *stream);

/* 1 if the loaded links passed the SU(3) check (two-row storage in use). */
int tmq_gauge_is_su3(const tmq_lattice *lat);

/* ------------------------------------------------------------ operators */

/* out_odd = Qhat^{sign} in_odd (sign = +1 or -1), odd-site fields.  prec
 * selects the device storage: TMQ_FP64 (FP64 arithmetic, two-row FP64 links
 * when SU(3)), or FP32/FP16/BF16 spinors with FP32 arithmetic and FP32
 * (prec = FP32) or FP16 (prec = FP16/BF16) two-row links (full FP32 links
 * when the field is not SU(3), see tmq_load_gauge); the input is
 * encoded to that storage and the result decoded back to complex128.
 * in and out must not overlap. */
int tmq_apply_Qhat(tmq_lattice *lat, const tmq_params *p, int sign, tmq_prec prec,
                   const double *in_odd, double *out_odd);
int tmq_apply_Qhat_dev(tmq_lattice *lat, const tmq_params *p, int sign, tmq_prec prec,
                       const double *in_odd, double *out_odd, void *stream);

/* The same operator for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): identical arguments and result (the same kernels; the output
 * equals tmq_apply_Qhat_dev's bit for bit), but its three work fields (the
 * encoded input, the even-site intermediate and the encoded output) live in a
 * fixed array of TMQ_NOALLOC_SCRATCH_BYTES that the library's code object
 * holds on every GPU it runs on until the process ends, and the call makes no
 * hipMalloc, hipFree, event creation or other allocating call (a format the
 * autotuner has not timed on this lattice runs its default kernel variant,
 * without tuning; kernel timing is not recorded).  Device pointers only.
 * The array is shared by every lattice on the device and keeps the last
 * call's contents (each call writes all it reads): calls on one GPU must not
 * overlap in time (serialise them on one stream or wait in between).
 * TMQ_EINVAL when the three fields of this lattice in storage prec exceed the
 * array: 3 x V/2 x (192 B FP64, 96 B FP32, 52 B FP16/BF16), each rounded up to
 * 256 B (FP64 up to 16^3 x 32, FP16 up to 24^3 x 48); TMQ_EDEVICE if the
 * array's address could not be obtained when the lattice was created. */
#define TMQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int tmq_apply_Qhat_noalloc_dev(tmq_lattice *lat, const tmq_params *p, int sign, tmq_prec prec,
                               const double *in_odd, double *out_odd, void *stream);

/* out_odd = Qhat^+ Qhat^- in_odd in FP64. */
int tmq_apply_QhatQhat_dev(tmq_lattice *lat, const tmq_params *p, const double *in_odd,
                           double *out_odd, void *stream);

/* out = Q^{sign} in = gamma_5 M^{sign} in on the full lattice (eq. (eo1)), FP64,
 * full-lattice canonical spinors. */
int tmq_apply_Q_full(tmq_lattice *lat, const tmq_params *p, int sign, const double *in, double *out);
int tmq_apply_Q_full_dev(tmq_lattice *lat, const tmq_params *p, int sign, const double *in,
                         double *out, void *stream);

/* --------------------------------------------------------------- solves */

/* Solve Qhat^+ Qhat^- x = b on the odd sites, x_0 = 0.  opts->sloppy = TMQ_FP64
 * runs textbook FP64 CG; a lower precision runs CG with FP32 arithmetic on
 * reduced-precision storage and recomputes the residual b - A x in FP64 (and
 * folds the accumulated correction into the FP64 x) whenever the iterated
 * residual has dropped by opts->delta (the paper's reduced-precision CG with a
 * true-residual check, Sec. 4.4).  Returns TMQ_OK when the FP64 true residual
 * meets opts->tol, TMQ_ENOCONV after opts->max_iter iterations, TMQ_ENAN on a
 * non-finite value.  info may be NULL.  The _dev form synchronises the stream
 * before returning (the iteration is steered from the host). */
int tmq_solve(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts,
              const double *b_odd, double *x_odd, tmq_solve_info *info);
int tmq_solve_dev(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts,
                  const double *b_odd, double *x_odd, void *stream, tmq_solve_info *info);

/* Solve Qhat^+ Qhat^- x_r = b_r for nrhs right-hand sides at once
 * (1 <= nrhs <= TMQ_MAX_RHS), each with its own kappa and mu_tilde in p[r]
 * (the boundary phases must be the same for all).  The right-hand sides go
 * through every kernel launch together, so each link is fetched from HBM once
 * per half-sweep for the whole batch (many inversions per gauge field, Sec.
 * 3.2); each one still runs its own CG with its own scalars and stopping
 * test, and its result equals, bit for bit, the same solve done alone with
 * tmq_solve on this lattice.  b[r], x[r]: odd-site fields as for tmq_solve
 * (device pointers in the _dev form, host pointers otherwise); info: nrhs
 * entries or NULL.  Returns TMQ_ENAN if any right-hand side hit a non-finite
 * value, else TMQ_ENOCONV if any did not converge, else TMQ_OK. */
#define TMQ_MAX_RHS 64
int tmq_solve_batch(tmq_lattice *lat, int nrhs, const tmq_params *p, const tmq_solver_opts *opts,
                    const double *const *b, double *const *x, tmq_solve_info *info);
int tmq_solve_batch_dev(tmq_lattice *lat, int nrhs, const tmq_params *p, const tmq_solver_opts *opts,
                        const double *const *b, double *const *x, void *stream, tmq_solve_info *info);

/* Solve Q^+ Q^- x = b on the full lattice (no even/odd preconditioning) by FP64 CG.
 * Full-lattice canonical spinors; x_0 = 0. */
int tmq_solve_full_dev(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts,
                       const double *b, double *x, void *stream, tmq_solve_info *info);

/* Solve Qhat^{sign} x = b on the odd sites by BiCGstab (one of the solvers the
 * paper lists for D chi = phi, Sec. 4.4) applied to the non-Hermitian
 * operator itself: two applications of Qhat per iteration, against four (one
 * Qhat^+ Qhat^-) for a CG iteration on the normal equations.  FP64 only
 * (opts->sloppy must be TMQ_FP64; opts->mode is ignored).  x_0 = 0; the
 * iteration stops on the iterated residual, then the FP64 true residual
 * b - Qhat x is recomputed: the solve ends if it meets opts->tol, otherwise
 * BiCGstab restarts from it (also after a breakdown, rho or omega = 0).
 * info->iters = BiCGstab iterations, info->reliable_updates = true-residual
 * recomputations, info->true_rel_residual = |b - Qhat x| / |b|.  Odd-site
 * canonical fields; TMQ_ENOCONV if max_iter is reached. */
int tmq_solve_Qhat(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts, const double *b,
                   double *x, tmq_solve_info *info);
int tmq_solve_Qhat_dev(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts,
                       const double *b, double *x, void *stream, tmq_solve_info *info);

/* Solve M^{sign} psi = phi on the full lattice (eq. (eo0), sign = +1 or -1)
 * with the even/odd factorisation of App. B ("Inversion"):
 *   phi'_e = (M_ee)^-1 phi_e,  phi'_o = phi_o - M_oe (M_ee)^-1 phi_e,
 *   psi_o = (M_oo - M_oe (M_ee)^-1 M_eo)^-1 phi'_o,
 *   psi_e = phi'_e - (M_ee)^-1 M_eo psi_o,
 * where the odd-site operator is gamma_5 Qhat^{sign}, inverted by the CG of
 * tmq_solve on Qhat^+ Qhat^- (options as there, mixed precision included):
 * psi_o = Qhat^- A^-1 g5 phi'_o (sign +1) or A^-1 Qhat^+ g5 phi'_o (sign -1).
 * The residual phi - M psi is then recomputed in FP64 on the full lattice and,
 * while it is above opts->tol (relative to |phi| or absolute), the same steps
 * solve for the correction (at most 4 rounds).  info->true_rel_residual is that
 * full-lattice residual, info->iters the CG iterations of all rounds.
 * With opts->mode = TMQ_MODE_BICGSTAB the odd-site system is solved by
 * BiCGstab on Qhat^{sign} directly (as tmq_solve_Qhat), FP64.
 * Full-lattice canonical spinors; phi and psi must not overlap.  TMQ_ENOCONV if
 * the tolerance is not reached. */
int tmq_solve_M(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts,
                const double *phi, double *psi, tmq_solve_info *info);
int tmq_solve_M_dev(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts,
                    const double *phi, double *psi, void *stream, tmq_solve_info *info);
/* n full-lattice sources with common parameters (1 <= n <= TMQ_MAX_RHS), e.g.
 * the 12 spin-colour point sources of a propagator (Sec. 3.2, the inversion
 * program): the steps above run on all of them together, the odd-site CG as one
 * batch (links read once per half-sweep for the batch); each source keeps its
 * own correction rounds, status and info[r], and psi[r] equals what
 * tmq_solve_M_dev gives for phi[r] alone.  Device pointers; no psi[r] may
 * overlap another psi or any phi.  Returns the worst status (TMQ_ENAN before
 * TMQ_ENOCONV). */
int tmq_solve_M_batch_dev(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts, int n,
                          const double *const *phi, double *const *psi, void *stream, tmq_solve_info *info);

/* ------------------------------------------------- flavour doublet */

/* The mass non-degenerate doublet of eq. (Dh), D_h = D_W 1_f + i mubar g5 tau^3
 * + epsbar tau^1, in the hopping normalisation of eq. (eo0):
 *   M_h = A - kappa H 1_f,   A = 1 + i mubar g5 tau^3 + epsbar tau^1,
 *   Q_h = g5 M_h,
 * and its even/odd reduction on the odd sites (App. B, the doublet's Q^h_oo)
 *   Qhat_h^{+-} = g5 [ A_oo - kappa^2 H_oe A_ee^-1 H_eo ],
 *   A^-1 = (1 - i mubar g5 tau^3 - epsbar tau^1) / (1 + mubar^2 - epsbar^2),
 * with mubar -> -mubar for the minus sign, so that (Qhat_h^+)^dagger =
 * Qhat_h^-.  The printed eq. (Dheo) carries epsbar with the opposite sign,
 * which is the flavour rotation tau^3 of this operator (same spectrum).
 * Solves are CG on Qhat_h^+ Qhat_h^- x = b (Qhat_h^- first), with the options
 * of tmq_solve (mixed precision and modes included).
 * Doublet fields are complex128 [2][V/2][4][3]: the upper flavour's odd-site
 * field, then the lower's, each in the odd-site order above. */
typedef struct {
    double kappa;        /* hopping parameter */
    double mubar_tilde;  /* 2 kappa mubar */
    double epsbar_tilde; /* 2 kappa epsbar; 1 + mubar_tilde^2 - epsbar_tilde^2 must be > 0 */
    double theta[4];     /* boundary phases along t, x, y, z (1 = antiperiodic) */
} tmq_nd_params;

/* out = Qhat_h^{sign} in, storage precision prec as for tmq_apply_Qhat. */
int tmq_apply_Qhat_nd(tmq_lattice *lat, const tmq_nd_params *p, int sign, tmq_prec prec, const double *in,
                      double *out);
int tmq_apply_Qhat_nd_dev(tmq_lattice *lat, const tmq_nd_params *p, int sign, tmq_prec prec, const double *in,
                          double *out, void *stream);
/* Solve Qhat_h^+ Qhat_h^- x = b; x_0 = 0; info as for tmq_solve (the
 * residual is over both flavours). */
int tmq_solve_nd(tmq_lattice *lat, const tmq_nd_params *p, const tmq_solver_opts *opts, const double *b, double *x,
                 tmq_solve_info *info);
int tmq_solve_nd_dev(tmq_lattice *lat, const tmq_nd_params *p, const tmq_solver_opts *opts, const double *b,
                     double *x, void *stream, tmq_solve_info *info);
/* n doublets (1 <= n <= TMQ_MAX_RHS / 2) solved together, each with its own
 * kappa, mubar and epsbar (common theta), links read once per half-sweep for
 * all of them; each result equals its solve alone bit for bit. */
int tmq_solve_nd_batch_dev(tmq_lattice *lat, int n, const tmq_nd_params *p, const tmq_solver_opts *opts,
                           const double *const *b, double *const *x, void *stream, tmq_solve_info *info);

/* ---------------------------------------------- consumers of the solver */

/* The solves of the HMC fermion force (eq. (eo6)): X_o = (Qhat^+ Qhat^-)^-1 phi_o
 * (tmq_solve with opts) and Y_o = Qhat^- X_o (FP64), whose combination
 * -[X_o^+ dQhat^+ Y_o + Y_o^+ dQhat^- X_o] is the variation of the pseudo-fermion
 * action (eq. (eo5)).  Y may be NULL (not computed); action != NULL (host)
 * receives S_PF = Re phi_o^+ X_o.  With phi_o = Qhat^+ r_o (the heatbath of
 * eq. (eo10)), Y_o = r_o and S_PF = |r_o|^2 up to the tolerance.  Odd-site
 * canonical device fields that must not overlap; info as for tmq_solve.
 * Returns when the action is on the host (else when enqueued). */
int tmq_solve_force_dev(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts, const double *phi,
                        double *X, double *Y, double *action, void *stream, tmq_solve_info *info);

/* Time-slice sums of a spin bilinear of a full-lattice field:
 *   out[t] = sum over the sites x of time slice (t0 + t) mod T of
 *            sum_colour psi(x)^+ Gamma psi(x),
 * gamma = the 4x4 complex spin matrix Gamma, row-major (host, 16 complex),
 * psi = full-lattice canonical field (device), out = T complex (host; the call
 * returns when it is written).  The contraction of the one-end-trick
 * correlators (eq. (oneend)): for phi = M^-1 xi, Gamma = 1 gives the
 * pseudoscalar correlator, other Gamma the source-side insertions. */
int tmq_timeslice_bilinear_dev(tmq_lattice *lat, const double *gamma, const double *psi, int t0, double *out,
                               void *stream);

/* One-end-trick estimator of the pseudoscalar correlator for one noise
 * sample (eqs. (source), (oneend)): phi = (M^+)^-1 xi by tmq_solve_M with
 * opts, then corr[t] = sum over the spatial sites at time (t0 + t) mod T of
 * |phi|^2 (spin and colour summed), t = 0 .. T-1 (host, T doubles).  xi is a
 * full-lattice canonical device field, normally a noise source on time slice
 * t0 whose components satisfy [xi_i^* xi_j] = delta_ij over samples (drawn by
 * the caller); the average over samples estimates tr[G G^+] for G = M^-1 in
 * the hopping normalisation of eq. (eo0) (the conventionally normalised
 * propagator is 2 kappa G).  phi (device, full canonical) receives the
 * solution if not NULL.  info as for tmq_solve_M. */
int tmq_pion_correlator_dev(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts, const double *xi,
                            int t0, double *corr, double *phi, void *stream, tmq_solve_info *info);

/* Even/odd split and merge of canonical spinor fields (App. B: the even/odd
 * decomposition of a field): full = complex128 [V][4][3] over lexicographic
 * sites, even/odd = complex128 [V/2][4][3] over the sites of that parity in
 * the same order (eo index = site >> 1), the layout of every odd-site call
 * above.  A copy: no arithmetic.  Split: either output may be NULL (not
 * written).  Merge: a NULL parity is taken as zero.  The buffers must not
 * overlap.  The gauge field need not be loaded.  *_dev: device pointers,
 * ordered on the stream. */
int tmq_split_eo(tmq_lattice *lat, const double *full, double *even, double *odd);
int tmq_merge_eo(tmq_lattice *lat, const double *even, const double *odd, double *full);
int tmq_split_eo_dev(tmq_lattice *lat, const double *full, double *even, double *odd, void *stream);
int tmq_merge_eo_dev(tmq_lattice *lat, const double *even, const double *odd, double *full, void *stream);

/* ---------------------------------------------------------------- serving */

/* A solve server: a stream of independent even/odd solves (each a request
 * with its own lattice, kappa, mu_tilde, source and tolerance) served on one
 * device, the pattern of the paper's inversion program that solves on many
 * sources and masses per gauge configuration (Sec. 3.2) turned into a
 * long-running service.
 *
 * Lattices (gauge fields) are registered once and stay resident.  A request
 * runs in a CG engine: batch work fields with a number of slots, one engine
 * per (lattice, inner precision, inner link format, boundary phases), each on
 * its own HIP stream, so different lattice sizes overlap on the device.
 * Continuous batching: a request joins a free slot of its engine at the next
 * iteration boundary and leaves as soon as its FP64 true residual meets its
 * tolerance; the others keep iterating.  Every iteration advances all slots of
 * an engine in the same kernel launches (links read once per half-sweep for
 * all of them).  A request computes exactly what tmq_solve computes for it
 * on the server's lattice, whatever else is in flight: its result does not
 * depend on the mix.
 *
 * Admission by device-memory footprint: engines hold the work fields of all
 * their slots (tmq_footprint_bytes less the gauge copies, per slot); the sum
 * over engines never exceeds the server's budget.  A request waits in the
 * queue until a slot of its engine is free or memory for one can be found
 * (idle engines of other keys are released for it); requests of other keys
 * may pass a waiting one.  A request whose single slot exceeds the whole
 * budget is rejected at submission with TMQ_ENOMEM; one whose engine the
 * device cannot allocate while no other engine exists finishes with
 * TMQ_ENOMEM.
 *
 * Threads: the server runs one worker thread that drives every engine; all
 * tmq_server_* calls are thread-safe.  Fields are DEVICE pointers on the
 * server's device in the odd-site canonical layout of tmq_solve_dev.  The
 * server's streams do not wait for the caller's: b must hold its values when
 * tmq_server_submit is called (work producing it has completed), and the
 * caller keeps b and x alive and untouched until the request has finished
 * (poll/wait returned something other than TMQ_PENDING); x is complete then. */
typedef struct tmq_server tmq_server;

typedef struct {
    size_t budget_bytes; /* device memory for the engines' work fields; 0: 60% of the
                            device memory free at creation */
    int max_batch;       /* slots per engine, 1..TMQ_MAX_RHS; <= 0: 16 */
} tmq_server_config;

typedef struct {
    long submitted, completed, failed, rejected; /* failed: finished with a non-OK status */
    long queued, running;        /* now: waiting for admission / admitted and not finished */
    double p50_s, p99_s, mean_s; /* latency submit -> result ready, completed requests */
    double mean_wait_s;          /* time from submission to admission, completed requests */
    double solves_per_s;         /* completed / (last completion - first submission) */
    double elapsed_s;            /* first submission -> last completion */
    size_t budget_bytes, bytes_in_use, peak_bytes;
    int engines, peak_running;   /* engines now, largest number of requests admitted at once */
    long steps;                  /* engine iteration steps driven */
} tmq_server_stats;

/* Create a server on HIP device `device`; cfg may be NULL (defaults). */
int tmq_server_create(int device, const tmq_server_config *cfg, tmq_server **out);

/* Register a lattice: extents dims as for tmq_lattice_create and its gauge
 * field as for tmq_load_gauge_dev (device pointer; copied, the caller may free
 * it on return).  *lattice_id receives the id used by tmq_server_submit. */
int tmq_server_add_lattice(tmq_server *srv, const int dims[4], const double *U_dev, int *lattice_id);

/* Queue a solve of Qhat^+ Qhat^- x = b on lattice lattice_id (options as for
 * tmq_solve).  *ticket receives the request's id.  TMQ_EINVAL for bad
 * arguments, TMQ_ENOMEM if one slot for it exceeds the budget, TMQ_EDEVICE
 * if the server has failed. */
int tmq_server_submit(tmq_server *srv, int lattice_id, const tmq_params *p, const tmq_solver_opts *opts,
                      const double *b_dev, double *x_dev, uint64_t *ticket);

/* TMQ_PENDING while the request is queued or running.  Once it has finished
 * (x written), returns its status (as tmq_solve would), fills info (seconds =
 * latency from submission to result) if non-NULL and retires the ticket;
 * TMQ_EINVAL for an unknown or retired ticket. */
int tmq_server_poll(tmq_server *srv, uint64_t ticket, tmq_solve_info *info);
/* As poll, waiting up to timeout_s seconds (< 0: without limit). */
int tmq_server_wait(tmq_server *srv, uint64_t ticket, double timeout_s, tmq_solve_info *info);

/* Counters and latency figures since creation or the last reset. */
int tmq_server_get_stats(tmq_server *srv, tmq_server_stats *out);
int tmq_server_reset_stats(tmq_server *srv);

/* Stop the worker after the requests in flight have finished (queued ones
 * are dropped), free every engine and lattice.  NULL is allowed. */
void tmq_server_destroy(tmq_server *srv);

/* ---------------------------------------------------------- diagnostics */

/* Per-kernel timing with HIP events recorded on the launch stream around each
 * hopping half-sweep launch (timing-only events, without the system-scope
 * cache writeback a default event performs), off by default.  tmq_set_kernel_timing
 * synchronises the device and clears the records.  tmq_kernel_stats returns,
 * for the launches recorded since then, their number, total time in ms, and
 * the algorithmic bytes and flops they move (each input spinor, link and
 * output counted once; 1320 flop per output site per half-sweep; a fused CG
 * epilogue adds its reads of r and p and its read and write of x, a fused
 * residual its read of b).  family is "hop" (all), "hop64", "hop32" or "hop16"
 * (FP16 and BF16 spinor storage), optionally followed by ":pure" (the plain
 * half-sweeps K1 and K2 of eqs. (eo3)/(eo4) only), ":k1", ":k2" or ":fused"
 * (the half-sweeps whose epilogue carries the CG update or the true residual).
 * Reading the stats synchronises the device. */
int tmq_set_kernel_timing(tmq_lattice *lat, int on);
int tmq_kernel_stats(tmq_lattice *lat, const char *family, int *launches, double *total_ms,
                     double *bytes, double *flops);

/* Calibration: copy `bytes` (rounded down to 16) between two device buffers
 * with a plain 16-byte-per-lane kernel, `reps` times after one warm-up, and
 * report the achieved read + write bandwidth in GB/s.  Allocates and frees
 * its own buffers on `device`. */
int tmq_stream_copy(int device, size_t bytes, int reps, double *gbps);

/* JSON text of the autotuner's choices so far: for every (spinor storage,
 * link format) used on this lattice, the hop kernel variant picked, the
 * measured microseconds per launch of each variant (-1: not applicable), and
 * the cap on resident blocks per CU picked for it (0: none) with the time of
 * each cap tried.  The variants order the blocks of each XCD differently: 0
 * lexicographic (an eighth of the time-slices per XCD); 1 each XCD walks its
 * own range of z-planes time-slice by time-slice (needs LZ >= 8); 2 as 1 with
 * scheduling barriers between directions; 3 each XCD walks its own range of
 * time-slices z-plane by z-plane (needs T >= 8); 4 as 3 with barriers.  The
 * tuner runs at the first launch of each format on a lattice;
 * TMQ_HOP_VARIANT=0..4 in the environment forces a variant and
 * TMQ_HOP_CAP=0..5 a cap (single-field and batched launches).  Batched
 * launches list, per (format, power-of-two batch size class), the RHS per
 * lane, the RHS group and the cap picked, the time of the picked shape under
 * each cap tried, and every (RHS per lane, group, us) tried.  TMQ_EINVAL if
 * buf (len bytes) is too small. */
int tmq_tuning_report(tmq_lattice *lat, char *buf, size_t len);

/* Encode n_sites canonical complex128 sites (12 complex each) into the device
 * FP16 (prec = TMQ_FP16) or BF16 storage and export the codes in canonical
 * order: codes[n_sites][24] (real, imaginary of spin-colour component k at
 * 2k, 2k+1) and scale[n_sites] (FP32).  Device pointers.  Used to check the
 * codec bit for bit. */
int tmq_encode_dev(tmq_lattice *lat, tmq_prec prec, long n_sites, const double *in,
                   uint16_t *codes, float *scale, void *stream);

/* Device memory (bytes) the lattice would hold for its gauge copies plus the
 * work space of one solve with these options (opts may be NULL: FP64). */
int tmq_footprint_bytes(const int dims[4], const tmq_solver_opts *opts, int nrhs, size_t *out);

/* Message of the last error on this thread ("" if none). */
const char *tmq_last_error(void);

/* Library version string. */
const char *tmq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TMQ_H */
