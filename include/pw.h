/*
 * pw.h -- C ABI of libpwdft: plane-wave Hamiltonian application and the
 * Chebyshev-filtered block subspace iteration around it, on AMD MI355X (gfx950).
 *
 * Paper: arXiv 2507.08578 ("Abinit 2025").  Section 5.1 (GPU use for the
 * ground state) frames the hot path as a "matrix-free" diagonalisation made of
 * two operations -- applying H to a set of vectors, and the Rayleigh-Ritz
 * step -- and recommends Chebyshev filtering because it needs few Rayleigh-Ritz
 * calls; section 5.2, Eq. (ham-nl), gives the Kleinman-Bylander non-local
 * term applied through stored projectors as matrix products; section 5.4
 * uses a full-band Cholesky orthogonalisation.  Hartree atomic units
 * (section 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All functions are extern "C", never throw and never abort; they return a
 *    pw_status.  On error, outputs are unspecified, handles stay valid, and
 *    pw_last_error() holds a message.
 *  - A block of nb wavefunctions is a column-major npw x nb complex matrix
 *    (band b occupies elements [b*ld, b*ld + npw)), ld >= npw, complex values
 *    interleaved (re, im).  pw_apply_h blocks are complex128 for PW_FP64,
 *    complex64 for PW_FP32 and interleaved bfloat16 pairs (4 bytes per
 *    element: a torch bfloat16 tensor of shape (nb, ld, 2)) for PW_BF16;
 *    every other entry point takes complex128 blocks whatever its internal
 *    precision.
 *  - Precision of a call: PW_FP64 everything in FP64.  PW_FP32: FFT route in
 *    FP32, projector products with FP32 operands on the bf16 MFMA, every
 *    operand split exactly into three bfloat16 terms (six term products per
 *    real product; the accuracy of FP32 products).  PW_BF16: blocks stored
 *    as bf16 pairs (loads widen to FP32, stores round to nearest even), FFT
 *    route in FP32 (FP32 column intermediate), projector products with
 *    bfloat16 operands (the block operand read straight from its bf16
 *    storage); needs a box with the register column kernels (else
 *    UNSUPPORTED).  All accumulate in FP32.  In a pw_batch, PW_BF16 runs
 *    the filter on complex64 blocks with bfloat16 projector operands.
 *  - Pointers named *_dev are device memory on the context's device, owned by
 *    the caller; the library never frees them.  Pointers named *_host are host
 *    memory read during the call only.
 *  - Every kernel is enqueued on the stream given to pw_ctx_create.  Calls
 *    return once the work is enqueued, except where a description says the
 *    call synchronises (it then waits for that stream only).  The hot calls
 *    (pw_apply_h, pw_cheb_filter, pw_orthonormalize, pw_rayleigh_ritz,
 *    pw_lobpcg, pw_rmm_diis, pw_density after its first call) never
 *    synchronise and never allocate, so a sequence of them can be captured
 *    into a HIP graph; failures only the device can see (a Cholesky pivot,
 *    the eigensolver's sweep limit) are recorded on the device and reported
 *    by pw_ctx_check.
 *  - A context is not thread-safe; separate contexts are independent.
 */
#ifndef PW_H
#define PW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PW_OK = 0,
  PW_ERR_INVALID_ARG = 1,   /* null pointer, size or leading dimension out of range   */
  PW_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement            */
  PW_ERR_HIP = 3,           /* a HIP runtime call failed (message has the HIP string)  */
  PW_ERR_OOM = 4,           /* device allocation failed                                */
  PW_ERR_NOT_POSDEF = 5,    /* Gram matrix not numerically positive definite           */
  PW_ERR_NONFINITE = 6,     /* NaN/Inf met in a result that must be finite             */
  PW_ERR_NO_CONVERGENCE = 7 /* the dense eigensolver hit its sweep limit               */
} pw_status;

typedef enum { PW_FP64 = 0, PW_FP32 = 1, PW_BF16 = 2 } pw_prec;

typedef struct pw_ctx pw_ctx;
typedef struct pw_ham pw_ham;

/* Name of a status code (static string). */
const char* pw_status_string(pw_status s);

/* Library version string (static). */
const char* pw_version(void);

/*
 * Create a context on HIP device `device` whose work goes to `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  Errors:
 * INVALID_ARG (out == NULL, device < 0), HIP (no such device / not gfx950-
 * class LDS), OOM.
 */
pw_status pw_ctx_create(int device, void* hip_stream, pw_ctx** out);
/* Drops the caller's handle.  Hams and batches made on the context keep it
 * alive; it is freed when the last of them is destroyed, in any order. */
pw_status pw_ctx_destroy(pw_ctx* ctx);

/* Message of the last error on this context ("" if none); valid until the
 * next call on it.  pw_last_error(NULL) returns the last error of calls that
 * had no valid context. */
const char* pw_last_error(const pw_ctx* ctx);

/*
 * Deferred status of the hot calls.  A failure that only the device can see
 * -- a Cholesky pivot at or below the threshold (PW_ERR_NOT_POSDEF), a Gram
 * diagonal entry that is NaN or infinite, i.e. a column of the block that
 * is not finite (PW_ERR_NONFINITE, naming the column), the dense
 * eigensolver reaching its sweep limit (PW_ERR_NO_CONVERGENCE) -- is
 * written to a status word of the context by the kernels themselves; the
 * first one since the last check is kept, later ones are dropped, and the
 * outputs of the failing call and of every later call that used them are
 * unspecified.  pw_ctx_check synchronises the context's stream, returns that
 * status (PW_OK if none), names the call and the pivot in pw_last_error, and
 * clears the word.  Callers that read results back once per iteration
 * check once per iteration.
 */
pw_status pw_ctx_check(pw_ctx* ctx);

/*
 * Sweep limit of the dense Hermitian eigensolver inside the hot calls
 * (pw_rayleigh_ritz and the subspace steps of pw_lobpcg / pw_rmm_diis), in
 * [1, 40]; default 24.  For n > 64 the solver issues that many outer sweeps
 * with the convergence test on the device; sweeps after convergence return
 * at once.  Reaching the limit is reported by pw_ctx_check.
 */
pw_status pw_ctx_set_sweep_limit(pw_ctx* ctx, int32_t max_sweeps);

/*
 * Concurrency inside H psi (default off): the projection product P^H psi
 * runs on a second stream of the context, forked from and joined back to
 * the context's stream by events, so it overlaps the FFT route of the same
 * application; P C waits for both.  Results are bit-identical either way;
 * graph capture sees the fork and join.  Off: everything on one stream
 * (faster on the benchmarked cell, where the persistent plane kernel and
 * the projection each fill the compute units).  Applies to calls issued on
 * the context's own stream (not to a batch's branch streams).
 */
pw_status pw_ctx_set_overlap(pw_ctx* ctx, int32_t enable);

/*
 * Description of H at one k-point (section 5.2, Eq. ham-nl, norm-conserving
 * case: h_{a,ij} diagonal).
 *   n[3]     FFT box N1, N2, N3.  Each N_i must be a product of the radices
 *            2, 3, 4, 5 with a factorisation the library supports (all
 *            {2,3,5}-smooth sizes 2..256 are) and must hold the sphere:
 *            N_i >= 2*max|n_i| + 1 is NOT required (the local term is the
 *            box-periodic convolution, aliasing included), but distinct sphere
 *            points must land in distinct box cells (else INVALID_ARG).
 *   npw      number of plane waves (> 0).
 *   miller   HOST, npw x 3 int32 row-major (n1, n2, n3) per point; the order
 *            of points is the order of rows of every block.  Box index of a
 *            point: m_i = n_i mod N_i.
 *   recip    HOST-side values: rows b1, b2, b3 of the reciprocal lattice
 *            (bohr^-1), G = n1 b1 + n2 b2 + n3 b3.
 *   kpt      reduced coordinates of k; the kinetic energy is 1/2 |k + G|^2.
 *   vloc_dev DEVICE, N1*N2*N3 float64, layout [N3][N2][N1] (N1 fastest):
 *            V_loc at grid points r_j = (j1/N1, j2/N2, j3/N3) A, in Ha.
 *            Copied at creation; the caller may free it afterwards.
 *   nproj    number of projectors (>= 0).
 *   proj_dev DEVICE, npw x nproj complex128, column-major, leading dim npw:
 *            column j = <k+G|p_j>.  Referenced, not copied: it must stay
 *            valid and unchanged while the pw_ham lives.
 *   ekb      HOST, nproj float64: KB energies (diagonal of h), Ha.
 *   nb_max   largest block size that will be passed to this handle (> 0);
 *            workspaces are sized for it at creation so hot calls allocate
 *            nothing.
 *   low_prec 0: FP64 only.  1: also build the FP32 copies (projectors,
 *            V/N_box, kinetic energies, twiddles), the projectors' three-term
 *            bf16 split (projector index contiguous; 1.5x the FP32 copy's
 *            size; read by the FP32 P C) and complex64 workspaces
 *            that PW_FP32 / PW_BF16 calls need (cubic boxes of the lengths
 *            with register-resident FFT kernels; else UNSUPPORTED).
 */
typedef struct {
  int32_t n[3];
  int64_t npw;
  const int32_t* miller;
  double recip[9];
  double kpt[3];
  const double* vloc_dev;
  int64_t nproj;
  const void* proj_dev;
  const double* ekb;
  int64_t nb_max;
  int32_t low_prec;
} pw_ham_desc;

/* Build the plans (sphere columns, box extents, twiddle tables, kinetic
 * energies, scaled V copy) and workspaces.  Synchronises.  Errors:
 * INVALID_ARG, UNSUPPORTED (box size or shared-memory need beyond this GPU),
 * OOM, HIP. */
pw_status pw_ham_create(pw_ctx* ctx, const pw_ham_desc* desc, pw_ham** out);
pw_status pw_ham_destroy(pw_ham* ham);
/* Sizes the handle was built with (any pointer may be NULL). */
pw_status pw_ham_info(const pw_ham* ham, int64_t* npw, int64_t* nproj, int64_t* nb_max,
                      int64_t* ncolumns, int64_t* extent1);

/*
 * hpsi = H psi for a block of nb bands (section 5.1 "apply H to a set of
 * vectors"; section 5.2 Eq. ham-nl for the non-local part):
 *   (H psi)_g = 1/2|k+G_g|^2 psi_g + [F_fwd(V . F_bwd(scatter psi))]_g
 *               + sum_j P_gj E_j (P^H psi)_j,
 * F_bwd unnormalised with e^{+2 pi i m.j/N}, F_fwd with e^{-2 pi i m.j/N}
 * and 1/(N1 N2 N3).  psi_dev and hpsi_dev must not overlap.  1 <= nb <= nb_max.
 */
pw_status pw_apply_h(pw_ham* ham, pw_prec prec, int64_t nb, const void* psi_dev, int64_t ldpsi,
                     void* hpsi_dev, int64_t ldh);

/*
 * Electron density of a block of bands (section 2.4, Eq. nandtau; the band
 * sum of Eq. extfpmd_density in section 2.3, without its free-electron
 * term N_ext / Omega, which the caller adds):
 *   rho(r_j) [+]= (1/Omega) sum_b w_b |F_bwd(scatter psi_b)(r_j)|^2,
 * F_bwd the unnormalised e^{+2 pi i m.j/N} transform of pw_apply_h, Omega =
 * (2 pi)^3 / |det B| from the handle's reciprocal lattice; a band with unit
 * coefficient norm then holds one electron in the cell.
 *   psi_dev  DEVICE, npw x nb complex128, column-major, leading dim ldpsi >= npw
 *            (may be NULL when nb = 0).
 *   w_dev    DEVICE, nb float64: occupation times k-point weight of each band
 *            (any sign; may be NULL when nb = 0).
 *   rho_dev  DEVICE, N1*N2*N3 float64, layout [N3][N2][N1] (N1 fastest, as
 *            vloc).  accumulate = 0: overwritten (nb = 0 writes zeros);
 *            1: the block's density is added (sums over k-points).  Must not
 *            overlap psi_dev or w_dev.
 * 0 <= nb <= nb_max.  FP64 throughout.  Deterministic: every sum runs in an
 * order fixed by the handle (bands in chunks, partial sums per band group
 * added in group order).  The first call allocates the handle's partial-sum
 * array (a few x N1 N2 N3 float64; freed with the handle); later calls
 * allocate nothing.  Enqueued on the context's stream; returns without
 * synchronising.  Errors: INVALID_ARG (nb out of range, NULL pointers,
 * ld < npw, accumulate not 0/1, singular lattice), OOM, HIP.
 */
pw_status pw_density(pw_ham* ham, int64_t nb, const void* psi_dev, int64_t ldpsi,
                     const double* w_dev, double* rho_dev, int32_t accumulate);

/*
 * Chebyshev filter of degree m >= 1 (section 5.1; the paper cites the
 * filter without formulas, this is the textbook scaled three-term form):
 *   y <- p_m(H) y,  p_m(t) = T_m((t-c)/e) / T_m((a0-c)/e),  c=(a+b)/2, e=(b-a)/2,
 * run as  Y1 = (s/e)(H X - c X), Y_i = (2 s'/e)(H Y_{i-1} - c Y_{i-1}) - s s' Y_{i-2}
 * with s = e/(a0-c), s' = 1/(2/s_1 - s).  Requires a0 < a < b.
 * hx_dev (may be NULL): H X already computed (e.g. by the previous
 * Rayleigh-Ritz); then only m-1 products are formed.
 * prec PW_FP32 / PW_BF16: y and hx stay complex128; the recurrence runs on
 * complex64 (FP32) or bf16-pair (BF16) copies (y converted on entry, the
 * result converted back).
 */
pw_status pw_cheb_filter(pw_ham* ham, pw_prec prec, int32_t degree, double a, double b, double a0,
                         int64_t nb, void* y_dev, int64_t ld, const void* hx_dev, int64_t ldhx);

/*
 * Cholesky orthonormalisation (section 5.4): S = Y^H Y = U^H U (U upper,
 * positive diagonal), Y <- Y U^{-1}; if hy_dev != NULL, HY <- HY U^{-1} too.
 * U is factored in diagonal blocks of 64; Y U^{-1} is a blocked right-side
 * triangular solve (no explicit inverse).  y_dev and hy_dev must not overlap.
 * gram_prec PW_FP64: one pass.  PW_FP32 / PW_BF16 (handle made with
 * low_prec, else UNSUPPORTED): the overlap product in low precision -- S1
 * from a complex64 copy of Y on the matrix cores (FP32: three-term bf16
 * split operands; BF16: bf16 operands; FP32 accumulation) -- factored and
 * applied in FP64, then the FP64 pass above on the result (Cholesky QR
 * twice), so the final block is orthonormal to FP64 accuracy whatever S1's
 * precision.  Does not synchronise: a squared pivot at or below
 * nb * eps * max_i S_ii (either pass) is reported by pw_ctx_check as
 * PW_ERR_NOT_POSDEF naming the pivot, a column of Y holding a NaN or an
 * infinity (a non-finite S_ii) as PW_ERR_NONFINITE naming the column.
 */
pw_status pw_orthonormalize(pw_ham* ham, pw_prec gram_prec, int64_t nb, void* y_dev, int64_t ld,
                            void* hy_dev, int64_t ldhy);

/*
 * Rayleigh-Ritz (section 5.1), all in FP64: W = H Y (written to hy_dev);
 * Hs = (Y^H W + (Y^H W)^H)/2; Hs = Q diag(lambda) Q^H with lambda ascending;
 * Y <- Y Q; W <- W Q; resid_b = ||W_b - lambda_b Y_b||_2.  Y must be
 * orthonormal.  eig_dev (nb doubles) and resid_dev (nb doubles, may be NULL)
 * are device memory.  The eigensolve is cyclic Jacobi (one workgroup in LDS
 * for nb <= 64, block Jacobi above) with its convergence test on the device;
 * does not synchronise.  Reaching the sweep limit (pw_ctx_set_sweep_limit)
 * is reported by pw_ctx_check as PW_ERR_NO_CONVERGENCE.
 */
pw_status pw_rayleigh_ritz(pw_ham* ham, int64_t nb, void* y_dev, int64_t ld, void* hy_dev,
                           int64_t ldhy, double* eig_dev, double* resid_dev);

/*
 * One pass of block LOBPCG (section 5.1: the locally optimal block
 * preconditioned conjugate-gradient solver measured beside Chebyshev
 * filtering, with its block count nblock_lobpcg and line count nline; the
 * paper names it without its steps, this is Knyazev's method applied to
 * blocks of bands in turn).  All FP64.
 *   The nb bands of y_dev are orthonormalised (Cholesky), then split into
 *   nblock contiguous blocks (sizes differ by at most one, larger first).
 *   Block j: made orthogonal to the blocks below it (already updated),
 *   orthonormalised, Rayleigh-Ritzed; then nline times
 *     R = H X - X Lambda,  W = K R (Teter-Payne-Allan preconditioner:
 *       K_gb = k(T_g / Ekin_b), k(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4),
 *       Ekin_b = <x_b|T|x_b>/<x_b|x_b>),
 *     W orthogonal to the lower blocks and to X, columns normalised,
 *     orthonormalised; H W formed (the only H application of the line);
 *     P (from the second line on) orthogonal to X and W with H P alongside,
 *     normalised, orthonormalised;
 *     Rayleigh-Ritz on V = [X, W, P]: Hs = V^H (H V), Hs Z = Z Theta;
 *     X <- V Z[:, :m], P <- V[:, m:] Z[m:, :m], H X and H P by the same
 *     products, Lambda <- Theta[:m].
 *   Finally one Rayleigh-Ritz over all nb bands with the carried H X:
 *   y_dev <- Ritz vectors, hy_dev <- H y, eig_dev (nb, ascending), resid_dev
 *   (nb, may be NULL) = ||H y_b - eig_b y_b||.
 * hist_dev (may be NULL): (nline + 1) x nb doubles, hist[t nb + b] = the
 * Ritz value of band b after line t of its block (t = 0: the block's first
 * Rayleigh-Ritz).  1 <= nblock <= nb <= nb_max, 1 <= nline <= 1000; y and hy
 * must not overlap.  The first call (and a later one with a larger block or
 * nb) allocates the solver's workspace on the handle (two pairs of
 * npw x 3m blocks, m = ceil(nb / nblock), plus (3m)^2 matrices); other calls
 * allocate nothing.  Never synchronises; Cholesky and eigensolver failures
 * are reported by pw_ctx_check.
 */
pw_status pw_lobpcg(pw_ham* ham, int64_t nb, int32_t nblock, int32_t nline, void* y_dev,
                    int64_t ld, void* hy_dev, int64_t ldhy, double* eig_dev, double* resid_dev,
                    double* hist_dev);

/*
 * One RMM-DIIS pass (section 5.4: residual minimisation with direct
 * inversion in the iterative subspace; no orthogonalisation during the band
 * updates, one full-band Cholesky orthonormalisation and one subspace
 * rotation per call; the paper cites Kresse and Furthmuller for the steps).
 * Every band b of y_dev (normally Ritz vectors of an earlier solver) on its
 * own, all FP64:
 *   psi^0 = y_b; R(psi) = H psi - e(psi) psi, e(psi) = <psi|H psi>/<psi|psi>;
 *   K = the Teter-Payne-Allan preconditioner of pw_lobpcg with Ekin_b of psi^0;
 *   lam = the step minimising the Rayleigh quotient on span{psi^0, K R^0}
 *     (the lowest vector c of the 2 x 2 pencil, lam = c_1 / c_0; 0 when the
 *     two vectors are numerically dependent);  psi^1 = psi^0 + lam K R^0;
 *   for M = 1 .. ndiis - 1: alpha = the lowest vector of the pencil
 *     <R^i|R^j> alpha = e <psi^i|psi^j> alpha (i, j <= M; directions of the
 *     overlap matrix at or below 1e-12 of its largest eigenvalue dropped;
 *     alpha normalised so that alpha^H <psi|psi> alpha = 1 and sum alpha_i is
 *     real and non-negative);  psi^{M+1} = sum alpha_i psi^i
 *     + lam K sum alpha_i R^i;
 *   then y <- psi^ndiis, orthonormalised (Cholesky, H y carried), and one
 *   Rayleigh-Ritz with the carried H y: y_dev, hy_dev, eig_dev, resid_dev as
 *   in pw_lobpcg.
 * hy_valid = 1: hy_dev holds H y_dev on entry (e.g. from the previous
 * Rayleigh-Ritz) and the first application is skipped; 0: it is formed.
 * band_resid_dev (may be NULL): (ndiis + 1) x nb doubles, ||R^M_b|| /
 * ||psi^M_b|| for M = 0..ndiis.  1 <= ndiis <= 8; H is applied ndiis + 1
 * times (ndiis with hy_valid).  Workspace (2 (ndiis + 1) + 3 blocks of
 * npw x nb) allocated by the first call and by a later one with a larger nb
 * or ndiis.  Never synchronises; failures via pw_ctx_check.
 */
pw_status pw_rmm_diis(pw_ham* ham, int64_t nb, int32_t ndiis, void* y_dev, int64_t ld,
                      void* hy_dev, int64_t ldhy, int32_t hy_valid, double* eig_dev,
                      double* resid_dev, double* band_resid_dev);

/*
 * Projections kept in memory (section 5.2: the coefficients c = <p_j|psi_b>,
 * "cprj", stored for all bands so that every non-local operation is a
 * matrix product, with no approximation).  pw_rayleigh_ritz, pw_lobpcg and
 * pw_rmm_diis leave on the handle C = P^H Y for the Ritz vectors Y they
 * return: C is taken from the projection products their H applications
 * form anyway and carried through every later step by the same small
 * matrices that change Y -- (P^H Y) U^{-1} after a Cholesky solve,
 * (P^H Y) Q after a Rayleigh-Ritz rotation, C_B - C_X (X^H B) after a
 * projection, column scalings -- an nproj x nb x nb product each, never
 * P^H Y itself (nproj x npw x nb) again.  pw_ham_cprj copies the first nb
 * columns to out_dev (nproj x nb complex128, column-major, ld ldc >=
 * nproj; unscaled by the KB energies).  INVALID_ARG when the last such
 * call returned fewer than nb vectors (or failed argument checks, or none
 * ran).  nproj = 0: nothing is copied.  Enqueued; does not synchronise.
 */
pw_status pw_ham_cprj(pw_ham* ham, int64_t nb, void* out_dev, int64_t ldc);

/*
 * Upper bound of the spectrum of H used as the filter's upper edge b:
 * max_g T_g + max_r V(r) + lambda_max(D+^1/2 P^H P D+^1/2), D+ = max(E_KB, 0)
 * (each term bounds its operator from above).  Synchronises.
 */
pw_status pw_upper_bound(pw_ham* ham, double* b_host);

/* ---------------------------------------------------------------------------
 * Launch-shape tuning of H*psi.  A handle starts with the register-resident
 * FFT kernels where they exist, the largest band chunk its buffer holds and
 * 4096 target blocks for the split-K projector product (the FP64 product
 * uses at most 2048); pw_ham_autotune
 * times alternatives on the device and keeps the fastest.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t reg_col;        /* 1: register-resident column kernels (N3 in the fast set)       */
  int32_t reg_plane;      /* 1: register-resident plane kernel (N1 = N2 in the fast set)     */
  int32_t plane_variant;  /* FP64 plane kernel: 0 lane groups of up to 16 lanes; 1 up to 8
                             (N1 = N2 = 48, 64, 96)                                        */
  int32_t plane_variant32;/* FP32 plane kernel: 0, 1 as above (1 also for 120, 128, 144, 160);
                             2 transforms exchanged through LDS (N1 = N2 = 144)            */
  int32_t chunk;          /* bands per FFT launch, [1, the handle's buffer]                  */
  int32_t gemm_blocks;    /* split-K target block count of P^H psi, [1, 4096] (FP64: <= 2048) */
  int32_t nn_tile;        /* tall FP64 products P C, Y Q, Y U^-1: 0 64x64, 1 128x64 tiles    */
  int32_t nn_tile32;      /* the same choice for the FP32 / BF16 product P C                 */
  double ms;              /* pw_ham_autotune: median time of one H*psi of nb bands           */
} pw_tuning;

pw_status pw_ham_get_tuning(const pw_ham* ham, pw_tuning* t);
/* UNSUPPORTED for a kernel family the box has no kernel for. */
pw_status pw_ham_set_tuning(pw_ham* ham, const pw_tuning* t);
/*
 * Coordinate search over (1) the FFT kernel families, (2) the band chunk,
 * (3) the split-K block count, (4) the tile of the tall products, each step
 * keeping the fastest (an alternative replaces the current choice only when
 * it is more than 1% faster, above the spread of repeated timings); every
 * candidate timed as the median of reps H*psi applications of nb bands in
 * precision prec (after one warm-up) with HIP events on the context's
 * stream.  Leaves the handle at *best; *initial (may be NULL) receives the
 * starting tuning and its time.  Overwrites the handle's internal work
 * blocks; synchronises.
 */
pw_status pw_ham_autotune(pw_ham* ham, pw_prec prec, int64_t nb, int32_t reps, pw_tuning* best,
                          pw_tuning* initial);

/*
 * pw_ham_autotune behind a tuning cache file: the handle's shape key (box,
 * sphere columns and extent, npw, nproj, nb, precision) is looked up in the
 * text file cache_path (one line per key: the key, then name=value for the
 * eight tuning fields and ms); a hit whose tuning the handle accepts is
 * applied without timing (*cached = 1, initial->ms = 0); otherwise the
 * handle is tuned as by pw_ham_autotune (reps timings per candidate) and
 * the line written (the file is rewritten through a temporary and renamed;
 * not safe against concurrent writers).  cache_path NULL or "": no cache.
 * initial and cached may be NULL.  Synchronises.
 */
pw_status pw_autotune(pw_ham* ham, pw_prec prec, int64_t nb, int32_t reps, const char* cache_path,
                      pw_tuning* best, pw_tuning* initial, int32_t* cached);

/* ---------------------------------------------------------------------------
 * Batched subspace iteration over independent Hamiltonians (k-points of one
 * cell, or separate cells), section 5.1's Chebyshev-filtered iteration run
 * for many small problems at once (section 5.3 notes that the equations
 * are trivially parallel over k-points, the first level of distribution).
 *
 * One iteration of item i: filter coefficients are computed ON THE DEVICE
 * from the item's current Ritz values (a = largest, a0 = smallest) and its
 * upper bound b (pw_upper_bound, taken at creation); Y is filtered (degree
 * products, the first one reusing W = H Y of the last Rayleigh-Ritz), Gram
 * + Cholesky + Y <- Y U^{-1}, then Rayleigh-Ritz (FP64, one-workgroup Jacobi
 * eigensolve) leaving Y, W = H Y, eig and resid.  Nothing in an iteration
 * reads back to the host, so the whole iteration of every item is captured
 * once into one HIP graph (one independent branch per item, items spread
 * over the batch's streams) and replayed.
 * ------------------------------------------------------------------------- */
typedef struct pw_batch pw_batch;

/*
 * n items; for item i: hams[i] (distinct handles of this ctx, nb_max >= nb[i],
 * created with low_prec when filter_prec is not PW_FP64), nb[i] in [1, 64],
 * y_dev[i] / hy_dev[i]: complex128 npw_i x nb[i] blocks with ld = npw_i,
 * eig_dev[i] / resid_dev[i]: nb[i] doubles each.  All buffers are owned by
 * the caller and must outlive the batch; the batch keeps their addresses
 * (they are baked into the captured graph).  degree >= 1.  nstreams in
 * [1, 64]: the number of concurrent branches.  Synchronises.
 */
pw_status pw_batch_create(pw_ctx* ctx, int32_t n, pw_ham* const* hams, const int64_t* nb,
                          void* const* y_dev, void* const* hy_dev, double* const* eig_dev,
                          double* const* resid_dev, int32_t degree, pw_prec filter_prec,
                          int32_t nstreams, pw_batch** out);
pw_status pw_batch_destroy(pw_batch* b);
/* Iteration 0 of every item: orthonormalise the start block in y_dev, then
 * Rayleigh-Ritz.  Ordered after prior work on the context's stream;
 * synchronises and reports failures as pw_batch_iterate does. */
pw_status pw_batch_start(pw_batch* b);
/*
 * iters further iterations of every item.  use_graph 1: replay one
 * captured graph holding every branch; 2: replay one captured graph per
 * branch stream, each launched on its own stream (the branches then run
 * concurrently whatever the graph executor does with independent nodes);
 * 3: fused — items with the same FFT box share every launch (one kernel per
 * stage for the whole group, the items' sizes and buffers read from device
 * descriptors; needs each handle's FFT buffer to hold all nb bands), one
 * graph replayed; 4: the launches of mode 3 issued directly, without a
 * graph (with stage timing on, each stage is timed on its group's stream);
 * 0: issue the per-item kernels directly on the batch's streams.  Graphs
 * are captured on first use.  All modes compute the same
 * arithmetic item by item.  Ordered after prior work on the
 * context's stream and before later work on it.  Synchronises once at the
 * end and returns PW_ERR_NOT_POSDEF (Cholesky pivot), PW_ERR_NO_CONVERGENCE
 * (eigensolver sweep limit) or PW_ERR_INVALID_ARG (Ritz values not inside
 * a0 < a < b: that item's filter became the identity) for the first item
 * that failed in any of the iterations; pw_last_error names it.
 * With stage timing on, directly issued iterations (modes 0 and 4) are
 * timed per stage on the branch streams (kernels of concurrent branches
 * overlap, so stage sums can exceed wall time); graph replays are not timed.
 */
pw_status pw_batch_iterate(pw_batch* b, int32_t iters, int32_t use_graph);
/* The whole batched solve: pw_batch_start, then pw_batch_iterate(iters,
 * use_graph).  Synchronises; failures as pw_batch_iterate. */
pw_status pw_batch_chfsi(pw_batch* b, int32_t iters, int32_t use_graph);
/* Largest number of Jacobi sweeps any item used in the last start/iterate. */
pw_status pw_batch_max_sweeps(const pw_batch* b, int32_t* sweeps);

/* ---------------------------------------------------------------------------
 * Dense building blocks, exposed for testing and for callers that hold their
 * own subspace matrices.  All FP64 complex, column-major, device memory.
 * ------------------------------------------------------------------------- */

/* C (m x n, ldc) = alpha * A^H B with A k x m (lda), B k x n (ldb); k may be
 * large (split over the K dimension with a fixed-order reduction). */
pw_status pw_gemm_cn(pw_ctx* ctx, int64_t m, int64_t n, int64_t k, double alpha_re,
                     const void* a_dev, int64_t lda, const void* b_dev, int64_t ldb,
                     void* c_dev, int64_t ldc);
/* C (m x n, ldc) = alpha * A B + beta * C with A m x k (lda), B k x n (ldb). */
pw_status pw_gemm_nn(pw_ctx* ctx, int64_t m, int64_t n, int64_t k, double alpha_re,
                     const void* a_dev, int64_t lda, const void* b_dev, int64_t ldb,
                     double beta_re, void* c_dev, int64_t ldc);
/* Hermitian eigendecomposition a = Q diag(w) Q^H (n x n, lda) by cyclic
 * Jacobi (n > 64: block Jacobi over blocks of 16 indices, one inner sweep per
 * block pair and round): a is read only, q_dev (n x n, ldq) receives Q,
 * w_dev ascending.  Allocates its workspace, synchronises once at the end;
 * NO_CONVERGENCE after 40 sweeps. */
pw_status pw_heev(pw_ctx* ctx, int64_t n, void* a_dev, int64_t lda, double* w_dev,
                  void* q_dev, int64_t ldq);
/*
 * pw_heev for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same eigensolver and the same results as pw_heev, with its workspace
 * in a static device array of 13 MiB that every call on the device shares
 * (held by each GPU the library runs on until the process ends).  n <= 512
 * (INVALID_ARG above); a is read only.  Does not allocate and does not
 * synchronise: the sweep count goes to pw_ctx_last_sweeps and a sweep-limit
 * failure (40 sweeps) to pw_ctx_check.  Calls that overlap on one device
 * (from several contexts or streams) race on the shared array; calls on one
 * context's stream are ordered and safe.
 */
pw_status pw_heev_noalloc(pw_ctx* ctx, int64_t n, const void* a_dev, int64_t lda, double* w_dev,
                          void* q_dev, int64_t ldq);

/* Upper Cholesky factor in place: a = U^H U (upper triangle of a read and
 * overwritten; strictly lower part set to 0); then ainv_dev (n x n, ldi)
 * receives U^{-1} (upper, zeros below), formed as I U^{-1} by the same
 * blocked right-side triangular solve pw_orthonormalize applies to Y.
 * Synchronises; NOT_POSDEF as above; PW_ERR_NONFINITE when a diagonal
 * entry of a is NaN or infinite. */
pw_status pw_potrf_inv(pw_ctx* ctx, int64_t n, void* a_dev, int64_t lda, void* ainv_dev,
                       int64_t ldi);

/* ---------------------------------------------------------------------------
 * Stage timing: when enabled, every kernel launch of the hot path is
 * bracketed by HIP events on the context's stream, grouped by stage.
 * ------------------------------------------------------------------------- */
typedef enum {
  PW_STAGE_FFT_COL_INV = 0,  /* scatter + backward transform along N3 (sphere columns)   */
  PW_STAGE_FFT_PLANE = 1,    /* N2/N1 backward, x V, N1/N2 forward, per z-plane            */
  PW_STAGE_FFT_COL_FWD = 2,  /* forward along N3 + gather + kinetic + recurrence epilogue */
  PW_STAGE_PROJ = 3,         /* cprj C = P^H psi (split-K) + reduction x E_KB               */
  PW_STAGE_NONLOCAL = 4,     /* H psi += P C                                               */
  PW_STAGE_GRAM = 5,         /* Y^H Y and Y^H W                                            */
  PW_STAGE_CHOL = 6,         /* Cholesky + triangular inverse                              */
  PW_STAGE_ROTATE = 7,       /* Y U^{-1}, Y Q, W Q                                         */
  PW_STAGE_EIGH = 8,         /* dense Hermitian eigensolver                                */
  PW_STAGE_MISC = 9,         /* residuals, copies, reductions                              */
  /* the same H*psi stages run in FP32 / BF16 (low-precision filter path) */
  PW_STAGE_FFT_COL_INV_LP = 10,
  PW_STAGE_FFT_PLANE_LP = 11,
  PW_STAGE_FFT_COL_FWD_LP = 12,
  PW_STAGE_PROJ_LP = 13,
  PW_STAGE_NONLOCAL_LP = 14,
  PW_STAGE_DENSITY = 15,     /* density planes: N2/N1 backward, w |.|^2 summed (the final
                                sum of the band groups' partials counts under MISC)      */
  PW_STAGE_COUNT = 16
} pw_stage;

pw_status pw_ctx_set_timing(pw_ctx* ctx, int enable);
/* Synchronises; total milliseconds and launch count since the last reset. */
pw_status pw_ctx_stage_time(pw_ctx* ctx, int stage, double* total_ms, int64_t* launches);
pw_status pw_ctx_reset_timing(pw_ctx* ctx);
/* Sweeps used by the last dense Hermitian eigensolve on this context
 * (-1 if it hit the sweep limit).  Synchronises. */
pw_status pw_ctx_last_sweeps(const pw_ctx* ctx, int* sweeps);

#ifdef __cplusplus
}
#endif
#endif /* PW_H */
