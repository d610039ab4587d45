/*
 * ddsolve.h -- C ABI of the MI355X (gfx950) Clover-Wilson quark solver:
 * Dirac apply, SAP domain-decomposition preconditioner, BiCGStab with
 * mixed-precision defect correction.
 *
 * The operator is the Clover-Wilson Dirac matrix of arXiv 2109.10687,
 * appendix "Clover-Wilson Dirac operator":
 *
 *     D = 1 + C - kappa H,
 *     (H x)(n) = sum_mu [ (1 - gamma_mu) U_mu(n) x(n+mu)
 *                        + (1 + gamma_mu) U_mu(n-mu)^dagger x(n-mu) ],
 *     C = (i/2) kappa c_SW sigma_{mu nu} F_{mu nu}(n)   (four-leaf F),
 *
 * with the gamma matrices printed there (Dirac representation, gamma_4
 * diagonal), and A = C_inv D = I - kappa C_inv H with C_inv = (1 + C)^{-1}
 * (Sec. 3).  The Schwarz preconditioner M_SAP is Alg. 1 of Sec. 3 with the
 * block Jacobi of Alg. 2; BiCGStab is Alg. 5; the mixed-precision outer loop
 * is the defect correction of Alg. 4.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Lattice dims = {Lx, Ly, Lz, Lt}; direction mu = 0..3 is the paper's
 *    mu = 1..4 (mu = 3 is the direction of gamma_4).  Lexicographic site
 *    index n = x + Lx*(y + Ly*(z + Lz*t)).
 *  - Canonical spinor field: complex double (re, im interleaved), layout
 *    [Lt][Lz][Ly][Lx][colour 3][spin 4] -- the paper's K-computer order
 *    (Sec. 4): colour outer, spin inner.  24 doubles per site.
 *  - Canonical gauge field: complex double, [mu 4][Lt][Lz][Ly][Lx][3][3],
 *    U_mu(n)[a][b] row-major.  Links should be SU(3); the 12-real FP16 copy
 *    rebuilds the third row from the first two, which holds only for SU(3).
 *  - Boundary conditions are not stated in the paper: a hop that crosses
 *    the lattice edge in direction mu is multiplied by phase_mu (forward)
 *    or conj(phase_mu) (backward).  {1, 1, 1, -1} is periodic in space and
 *    antiperiodic in time.  The clover term is built from the links alone.
 *  - All *_dev pointers are device (HBM) addresses owned by the caller;
 *    the library never frees them.  The library owns its packed fields and
 *    work vectors, freed in dd_destroy: dd_create allocates those of the
 *    Dirac apply, the SAP and the solve modes DD_SOLVE_F64_PLAIN,
 *    DD_SOLVE_F32_SAP and DD_SOLVE_MIXED; the GCR and flexible GMRES modes,
 *    the batched solves and dd_force allocate their extra fields on first use
 *    (DD_ERR_NOMEM if that fails) and keep them.  dd_force_noalloc never
 *    allocates.
 *  - Work runs on the HIP stream given to dd_create (NULL = default stream).
 *    dirac_apply and sap_precondition are asynchronous on that stream;
 *    bicgstab_solve synchronises it.
 *  - Every function returns a dd_status and never throws.  A negative status
 *    means the outputs were not written; dd_last_error gives the reason.
 *  - A context is not thread-safe: use one context per host thread.
 */
#ifndef DDSOLVE_H
#define DDSOLVE_H

/* the library is built with hidden visibility; the declarations below are its
 * only exported symbols */
#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility push(default)
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DD_OK = 0,
    DD_NOT_CONVERGED = 1,      /* maxiter reached; x holds the last iterate       */
    DD_BREAKDOWN = 2,          /* a BiCGStab denominator vanished or went non-finite */
    DD_ERR_ARG = -1,           /* null pointer, bad enum, bad tolerance            */
    DD_ERR_GEOMETRY = -2,      /* dims/blocks not compatible (see dd_params)       */
    DD_ERR_HIP = -3,           /* a HIP runtime call failed                        */
    DD_ERR_NOMEM = -4,         /* device allocation failed in dd_create            */
    DD_ERR_NONFINITE = -5,     /* the source or the gauge field holds NaN or Inf   */
    DD_ERR_CLOVER_NOT_PD = -6, /* 1 + C is not positive definite at some site      */
    DD_ERR_STATE = -7          /* no gauge field loaded yet                        */
} dd_status;

typedef enum { DD_F64 = 0, DD_F32 = 1, DD_F16 = 2 } dd_prec;

typedef enum {
    DD_OP_D = 0,    /* D x = (1 + C) x - kappa H x                         */
    DD_OP_A = 1,    /* A x = x - kappa C_inv H x                           */
    DD_OP_DDAG = 2  /* D^dagger x = gamma_5 D gamma_5 x                    */
} dd_op;

typedef enum {
    /* plain BiCGStab (Alg. 5 without preconditioner) on D in FP64; tol is the
     * true relative residual |b - D x| / |b|, recomputed at exit */
    DD_SOLVE_F64_PLAIN = 0,
    /* BiCGStab on A M_SAP in FP32 with an FP32 SAP preconditioner, source
     * C_inv b, zero start (Alg. 5 as printed); tol is Alg. 5's test on the
     * recursive FP32 residual of the A-system */
    DD_SOLVE_F32_SAP = 1,
    /* defect correction (Alg. 4) in FP64 around FP32 SAP-BiCGStab with an FP16
     * preconditioner (per-site-scaled FP16 spinors, 12-real FP16 links, FP16
     * C_inv); tol is the true FP64 relative residual |b - D x| / |b| */
    DD_SOLVE_MIXED = 2,
    /* as DD_SOLVE_MIXED, but the inner FP32 solver is restarted flexible GCR
     * (cycle length gcr_nkv) right-preconditioned by the FP16 SAP: the flexible
     * alternative to BiCGStab that Sec. 3 names for a preconditioner that varies
     * between applications, as a rounded FP16 SAP does.  Each inner iteration
     * applies M_SAP and A once; the residual never grows. */
    DD_SOLVE_MIXED_GCR = 3,
    /* restarted flexible GMRES on D in FP64 (cycle length fgmres_nkv) in place of
     * the defect correction: the outer loop Sec. 3 proposes, with the FP32
     * SAP-BiCGStab of DD_SOLVE_MIXED (FP16 SAP) as a flexible preconditioner
     * that may differ from one application to the next.  Each outer iteration
     * runs one inner solve of A z = C_inv v for the current Arnoldi vector v and
     * keeps z; the solution minimises the FP64 residual over the kept z.  tol
     * is the true FP64 relative residual; maxiter bounds the outer iterations. */
    DD_SOLVE_FGMRES = 4
} dd_solve_mode;

typedef struct {
    int dims[4];        /* Lx, Ly, Lz, Lt                                       */
    int block[4];       /* SAP block extent per direction: a power of two in 2..16,
                           block volume <= 256, dims[mu] / block[mu] even          */
    double kappa;       /* hopping parameter                                     */
    double csw;         /* clover coefficient c_SW                               */
    double phase_re[4]; /* boundary phase per direction                          */
    double phase_im[4];
    int n_sap;          /* loop count of Alg. 1: M = K sum_{j=0}^{n_sap} (1 - A K)^j;
                           the paper's runs use 4.  A longer series makes a stronger
                           preconditioner while it converges, but near the critical
                           kappa it grows on the low modes (measured on 32^4 at kappa
                           0.1365, N_JAC 4: fastest at 6, slower at 9, breakdown from 10) */
    int n_jac;          /* A_EE applications in Alg. 2: B = sum_{j=0}^{n_jac} (1 - A_EE)^j */
    double inner_tol;   /* relative tolerance of each inner FP32 solve in DD_SOLVE_MIXED
                           (0 = 1e-6, the per-pass reduction Sec. 3 expects); a pass
                           whose start is already close to tol stops earlier       */
    int inner_maxiter;  /* iteration cap of each inner solve (0 = 2000)            */
    int gcr_nkv;        /* GCR cycle length for DD_SOLVE_MIXED_GCR, 1..16 (0 = 16); the
                           first such solve allocates gcr_nkv FP32 and FP16 fields   */
    int sap_fp16_arith; /* 1: the FP16-storage SAP (sap_precondition at DD_F16 and the
                           mixed modes) also does its block-local Jacobi sweeps in
                           packed FP16 arithmetic, on a source scaled per block to unit
                           maximum; 0: FP32 arithmetic on FP16 storage.  A zeroed
                           dd_params gives 0; the Python binding's default is 1      */
    int stall_window;   /* an inner FP32 solve stops (status detail 6) when its recursive
                           residual has not fallen 10x below the last such point within
                           this many iterations (0 = 200; negative = never)          */
    int sap_fused_tail; /* FP32 SAP-BiCGStab (DD_SOLVE_F32_SAP and the first fallback level):
                           1 forms A M_SAP by the fused tail of Alg. 3; 0 (default, as fast or
                           faster where measured) applies A separately to the SAP's output
                           (the same product, other rounding order)                  */
    int fgmres_nkv;     /* flexible GMRES cycle length for DD_SOLVE_FGMRES, 1..16 (0 = 4);
                           the basis takes four FP64 and the directions three FP32 work
                           vectors of the context, the first such solve allocates the
                           rest (fgmres_nkv - 3 FP64, fgmres_nkv - 3 FP32 fields)    */
    int no_fallback;    /* DD_SOLVE_MIXED / DD_SOLVE_MIXED_GCR: 0 (default) falls back in
                           precision when a defect-correction pass stagnates or its inner
                           solve breaks down (the mode's FP16-SAP inner solve, then FP32
                           SAP-BiCGStab, then plain FP64 BiCGStab from the current x),
                           except that the first such pass of a level that still cut the
                           true residual 10x is followed by a restarted pass of the same
                           level; 1 returns DD_BREAKDOWN there instead                */
    int debug_flags;    /* forces failures from the host, for tests: DD_DEBUG_ZERO_OMEGA_F16
                           sets omega = 0 in every FP16-SAP BiCGStab iteration,
                           DD_DEBUG_ZERO_OMEGA_F32 in every FP32-SAP one (0 = none)   */
} dd_params;

#define DD_DEBUG_ZERO_OMEGA_F16 1
#define DD_DEBUG_ZERO_OMEGA_F32 2

typedef struct {
    int iters_outer;          /* defect-correction passes or flexible GMRES iterations
                                 (1 for the single-level modes)                   */
    int iters_inner_total;    /* BiCGStab loop passes summed over all solves      */
    double relres_true;       /* |b - D x| / |b| in FP64 at exit                  */
    double relres_inner_last; /* last recursive residual of the last inner solve  */
    double seconds;           /* wall time of the call                            */
    int status_detail;        /* which breakdown: 1 <r~|q> = 0, 2 |t|^2 = 0, 3 omega = 0,
                                 4 non-finite scalar, 5 outer stagnation (a defect-
                                 correction pass did not lower the true residual, or
                                 lowered it by less than 10% twice in a row), 6 inner
                                 stagnation (an inner solve hit the stall window of
                                 dd_params and its pass gained less than 10x)      */
    int status;               /* the dd_status of this solve: the return value of a
                                 single solve, this right-hand side's (lattice's) own
                                 outcome in the batched and multi-lattice solves  */
    int precision_level;      /* inner solver the solve ended with: 0 the mode's own,
                                 1 FP32 SAP-BiCGStab, 2 plain FP64 BiCGStab (levels
                                 1 and 2 only after a fallback, see no_fallback)  */
} dd_solve_info;

typedef struct dd_ctx dd_ctx;

/* Create a context: checks the geometry, allocates every packed field and work
 * vector for all three solve modes (about 4.6 KB per site), binds the stream.
 * hip_stream is a hipStream_t (NULL = default stream).  Geometry rules: each
 * dims[mu] is a multiple of 2*block[mu]; block[mu] is a power of two; the block
 * volume is at most 256 (one workgroup per block, one thread per site).
 * Returns DD_ERR_GEOMETRY or DD_ERR_NOMEM on failure. */
dd_status dd_create(const dd_params *params, void *hip_stream, dd_ctx **out);

/* Free every device buffer the context owns.  NULL is accepted. */
dd_status dd_destroy(dd_ctx *ctx);

/* Load a gauge field (canonical layout, device memory, read only): packs the
 * FP64, FP32 and 12-real FP16 link copies, builds the four-leaf clover in
 * FP64, 1 + C as two 6x6 Hermitian blocks in the gamma_5-diagonal basis, and
 * C_inv by a Cholesky inverse in FP64 (stored in FP32 and FP16).  Synchronises
 * the stream.  DD_ERR_CLOVER_NOT_PD if 1 + C fails the Cholesky at any site,
 * DD_ERR_NONFINITE if a link holds NaN or Inf. */
dd_status dd_load_gauge(dd_ctx *ctx, const void *U_dev);

/* out = op(in) for canonical spinor fields (device, caller-owned, 24 doubles
 * per site; in and out must not overlap).  The field is packed into the
 * internal layout at precision prec, the operator is applied at that precision
 * (FP16: per-site-scaled FP16 storage, 12-real links and FP16 C_inv, FP32
 * arithmetic), and the result is unpacked to complex double.  DD_OP_D and
 * DD_OP_DDAG are available at DD_F64, DD_OP_A at DD_F32 and DD_F16; other
 * combinations return DD_ERR_ARG.  Asynchronous. */
dd_status dirac_apply(dd_ctx *ctx, void *out_dev, const void *in_dev, dd_prec prec, dd_op op);

/* x = M_SAP b (Alg. 1 with loop count n_sap, Jacobi count n_jac from the
 * params) for canonical fields (device, caller-owned, must not overlap),
 * computed with internal storage at precision prec: DD_F32 (FP32 spinors,
 * links and C_inv, FP32 arithmetic) or DD_F16 (per-site-scaled FP16 spinors,
 * 12-real FP16 links, FP16 C_inv), whose block-local Jacobi sweeps run in
 * packed FP16 arithmetic when dd_params.sap_fp16_arith is 1 and in FP32
 * otherwise.  Asynchronous. */
dd_status sap_precondition(dd_ctx *ctx, void *x_dev, const void *b_dev, dd_prec prec);

/* ax = A M_SAP b (Alg. 3: the preconditioned operator of the BiCGStab of Alg. 5) for canonical
 * fields (device, caller-owned, must not overlap).  DD_F32: FP32 storage and arithmetic, the
 * product formed by the fused tail of Alg. 3 -- the last two half-sweeps of Alg. 1 also apply
 * A to the blocks they have just solved, and one more pass over the even blocks adds the
 * cross-block hops of the final odd result.  DD_F16: the FP16-storage SAP (as
 * sap_precondition), then the FP32 operator applied to its FP16-stored output (the inner
 * solver's operator must stay accurate to FP32, which an FP16 product would not be).
 * Asynchronous. */
dd_status sap_precondition_amsap(dd_ctx *ctx, void *ax_dev, const void *b_dev, dd_prec prec);

/* Solve D x = b (canonical fields on the device).  On entry x holds the
 * initial guess for every mode but DD_SOLVE_F32_SAP (pass zeros for a cold
 * start; a previous solution resumes the solve) and is ignored for
 * DD_SOLVE_F32_SAP; on exit it holds the solution.  maxiter bounds the
 * BiCGStab loop passes of a single-level solve, the defect-correction
 * passes of DD_SOLVE_MIXED and DD_SOLVE_MIXED_GCR, or the outer iterations of
 * DD_SOLVE_FGMRES.  In the two defect-correction modes a pass that
 * stagnates or whose inner solve breaks down switches the remaining passes to
 * the FP32 SAP-BiCGStab, and a second such pass to plain FP64 BiCGStab from
 * the current x, capped at inner_maxiter iterations; the first such pass of a
 * level that still cut the true residual 10x restarts that level once instead
 * (unless
 * dd_params.no_fallback; info->precision_level tells which level ended the
 * solve).  Returns DD_OK, DD_NOT_CONVERGED or DD_BREAKDOWN
 * (x then holds the best iterate) and fills info (may be NULL).  A source
 * with NaN or Inf returns DD_ERR_NONFINITE without touching x.
 * Synchronises the stream. */
dd_status bicgstab_solve(dd_ctx *ctx, void *x_dev, const void *b_dev, double tol, int maxiter,
                         dd_solve_mode mode, dd_solve_info *info);

/* Text of the last error on this context (never NULL). */
const char *dd_last_error(const dd_ctx *ctx);

/* Residual history of the last bicgstab_solve / bicgstab_solve_dagger on this
 * context (host values, kept until the next solve):
 *   which = 0: the true FP64 relative residual |b - D x| / |b| at the start and
 *              after every defect-correction pass (Alg. 4);
 *   which = 1: the recursive relative residual of the inner solver after every
 *              iteration, all passes in order (Alg. 5's r, or GCR's).
 * Copies at most cap values into out (host, may be NULL when cap is 0) and sets
 * *n to the length of the whole history.  DD_ERR_ARG for a bad argument. */
dd_status dd_solve_history(dd_ctx *ctx, int which, double *out, int cap, int *n);

/* ---- differentiation: L = |D^{-1} phi|^2 --------------------------------- */

/* Solve D^dagger x = b, through D^dagger = gamma_5 D gamma_5 (gamma_5 =
 * gamma_1 gamma_2 gamma_3 gamma_4 in the appendix's basis): y = gamma_5 x solves
 * D y = gamma_5 b with the solver of bicgstab_solve, and gamma_5 is applied
 * while the fields are packed and unpacked (no extra memory).  Arguments,
 * modes, initial guess, tolerance (now on |b - D^dagger x| / |b|), return
 * values and info are those of bicgstab_solve.  Synchronises the stream. */
dd_status bicgstab_solve_dagger(dd_ctx *ctx, void *x_dev, const void *b_dev, double tol, int maxiter,
                                dd_solve_mode mode, dd_solve_info *info);

/* *out = |x|^2 = sum_n sum_{colour, spin} |x|^2 of a canonical spinor field,
 * accumulated in FP64 in a fixed order (bitwise reproducible).  Synchronises. */
dd_status dd_spinor_norm2(dd_ctx *ctx, const void *x_dev, double *out);

/* Replace c_SW in the context's parameters.  The clover blocks depend on it,
 * so the context needs dd_load_gauge before its next operator call
 * (DD_ERR_STATE until then). */
dd_status dd_set_csw(dd_ctx *ctx, double csw);

/* Derivatives of the loss L = |psi|^2, psi = D^{-1} phi, given psi and
 * chi = D^{-dagger} psi (canonical spinors, device, caller-owned): the
 * variation of L is -2 Re <chi| dD psi>, with D = 1 + C - kappa H of the
 * appendix and the four-leaf clover built from the loaded gauge field.
 *   out_dev: canonical [4][Lt][Lz][Ly][Lx][3][3] complex double (caller-owned,
 *     must not overlap psi or chi).  su3 = 0: per link the gradient
 *     G = dL/dRe U + i dL/dIm U entry by entry (PyTorch's convention for a
 *     real function of complex inputs).  su3 = 1: per link the traceless
 *     Hermitian F with dL = tr(omega F) for U -> exp(i omega) U, omega
 *     Hermitian (the force projected to su(3)).
 *   dcsw: host pointer receiving dL/dc_SW = -2 Re <chi| (C / c_SW) psi>, or
 *     NULL to skip it (formed from the clover blocks already built when
 *     c_SW != 0, from the four-leaf field strength when c_SW = 0).
 * The hop term carries the boundary phases; the clover term differentiates
 * every leaf through the link (24 per link).  FP64 throughout.  The first
 * call allocates a work field of 864 bytes per site, kept until dd_destroy
 * (DD_ERR_NOMEM if that fails).  Uses the context's internal FP64 work
 * vectors.  Synchronises the stream. */
dd_status dd_force(dd_ctx *ctx, void *out_dev, double *dcsw, const void *psi_dev, const void *chi_dev, int su3);

/* dd_force for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results as dd_force, but the work field (54 complex doubles = 864
 * bytes per site) lives in a fixed 64 MiB device array that the library holds on
 * every GPU it runs on until the process ends, instead of a field the first call
 * allocates; the call makes no hipMalloc, hipFree or other allocating call.
 * Lattices of at most 77672 sites (64 MiB / 864 B; 16^4 fits) -- a larger one
 * returns DD_ERR_ARG, naming the limit, before any device work.  Every call on one
 * GPU shares that array (each call rewrites all of it that it reads): calls that
 * overlap on one GPU, from two streams or two host threads, race -- serialise them.
 * Its launches are not recorded by dd_timing_*.  Synchronises the stream. */
dd_status dd_force_noalloc(dd_ctx *ctx, void *out_dev, double *dcsw, const void *psi_dev, const void *chi_dev,
                           int su3);

/* ---- batched right-hand sides ------------------------------------------- */

/* Inner solver of bicgstab_solve_batch: BiCGStab on A M_SAP with the SAP of
 * each right-hand side (Alg. 1, 5; FP16 storage, as in DD_SOLVE_MIXED), or on
 * A alone. */
typedef enum { DD_BATCH_INNER_SAP = 0, DD_BATCH_INNER_PLAIN = 1 } dd_batch_inner;

/* out_r = op(in_r) for nrhs canonical spinor fields stored one after another
 * (device, caller-owned, [nrhs][Lt][Lz][Ly][Lx][3][4] complex double, in and
 * out must not overlap).  DD_F32 / DD_OP_A runs the batched kernel: tiles of
 * up to 12 right-hand sides share every link and C_inv load, and each hop's
 * 3x3 link times 3x(2 x 12) half-spinor product runs on the matrix cores
 * (sixteen sites per wavefront, one 4x4x1 block per site), or, in the
 * vector variants, each thread takes one site and 1-4 right-hand sides and
 * loads the links and C_inv once for them, or, in the resident-field variant
 * (4^4 blocks), a workgroup holds its block's links and C_inv for the whole
 * tile and takes the right-hand sides in turn.  The kernel variant
 * (matrix-core: right-hand sides per pass and workgroup size; vector:
 * right-hand sides per thread; resident) is picked by timing every variant on
 * the first call for each tile
 * size, unless dd_batch_set_variant forced one.  The SAP-preconditioned
 * batched solve reads FP16-storage fields and tunes the vector variants for
 * them separately (a forced matrix-core variant leaves that choice to its
 * own timing).  DD_F64 / DD_OP_D and DD_OP_DDAG apply the
 * single-field kernel to each right-hand side.  The first call allocates the
 * batch work fields (kept until dd_destroy; DD_ERR_NOMEM if that fails).
 * Asynchronous, except for the first call of a tile size, which synchronises
 * while it times the variants. */
dd_status dirac_apply_batch(dd_ctx *ctx, void *out_dev, const void *in_dev, int nrhs, dd_prec prec, dd_op op);

/* x_r = M_SAP b_r (Alg. 1, loop count n_sap, Jacobi count n_jac) for nrhs (1..16) canonical
 * spinor fields stored one after another ([nrhs][Lt][Lz][Ly][Lx][3][4] complex double, device,
 * caller-owned, x and b must not overlap), with the FP16 storage of sap_precondition at DD_F16.
 * With packed FP16 arithmetic (dd_params.sap_fp16_arith = 1) each half-sweep is one launch for
 * all right-hand sides, every workgroup staging its block's links and C_inv once and sweeping
 * the block for each right-hand side in turn; the result of each equals that of
 * sap_precondition on it alone.  With FP32 arithmetic it runs one SAP per right-hand side.
 * The first call allocates the batch work fields (kept until dd_destroy; DD_ERR_NOMEM if that
 * fails).  Asynchronous. */
dd_status sap_precondition_batch(dd_ctx *ctx, void *x_dev, const void *b_dev, int nrhs);

/* Force the batched kernel variant (0 .. 12: 0-7 matrix-core, 8-11 vector
 * with 1-4 right-hand sides per thread, 12 resident links and C_inv with the
 * right-hand sides in turn, for 4^4 blocks, else as 8), or -1 to let the
 * autotuner choose (the default). */
dd_status dd_batch_set_variant(dd_ctx *ctx, int variant);

/* The variant in use for tiles of nrhs (1..12) right-hand sides of FP32
 * inputs (dirac_apply_batch; -1 before its first call of that size) and the
 * autotuner's times in ms per launch for the first n_ms variants (0 where not
 * timed); ms may be NULL. */
dd_status dd_batch_tuning(dd_ctx *ctx, int nrhs, int *variant, double *ms, int n_ms);

/* Name of a batched kernel variant ("?" if out of range). */
const char *dd_batch_variant_name(int variant);

/* Solve D x_r = b_r for nrhs (1..16) right-hand sides at once (canonical
 * fields one after another, device, caller-owned; x holds the initial guesses
 * on entry, zeros for a cold start).  FP64 defect correction (Alg. 4) per
 * right-hand side around an FP32 BiCGStab that runs all right-hand sides in
 * lockstep, each with its own scalars and exit, and applies A to all of them
 * in one batched launch per step; the preconditioner (inner) is the SAP of
 * each right-hand side (FP16 storage) or none.  tol is on each true FP64 residual
 * |b_r - D x_r| / |b_r|; maxiter bounds the defect-correction passes;
 * inner_tol and inner_maxiter of the params apply to each inner solve.
 * info (may be NULL) receives nrhs records.  Returns the worst status over
 * the right-hand sides (DD_OK < DD_NOT_CONVERGED < DD_BREAKDOWN).  The first
 * call allocates the batch work fields (about 1.8 KB per site and right-hand
 * side), kept until dd_destroy.  Synchronises the stream. */
dd_status bicgstab_solve_batch(dd_ctx *ctx, void *x_dev, const void *b_dev, int nrhs, double tol, int maxiter,
                               dd_batch_inner inner, dd_solve_info *info);

/* ---- several lattices ---------------------------------------------------- */

/* A set of independent lattices (sizes, blocks, kappa, c_SW and phases of their
 * own, each with its own gauge field) whose FP32 operator A is applied to all of
 * them in one persistent launch: the work items are (lattice, 256-site chunk)
 * pairs taken from a global counter, so uneven lattices fill the chip together. */
typedef struct dd_multi dd_multi;

/* params: nlat (1..64) parameter sets, each checked as by dd_create (every
 * lattice gets a context of its own, with its fields and work vectors). */
dd_status dd_multi_create(const dd_params *params, int nlat, void *hip_stream, dd_multi **out);
dd_status dd_multi_destroy(dd_multi *m);
const char *dd_multi_last_error(const dd_multi *m);

/* The context of lattice lat (owned by m: do not destroy it; its timers hold the
 * multi-lattice launches for lattice 0), or NULL. */
dd_ctx *dd_multi_context(dd_multi *m, int lat);

/* Load lattice lat's gauge field, as dd_load_gauge. */
dd_status dd_multi_load_gauge(dd_multi *m, int lat, const void *U_dev);

/* out[k] = A_k in[k] for every lattice k (canonical fields of each lattice's
 * size, device, caller-owned, must not overlap), FP32, in one launch of the
 * multi-lattice kernel.  Synchronises the stream. */
dd_status dirac_apply_multi(dd_multi *m, void *const *out_dev, const void *const *in_dev);

/* Solve D_k x_k = b_k on every lattice to the true FP64 relative residual tol:
 * the mixed-precision solver of DD_SOLVE_MIXED (FP64 defect correction, FP32
 * BiCGStab on A M_SAP with the FP16 SAP) run for all lattices in lockstep,
 * each with its own scalars and exit, every A application of a step one
 * multi-lattice launch.  x holds the initial guesses (zeros for a cold start).
 * info (may be NULL) receives nlat records; returns the worst status.
 * Synchronises the stream. */
dd_status bicgstab_solve_multi(dd_multi *m, void *const *x_dev, const void *const *b_dev, double tol, int maxiter,
                               dd_solve_info *info);

/* ---- internal-layout entry points (benchmarks, no pack/unpack) ----------- */

/* Bytes of one internal spinor field at precision prec (FP16 includes the
 * per-site scales).  The caller allocates such buffers, 256-byte aligned. */
long long dd_field_bytes(const dd_ctx *ctx, dd_prec prec);

/* Pack a canonical spinor into the internal layout (dst) and back. */
dd_status dd_pack_spinor(dd_ctx *ctx, void *dst_internal, const void *src_canonical, dd_prec prec);
dd_status dd_unpack_spinor(dd_ctx *ctx, void *dst_canonical, const void *src_internal, dd_prec prec);

/* dirac_apply on internal-layout fields (same operator set as dirac_apply). */
dd_status dirac_apply_packed(dd_ctx *ctx, void *out_internal, const void *in_internal, dd_prec prec, dd_op op);

/* out = A in for an FP16-storage internal field in and an FP32 internal field
 * out, with FP32 links and C_inv: the operator application of the mixed
 * solver's inner BiCGStab on A M_SAP (Alg. 5), whose SAP output is stored in
 * FP16 (Alg. 1).  Buffers as from dd_field_bytes (DD_F16 for in, DD_F32 for
 * out), device, caller-owned, not overlapping.  DD_ERR_ARG for a null
 * pointer, DD_ERR_STATE without a gauge field.  Asynchronous on the context's
 * stream. */
dd_status dirac_apply_packed_f16in(dd_ctx *ctx, void *out_f32_internal, const void *in_f16_internal);

/* ---- kernel timing for roofline reporting -------------------------------- */

typedef enum {
    DD_KT_DIRAC_F64 = 0,    /* D or D^dagger, FP64 fields                       */
    DD_KT_DIRAC_F32 = 1,    /* A, FP32 spinors, links and C_inv                 */
    DD_KT_DIRAC_F16IN = 2,  /* A, FP16 input spinor, FP32 links/C_inv/output    */
    DD_KT_DIRAC_F16 = 3,    /* A, FP16 spinors, 12-real FP16 links, FP16 C_inv  */
    DD_KT_SAP = 4,          /* SAP half-sweep kernels (all precisions)           */
    DD_KT_BLAS = 5,         /* vector updates and reductions                     */
    DD_KT_FORCE = 6,        /* fermion force (dd_force), FP64                    */
    DD_KT_DIRAC_MRHS = 7,   /* A on a batch of right-hand sides, matrix cores    */
    DD_KT_DIRAC_MULTI = 8,  /* A on several lattices in one launch (timers of the
                               first lattice's context)                          */
    DD_KT_COUNT = 9
} dd_kernel_class;

/* When enabled, every launch of the timed classes is bracketed by HIP events
 * on the context's stream.  Enabling (or disabling) clears the counters. */
dd_status dd_timing_enable(dd_ctx *ctx, int on);

/* Launch count, summed launch time (ms), and the algorithmic bytes and flops
 * of those launches for one class since enabling; synchronises the stream.
 * Algorithmic bytes count every field a launch must read or write once per
 * site (a link or neighbour spinor used by two sites counts once); flops use
 * 168 per x/y/z hop, 156 per t hop and 600 per clover multiply.  Any output
 * pointer may be NULL. */
dd_status dd_timing_query(dd_ctx *ctx, dd_kernel_class cls, long long *launches, double *ms, double *bytes,
                          double *flops);

#ifdef __cplusplus
}
#endif

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility pop
#endif

#endif /* DDSOLVE_H */
