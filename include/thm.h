/*
 * thm.h -- C ABI of the MI355X (gfx950) time-harmonic Maxwell solver.
 *
 * Method (Beuchler, Kinnewig, Wick, arXiv 2105.11993):
 *   eq. (1)  curl(mu^{-1} curl E) - w^2 E = 0 in Omega,
 *            mu^{-1} g^t(curl E) - i k w g^T(E) = 0 on Gamma^inf,
 *            g^T(E) = g^T(E^inc) on Gamma^inc;
 *   eqs. (2)-(4) Nedelec discretisation -> real 2x2 block system
 *            [[K, -C], [C, K]] [E_re; E_im] = [f_re; f_im],  K = A - w^2 M, C = k w M_inf;
 *   eq. (11) GMRES preconditioned by diag(K, K)^{-1};
 *   eqs. (5)-(10) impedance-transmission domain decomposition (S = 1).
 *
 * Conventions shared by every entry point
 *   - Meshes are axis-aligned boxes [box_lo, box_hi] split into cells[0] x cells[1]
 *     (x cells[2]) equal cells; ids are lexicographic with x fastest.
 *   - Nedelec degree p >= 0 (0 = lowest order), first-kind tensor-product space.
 *   - DoF vectors are complex128, stored interleaved (re, im) in the global DoF
 *     order: edge DoFs (x-, y-[, z-]edges), [3D: face DoFs (x-, y-, z-faces)],
 *     then cell-interior DoFs.  thm_system_info gives the length.
 *   - Device pointers are HIP device memory on the current device; `stream` is a
 *     hipStream_t (NULL = default stream).  All work is enqueued on `stream`;
 *     solves synchronise it before returning so stats are valid.
 *   - The caller owns every buffer it passes; the library never frees them.
 *     The library owns everything inside a thm_system until thm_system_destroy.
 *   - Return value: 0 = OK; > 0 warning with valid output; < 0 error (no output
 *     guarantee).  The message of the last error on this thread is returned by
 *     thm_last_error().  No exception or abort crosses this interface.
 */
#ifndef THM_H
#define THM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    THM_OK = 0,
    THM_NOT_CONVERGED = 1,  /* best iterate written, stats filled */
    THM_EINVAL = -1,        /* null pointer, bad size, mu <= 0 or non-finite, w <= 0, no Gamma^inf */
    THM_EUNSUPPORTED = -2,  /* dim not in {2,3}, degree > 3 (2D) / > 1 (3D), uneven partition */
    THM_ENOMEM = -3,        /* device allocation failed */
    THM_EHIP = -4,          /* HIP runtime error (message carries hipGetErrorString) */
    THM_ESINGULAR = -5      /* zero or non-finite pivot while factorising the preconditioner */
} thm_status;

typedef enum { THM_FP64 = 0, THM_FP32_IR = 1 } thm_precision;
typedef enum { THM_DDM_GMRES = 0, THM_DDM_JACOBI = 1 } thm_ddm_outer;
typedef enum { THM_ORTH_CGS = 0, THM_ORTH_CGS2 = 1 } thm_orth;
/* Scalars of the Arnoldi process on the real block vectors: THM_KRYLOV_REAL is the
 * GMRES of the 2N real block system of eq. (4) taken literally (real Hessenberg);
 * THM_KRYLOV_COMPLEX uses complex scalars (inner products <v, w> = sum conj(v) w on
 * the interleaved (re, im) pairs), i.e. the Krylov space is closed under
 * multiplication by i.  Operator, preconditioner and solution are the same. */
typedef enum { THM_KRYLOV_COMPLEX = 0, THM_KRYLOV_REAL = 1 } thm_krylov;
/* Preconditioner of the subdomain / single-domain GMRES.  THM_PREC_BLOCK is the paper's
 * block-diagonal diag(K, K)^{-1} (eq. (11)).  THM_PREC_FULL is the complete inverse of the
 * block system, which Sec. 3.2 names as the alternative: here (K + iC)^{-1} (transpose:
 * (K - iC)^{-1}) applied exactly as z - K^{-1} P^T M^{-1} (i C_G P z), z = K^{-1} b, where P
 * restricts to the boundary DoFs Gamma that carry C, C_G is C on Gamma and
 * M = I + i C_G P K^{-1} P^T (r x r complex, r = |Gamma|; stored once per distinct system).
 * One application costs two applications of K^{-1} plus an r x r complex product.  Use it
 * with THM_FP64: in FP32 the correction cancels and refinement needs many inner steps.
 * Supported for r <= 4096 per subdomain (THM_EUNSUPPORTED above: the setup inverts the
 * dense 2r x 2r real form of M). */
typedef enum { THM_PREC_BLOCK = 0, THM_PREC_FULL = 1 } thm_precond;
/* How THM_FP32_IR refines (either preconditioner).  THM_IR_CLASSIC: FP64 residuals, each
 * correction by one cycle of FP32 GMRES (FP32 operator, basis and preconditioner); a step that
 * does not halve a system's FP64 residual is undone and that system continues by GMRES-based
 * refinement, as do its later solves with the same preconditioner in the same batch (until its
 * matrices change).
 * THM_IR_GMRES: GMRES-based refinement from the start (Carson and Higham's GMRES-IR: the
 * correction is solved by FP64 GMRES -- FP64 operator, basis and Hessenberg -- preconditioned by
 * the FP32 preconditioner, block or complete inverse, so its accuracy limits only the
 * convergence rate).  Either way a system GMRES-IR leaves above rtol is finished by FP64 GMRES
 * with the FP64 preconditioner. */
typedef enum { THM_IR_CLASSIC = 0, THM_IR_GMRES = 1 } thm_ir_mode;

/* Problem statement (paper Sec. 2, eq. (1); partition eq. (5)).  Copied by thm_assemble. */
typedef struct {
    int32_t dim;             /* 2 or 3 */
    int32_t cells[3];        /* cells per axis (cells[2] ignored in 2D) */
    double box_lo[3];
    double box_hi[3];
    int32_t degree;          /* Nedelec degree p */
    double omega;            /* w > 0 */
    double kappa;            /* k > 0, impedance coefficient of eq. (1) */
    const double *mu;        /* host, n_cells values > 0 (x fastest); NULL -> mu = 1 */
    uint32_t inc_faces;      /* bit 2*axis+side set -> that side is Gamma^inc; others Gamma^inf */
    double inc_dir[3];       /* E^inc(x) = pol * exp(-i w dir.x) */
    double inc_pol_re[3];
    double inc_pol_im[3];
    int32_t subdomains[3];   /* box partition for thm_ddm_solve; {1,1,1} = single domain */
    const double *eps;       /* host, n_cells relative permittivities > 0 (x fastest): a material of
                                refractive index n (Sec. 4.1's block benchmark) has eps = n^2 and enters
                                the mass term, K_c = mu_c^{-1} A_c - w^2 eps_c M_c; NULL -> 1 (eq. (3)) */
    double transmission[2];  /* DDM transmission operator S = s 1 on the interfaces, s = transmission[0]
                                + i transmission[1] (eqs. (7)-(8): subdomain i carries i k w s M_Sigma on
                                its interfaces, the update is G_{i->j} = -G_{j->i} - 2 i k w s M_Sigma E_i);
                                the paper's S = 1 (eq. (10)) is {1, 0}, and {0, 0} also means s = 1.  Any
                                s != 0 keeps the global discrete solution as the fixed point; Re(s) > 0 keeps
                                the subdomain problems absorbing.  Ignored without a partition. */
} thm_problem;

/* Solver options.  thm_default_opts fills the defaults listed here. */
typedef struct {
    int32_t restart;         /* GMRES restart length m (50) */
    int32_t max_iter;        /* total inner iterations per solve (5000) */
    double rtol;             /* stop at ||b - A x|| / ||b|| <= rtol on the real block system (1e-8) */
    int32_t precision;       /* thm_precision (THM_FP64) */
    int32_t orth;            /* thm_orth (THM_ORTH_CGS) */
    int32_t transpose;       /* 1: solve with A^T = [[K, C], [-C, K]] (adjoint) */
    int32_t ddm_outer;       /* thm_ddm_outer (THM_DDM_GMRES) */
    double inner_rtol;       /* subdomain solve tolerance inside the DDM (1e-10) */
    int32_t max_outer;       /* DDM outer iterations / Jacobi sweeps (500) */
    int32_t outer_restart;   /* restart of the DDM interface GMRES (200) */
    int32_t batched;         /* 1: all systems/subdomains in one batched launch sequence (1) */
    int32_t use_graph;       /* 1: replay Arnoldi steps from a captured hipGraph (1) */
    double ir_inner_rtol;    /* floor of the FP32 inner tolerance per refinement step (1e-6) */
    int32_t max_refine;      /* refinement steps for THM_FP32_IR (30) */
    int32_t krylov;          /* thm_krylov (THM_KRYLOV_COMPLEX) */
    int32_t relax_inner;     /* DDM interface GMRES only: 1 = before each Arnoldi step of the outer GMRES the
                                subdomain tolerance is max(inner_rtol, min(1e-2, s rtol / r)), with r the
                                outer GMRES's relative residual estimate after the previous step and s an
                                estimate of the smallest singular value of its Hessenberg matrix (the
                                inexact Krylov bound of Simoncini and Szyld: late outer steps tolerate less
                                accurate subdomain solves, the less so the worse the outer operator is
                                conditioned); residuals at restarts and the final field use inner_rtol,
                                and the returned field still meets rtol in the global FP64 residual;
                                0 = inner_rtol throughout (0) */
    int32_t precond;         /* thm_precond (THM_PREC_BLOCK) */
    int32_t ir_mode;         /* thm_ir_mode (THM_IR_CLASSIC) */
} thm_solve_opts;

typedef struct {
    int32_t status;
    int32_t iters;           /* inner GMRES iterations (max over systems; summed over DDM sweeps) */
    int32_t outer_iters;     /* DDM outer iterations */
    int32_t refinements;     /* FP64 refinement steps (THM_FP32_IR) */
    double rel_residual;     /* final FP64 relative residual of the (glued) solution */
    double setup_ms;         /* preconditioner factorisation time inside this call */
    double solve_ms;         /* solve time inside this call */
    int32_t fp64_fallback;   /* THM_FP32_IR: solves finished by FP64 GMRES with the FP64 factor because
                                GMRES-IR left them above rtol (DDM: summed over the subdomain solves);
                                0 otherwise */
    int64_t precond_extra_bytes; /* THM_PREC_FULL: device bytes of the stored M^{-1} (FP64 + FP32) of the
                                context that solved (all subdomains for the DDM); 0 otherwise */
    int32_t gmres_ir;        /* THM_FP32_IR: solves finished by GMRES-IR (FP64 GMRES, FP32 factor), either
                                after a classical step failed to contract or from the start (THM_IR_GMRES)
                                (DDM: summed over the subdomain solves); 0 otherwise */
} thm_stats;

typedef struct {
    int64_t n_dofs;          /* complex DoFs (vector length) */
    int64_t n_free;          /* DoFs not on Gamma^inc */
    int64_t nnz;             /* stored entries of K (structural pattern) */
    int64_t nnz_c;           /* stored entries of C */
    int64_t n_cells;
    int32_t n_subdomains;
    int32_t n_layers;        /* block-tridiagonal preconditioner layers */
    int64_t factor_bytes;    /* device bytes of the preconditioner factor (FP64 and FP32 copies) */
    int64_t n_interface;     /* complex interface unknowns of the DDM (sum over directed interfaces; -1 before
                                the first DDM solve) */
    int32_t spmv_variant;    /* autotuned FP64 SpMV variant of this system's context (10 x lanes per row +
                                unroll for CSR-vector, 19 for SELL-64, 20 for grouped SELL-64), -1 before
                                the first solve */
    int32_t ddm_spmv_variant; /* FP64 SpMV variant of the DDM's batched subdomain context, -1 before the
                                 first DDM solve */
    int32_t ddm_spmv_groups;  /* groups of subdomains with the same K in that context (each group shares
                                 one read of K in the grouped SELL-64 product), -1 before the first DDM
                                 solve */
} thm_info;

typedef struct thm_system thm_system;

/* Defaults for thm_solve_opts. */
void thm_default_opts(thm_solve_opts *o);

/*
 * Assembly (paper eq. (3), (4)).  Builds the DoF map, K = A - w^2 M (batched
 * element kernel + deterministic gather into CSR), C = k w M_inf, the Dirichlet
 * values (boundary L2 projection of g^T(E^inc) on Gamma^inc) and the lifted
 * right-hand side -S_FD g_D.  With subdomains != {1,1,1} it also builds every
 * subdomain system of eq. (7) and the interface maps of eq. (8).  The
 * preconditioner of eq. (11) is factorised lazily by the first solve.
 * Errors: THM_EINVAL, THM_EUNSUPPORTED, THM_ENOMEM, THM_EHIP.
 */
thm_status thm_assemble(const thm_problem *p, void *stream, thm_system **out);

/*
 * Block-preconditioned GMRES on the real 2x2 block form (Sec. 3.2, eq. (11)) for
 * nsys independent systems; nsys > 1 with opts->batched runs them as one batched
 * launch sequence.  E_dev[k]: device complex128 of length n_dofs(sys[k]); on
 * input the initial guess of the free entries (pass zeros), on output the
 * solution with the Dirichlet entries filled.  stats: host array of nsys.
 * opts->precision = THM_FP32_IR runs FP32 inner GMRES inside FP64 refinement.
 * Returns THM_NOT_CONVERGED (best iterate written) if any system misses rtol.
 */
thm_status thm_gmres_solve(int32_t nsys, thm_system *const *sys, const thm_solve_opts *opts,
                           void *const *E_dev, thm_stats *stats, void *stream);

/*
 * Impedance-transmission domain decomposition (eqs. (5)-(10), S = 1) over the
 * partition given at assembly, all subdomains resident on this GPU.  Outer
 * solver: GMRES on (I - A0) g = b (default) or Jacobi sweeps g <- A0 g + b
 * (with max_outer sweeps and rtol = 0 it returns the iterate after exactly
 * max_outer sweeps).  Subdomain solves use block-preconditioned GMRES to
 * opts->inner_rtol.  E_dev: device complex128, global length; output = glued
 * field (shared DoFs from the lowest subdomain id).
 */
thm_status thm_ddm_solve(thm_system *sys, const thm_solve_opts *opts, void *E_dev,
                         thm_stats *stats, void *stream);

/*
 * Adjoint gradient of J = int_T |E_h|^2, T = [tgt_lo, tgt_hi] (exact integration
 * over cell n T), with respect to the per-cell mu:
 *   dJ/dmu_c = 2 mu_c^{-2} Re(lambda_c^H Ahat_c E_c),  (K - iC)_FF lambda = (M_T E)_F,
 * lambda computed by one transposed block solve.  E_dev: forward solution
 * (device complex128, n_dofs).  dJdmu_dev: device double[n_cells].  J_host: J.
 */
thm_status thm_adjoint_grad(thm_system *sys, const void *E_dev, const double tgt_lo[3],
                            const double tgt_hi[3], const thm_solve_opts *opts,
                            double *dJdmu_dev, double *J_host, void *stream);

/* ---- lifecycle ---------------------------------------------------------- */
thm_status thm_system_info(const thm_system *sys, thm_info *info);
/* Replace mu (device double[n_cells]) and re-assemble K in place; the
 * preconditioner is re-factorised by the next solve. */
thm_status thm_system_set_mu(thm_system *sys, const double *mu_dev, void *stream);
void thm_system_destroy(thm_system *sys);
/* Free the solve workspaces the library keeps after a solve on sys (every batch context that
 * holds sys: Krylov basis, SpMV schedules, preconditioner work vectors; for a partitioned system
 * also its subdomain batch).  The system, its matrices and its factorisation stay; the next solve
 * rebuilds what it needs.  For callers that solve many systems one at a time with little device
 * memory to spare.  Errors: THM_EINVAL (NULL). */
thm_status thm_system_release_workspaces(thm_system *sys);
const char *thm_last_error(void);

/* ---- kernel-level entry points (for parity tests and measurement) -------- */
/* y = A x (transpose: A^T) on the full DoF vector with Dirichlet rows/columns as
 * identity; x, y: device complex128[n_dofs].  precision THM_FP32_IR uses the FP32
 * operator (x, y still complex128). */
thm_status thm_apply_operator(thm_system *sys, int32_t transpose, int32_t precision,
                              const void *x_dev, void *y_dev, void *stream);
/* y = diag(K, K)^{-1} x (eq. (11)), exact factorised inverse; factorises on first use.  After
 * static condensation of cell interiors, K's skeleton is block tridiagonal over layers of the
 * mesh; it is factorised by block LU when there are at most 64 layers and the widest has at
 * least 1024 skeleton DoFs (3D subdomains), else by block cyclic reduction.  The environment
 * variable THM_FACTOR_FORM = "bcr" or "lu", read when a factorisation is built, forces one
 * form (any other value: THM_EINVAL). */
thm_status thm_apply_precond(thm_system *sys, int32_t precision, const void *x_dev, void *y_dev,
                             void *stream);
/* y = (K + iC)^{-1} x (transpose = 0) or (K - iC)^{-1} x (transpose = 1): the complete
 * inverse of the block system (Sec. 3.2; see THM_PREC_FULL), in the real block form of
 * eq. (4), x and y complex128[n_dofs] on the device (interleaved re, im).  Builds the
 * factorisation and the boundary correction on first use.  precision THM_FP32_IR applies
 * it in FP32 (input and output still FP64).
 * Errors: THM_EINVAL (null arguments), THM_ESINGULAR (singular I + i C_G S_G), THM_EHIP. */
thm_status thm_apply_precond_full(thm_system *sys, int32_t transpose, int32_t precision, const void *x_dev,
                                  void *y_dev, void *stream);
/* Copy the assembled (not Dirichlet-modified) matrices to host memory.  Arrays
 * of sizes n_dofs+1 / nnz / nnz / n_dofs+1 / nnz_c / nnz_c; any may be NULL. */
thm_status thm_export_matrices(thm_system *sys, int32_t *k_rowptr, int32_t *k_col, double *k_val,
                               int32_t *c_rowptr, int32_t *c_col, double *c_val);
/* Dirichlet flags (uint8[n_dofs], 1 on Gamma^inc DoFs), the full Dirichlet
 * vector (complex128[n_dofs], g_D on D else 0) and the lifted right-hand side
 * (complex128[n_dofs], -S_FD g_D on F else 0), copied to host memory. */
thm_status thm_export_rhs(thm_system *sys, uint8_t *dir_flags, double *gD, double *rhs);
/* Element matrices K_c = Ahat_c / mu_c - w^2 Mhat_c of cells [c0, c0+count) (host, row-major). */
thm_status thm_export_elements(thm_system *sys, int64_t c0, int64_t count, double *out);
/* Average device time (ms) of `reps` launches of the block SpMV on this system,
 * measured with HIP events on `stream`; bytes_out: algorithmic bytes per launch. */
thm_status thm_time_spmv(thm_system *sys, int32_t precision, int32_t reps, double *ms_out,
                         double *bytes_out, void *stream);

/* Average device time (ms) of `reps` block SpMVs of eq. (4) over every subdomain of the
 * DDM's batched subdomain context (built by the first thm_ddm_solve on `sys`; THM_EINVAL
 * before), all systems active, with SpMV variant `variant` (a code below, or -1 for the
 * context's own choice), measured with HIP events on `stream`.  bytes_out: algorithmic
 * bytes per product, the same for every variant: each distinct K (values, columns, row
 * pointers) once, and per subdomain its C, its row pointers, x read once and y written
 * once. */
thm_status thm_time_spmv_batch(thm_system *sys, int32_t precision, int32_t variant, int32_t reps, double *ms_out,
                               double *bytes_out, void *stream);
/* Average device time (ms) of `reps` block SpMVs of eq. (4) applied to every system of the
 * batch sys[0 .. nsys) in one launch sequence (the batch context of a thm_gmres_solve on the
 * same systems in the same order if one exists, else a new one), all systems active, with the
 * context's autotuned variant, measured with HIP events on `stream`.  bytes_out: algorithmic
 * bytes per product (every system's K, C and row pointers once -- a K shared by a group of
 * identical systems once when the grouped variant runs -- x read once, y written once).
 * Errors: THM_EINVAL (nsys < 1, NULL pointers, reps < 1, unknown precision), THM_ENOMEM, THM_EHIP. */
thm_status thm_time_spmv_systems(int32_t nsys, thm_system *const *sys, int32_t precision, int32_t reps,
                                 double *ms_out, double *bytes_out, void *stream);

/* Block SpMV variants of eq. (4)'s operator: CSR-vector with L lanes per row and unroll U
 * (code 10 L + U, L in {2, 4, 8, 16, 32, 64}, U in {1, 4}; L = 64 only with U = 1) or
 * SELL-64 (code 19: one wave per slice of 64 rows, column-major padded entries). */
#define THM_SPMV_SELL 19
/* Grouped SELL-64 (code 20): systems of a batch whose K (pattern, values and Dirichlet
 * set) are identical -- the subdomains of a uniform decomposition, say -- form groups of
 * at most 16, and one wave applies a slice of the shared K to every member's vector, so
 * K is read once per group instead of once per system; each member's C is applied from
 * its own rows.  Results are bitwise those of code 19. */
#define THM_SPMV_SELL_GROUP 20
/* Grouped SELL-64 reading every member's vector from one member-interleaved copy (code 29):
 * chosen for a batch with shared K, the preconditioner of an Arnoldi step writes its output
 * straight into that copy (member j's value at row r next to the other members' values of row
 * r) and the product reads each row's values of all members as one contiguous run; outside
 * the Arnoldi step the batch uses code 20.  The same bits as code 20.  thm_time_spmv_batch
 * times the product alone on the copy's current contents. */
#define THM_SPMV_SELL_GROUP_IL 29

/* Pin the SpMV variant of the single-system context of `sys` (the one used by
 * thm_gmres_solve on {sys}, thm_apply_operator and thm_time_spmv) and, once a DDM solve
 * has built it, of the DDM's batched subdomain context, overriding the autotuner's
 * choice for that precision; variant = -1 re-runs the autotuner.  Captured GMRES step
 * graphs of those contexts are dropped, so the next solve uses the new variant.
 * Returns THM_EINVAL for an unknown variant or precision. */
thm_status thm_set_spmv_variant(thm_system *sys, int32_t precision, int32_t variant);

/* Average device time (ms) of `reps` applications of the factor phases (block cyclic
 * reduction or block LU) of the preconditioner (eq. (11)) -- the DDM's batched subdomain context if a
 * DDM solve has run on `sys`, else the system's own -- measured with HIP events on the
 * library's stream.  bytes_out: algorithmic bytes per application (every factor matrix
 * once plus member vectors); launches_out: kernel launches per application. */
thm_status thm_time_precond(thm_system *sys, int32_t precision, int32_t reps, double *ms_out, double *bytes_out,
                            int32_t *launches_out, void *stream);

/* ---- allocation-free entry point ------------------------------------------
 * For callers that cannot allocate device memory (work under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): y = diag(K, K)^{-1} x exactly as
 * thm_apply_precond computes it (same kernels, same results), with every work vector of the
 * apply (reduced skeleton right-hand side, skeleton solution, condensation terms, FP32
 * copies of x and y) in one static device array of the library, THM_NOALLOC_SCRATCH_BYTES
 * per device, held until the process ends.  The call allocates and frees nothing, copies
 * nothing between host and device and does not synchronise: it only enqueues kernels on
 * `stream` (a hipStream_t; NULL = the null stream) and returns.  x_dev, y_dev: device
 * complex128[n_dofs] (interleaved re, im), caller-owned; they must not overlap.
 * Preconditions: sys is a single-domain system and its factor and apply schedule already
 * exist, i.e. thm_apply_precond (either precision) or a thm_gmres_solve on {sys} alone has
 * run on it since its last thm_system_set_mu / thm_system_release_workspaces.
 * Every call on one device shares the array and leaves its contents there (work vectors are
 * cleared by the call where they must start at zero): calls that overlap in time on one
 * device -- on different streams or threads -- race and give undefined results.
 * Errors: THM_EINVAL (NULL arguments, unknown precision, factor or schedule not built yet,
 * or a system whose work vectors exceed THM_NOALLOC_SCRATCH_BYTES -- the message gives the
 * size needed), THM_EHIP (the array's address could not be obtained, or a launch failed). */
#define THM_NOALLOC_SCRATCH_BYTES (64u << 20)
thm_status thm_apply_precond_noalloc(thm_system *sys, int32_t precision, const void *x_dev, void *y_dev,
                                     void *stream);

#ifdef __cplusplus
}
#endif
#endif /* THM_H */
