/*
 * mpcare.h - C ABI of the MI355X (gfx950) mixed-precision Newton refinement
 * library for large sparse continuous-time algebraic Riccati equations
 *
 *      A^T X + X A - X B B^T X + C^T C = 0,     X ~ Z Z^T          (eq. (1.1))
 *
 * with A sparse (n x n, CSR), B dense n x m, C dense p x n, m, p << n
 * (problem statement, Sec. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * All array arguments are DEVICE pointers (memory of the device the
 *    context was created on) unless the comment says "host".  The caller owns
 *    every input and output buffer; the library never frees or keeps them.
 *    The library owns only its internal workspace (allocated lazily, cached in
 *    the context, released by care_ctx_destroy).
 *  * Dense matrices are column-major FP64 with a leading dimension >= n.
 *    C is passed as stored by the problem statement, p x n ROW-major, which is
 *    the same bytes as C^T column-major n x p with leading dimension n.
 *  * Each call starts after the work already queued on the stream given at
 *    context creation, runs on the context's own non-blocking stream (so
 *    that Krylov iterations can be replayed as HIP graphs), and returns after
 *    its device work has completed, because the method takes host-side
 *    decisions (convergence checks, eigenvalue splits).
 *  * Every function returns care_status: 0 = OK, > 0 = warning (outputs are
 *    valid), < 0 = error.  On an error the outputs are unspecified, except for
 *    CARE_ERR_CAPACITY, where *r_out (or *rp/*rm) holds the number of columns
 *    that would have been needed.  Argument checks happen before any device
 *    work.  care_last_error() returns a message for the calling thread.
 *  * No C++ exception crosses this interface.
 */
#ifndef MPCARE_H
#define MPCARE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t care_status;

enum {
  CARE_OK = 0,
  CARE_WARN_STAGNATED = 1,      /* refinement stopped on the stagnation test (Sec. 5) */
  CARE_WARN_MAXIT = 2,          /* k_max / j_max / Krylov iteration cap reached      */
  CARE_ERR_ARG = -1,            /* invalid argument (message via care_last_error)    */
  CARE_ERR_CAPACITY = -2,       /* output too small; required size reported         */
  CARE_ERR_UNSTABLE = -3,       /* iteration diverged (A or A_k not stable)         */
  CARE_ERR_BREAKDOWN = -4,      /* Krylov breakdown that could not be recovered      */
  CARE_ERR_NONFINITE = -5,      /* NaN/Inf met in inputs or iterates                 */
  CARE_ERR_DEVICE = -6,         /* HIP / rocBLAS / rocSOLVER runtime error           */
  CARE_ERR_NOMEM = -7,          /* device allocation failed                          */
  CARE_ERR_NOT_IMPLEMENTED = -8
};

/* Inner precision u_s of the initial solve and of the inner Lyapunov
 * solves (Sec. 2, precision levels; hierarchy u_s >= u >= u_r, u_c).
 * Residual evaluation, storage and update are always FP64 (u = u_r = u_c,
 * as in the experiments of Sec. 5). */
enum {
  CARE_FP64 = 0,                /* u_s = FP64 (the all-double baseline)             */
  CARE_FP32 = 1,                /* u_s = FP32                                       */
  CARE_BF16_SPMM = 2,           /* FP32 inner solves whose sparse products read the
                                   off-diagonal values of A in bfloat16            */
  CARE_AUTO = 3,                /* care_solve* only: a-priori choice after Theorem 1's
                                   condition d_1 kappa_F(L) u_s < 1, with kappa_F(L)
                                   estimated as sqrt(||A||_1 ||A||_inf) / min |Re p|
                                   over the shift set: CARE_FP32 when kappa u_32 is
                                   at most 6e-6 (kappa <= 100) for a sparse A or
                                   6e-3 (kappa <= 1e5) for a dense A, else CARE_FP64
                                   (thresholds measured, see care_solve); the choice
                                   is reported in care_stats.inner_prec            */
  CARE_FP16_SPMM = 4            /* FP32 inner solves whose sparse products read the
                                   off-diagonal values of A in IEEE half precision,
                                   stored as a_ij / 2^e with 2^e fixed per operator
                                   so that max |a_ij| / 2^e lies in [2^13, 2^14]
                                   (within half's range; the kernel multiplies by
                                   2^e exactly).  Sparse A only                     */
};

/* CSR of A itself (NOT of A^T); 0-based int32 indices, column indices sorted
 * within each row, no duplicates.  row_ptr has n+1 entries.  Device memory. */
typedef struct {
  int64_t n, nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
} care_csr;

/* ADI shift p = re + i im.  Re p < 0.  Complex shifts are given as adjacent
 * conjugate pairs (p, conj p) with Im p > 0 first.  Shift arrays are HOST
 * memory; shifts are cycled when more ADI steps than shifts are needed. */
typedef struct {
  double re, im;
} care_shift;

typedef struct care_ctx care_ctx;

/* Solver options; care_opts_default fills the values used in Sec. 5. */
typedef struct {
  int32_t inner_prec;     /* CARE_FP64 | CARE_FP32 | CARE_BF16_SPMM | CARE_FP16_SPMM |
                             CARE_AUTO                                              */
  int32_t k_max;          /* refinement steps of Framework 1 (20)                     */
  int32_t k0_max;         /* Newton steps of the initial NLR-ADI solve (20)           */
  int32_t j_max;          /* ADI steps per Lyapunov solve (50)                        */
  double eta_r_rel;       /* Alg. 1 threshold, relative to max|lambda(H)| (1e-4)      */
  double eta_s_rel;       /* Alg. 2 threshold, relative to max|lambda(P)| (10 u_fp64)  */
  double tau_L;           /* inner LR-ADI stop ||W^T W||_F <= tau_L ||W0^T W0||_F;
                             <= 0 selects 1e-12 (FP64) / 1e-6 (FP32) / 1e-4 (FP16
                             products) / 1e-3 (BF16 products)                      */
  double tau_0;           /* initial NLR-ADI stop on the relative Riccati residual;
                             <= 0 selects max(tol / 10, 10 tau_L0)                    */
  double stagnation;      /* stop when ||R_{k+1}|| / ||R_k|| > stagnation (0.999)     */
  int32_t krylov_maxit;   /* BiCGStab iteration cap per shifted solve (4000)          */
  double krylov_tol;      /* per-column relative residual; <= 0 selects
                             max(1e-13, min(1e-10, tol / 10)) (FP64), 1e-7 (FP32),
                             1e-4 (FP16 products) or 1e-3 (BF16 products).  Columns
                             that stagnate above it
                             are restarted on their true residual                   */
  int32_t check_every;    /* host convergence poll period of the Krylov loop (8)      */
  int32_t penzl_l0;       /* auto shifts: number of shifts (16)                       */
  int32_t penzl_kp;       /* auto shifts: Arnoldi steps on A^T (20)                   */
  int32_t penzl_km;       /* auto shifts: Arnoldi steps on A^-T (10)                  */
  int32_t profile;        /* 1: time every sparse-product launch with HIP events that
                             the launch records at the kernel's start and end
                             (care_stats.t_spmm); graph replay is then off         */
  const double* Z_init;   /* optional FP64 start factor Z_1 (device, n x r_init);
                             skips the initial NLR-ADI solve (resume)               */
  int64_t ldz_init;
  int32_t r_init;
  int32_t adi_deflate;    /* 1: LR-ADI stops iterating columns of W whose residual
                             is negligible for the stopping test (default 1)       */
  int32_t krylov_block_tol; /* 1: Krylov accuracy relative to the largest column of
                             the right-hand side block instead of each column (0);
                             -1 (default): 1 for FP32 inner solves (their LR-ADI
                             residual factor is rotated, so most columns are
                             small), 0 for FP64 and the 16-bit products            */
  int32_t penzl_real;     /* auto shifts: 1 keeps the real parts of the Ritz values */
  int32_t spmm_split;     /* BiCGStab products: 0 chooses by the L2 footprint of the
                             fused gathers, 1 fused, 2 split (update pass + product) */
  int32_t krylov_relax;   /* 1 (default): inexact LR-ADI, the inner tolerance of step j
                             grows as ktol / (4 ||W_j^T W_j|| / ||W_0^T W_0||), capped
                             at sqrt(ktol); 0: ktol for every solve                  */
  double refine_forcing;  /* theta of the inexact-Newton forcing of the refinement
                             corrections (0.25).  With rel_k = ||R(Z_k)||_F / ||C^T C||_F
                             the correction LR-ADI stops at
                             tau_k = min(0.1, max(tau_L, theta tol / rel_k)), its
                             Krylov tolerance is max(krylov_tol, tau_k / 10), and
                             Algorithm 1 also drops the smallest residual eigenvalues
                             whose joint Frobenius norm stays below
                             theta tol ||C^T C||_F.  0: tau_L, krylov_tol and eta_r
                             alone, as in Sec. 5                                    */
  double tau_L0;          /* LR-ADI tolerance inside the initial NLR-ADI solve; <= 0
                             selects tau_L                                          */
  int32_t spmm_tune;      /* 1 (default): the first sparse product of each shape
                             (operator, precision, mode, column count rounded up to
                             16) times 16- and 8-column panels, each with the
                             default panel grouping or one panel per workgroup, and
                             keeps the fastest for the context's operator; 0:
                             16-column panels, default grouping                    */
  int32_t shift_update;   /* heuristic shifts only (nshifts = 0): 1 recomputes them
                             for every Lyapunov solve from its closed-loop operator
                             A - B K^T (Newton steps >= 1, corrections), the
                             inverse Arnoldi through SMW; 2 projection shifts
                             (care_projection_shifts): every LR-ADI run takes its
                             first set from span(W0) and, whenever a set is used
                             up, the next from the span of its latest blocks of Z,
                             at most penzl_l0 per set; 0 (default): one Penzl set
                             from A for the whole solve                            */
  int32_t krylov_method;  /* shifted solves: 0 (default) column-batched BiCGStab;
                             1 restarted GMRES for real shifts (complex pairs stay
                             on BiCGStab); krylov_maxit then counts Arnoldi steps  */
  int32_t krylov_restart; /* GMRES restart length; <= 0 selects 30 (FP32) / 50 (FP64),
                             the values of Sec. 5; at most 1000                     */
  int32_t krylov_compact; /* BiCGStab: 1 (default) gathers the columns still
                             iterating into fewer 16-column panels whenever they
                             fit in fewer (same arithmetic per column, same
                             results); 0: every column stays in place              */
  int32_t adi_rotate;     /* with adi_deflate: 1 (default) turns the active columns
                             of the LR-ADI residual factor W (within the C+ and C-
                             groups of a correction) to their principal directions
                             each time the ADI residual has halved, so that the
                             column freezing can take the directions the residual
                             has left; 0: W is never rotated                       */
  int32_t krylov_rb;      /* 1 (default): when the pattern of A is two-colourable and its
                             diagonal one constant d (five- and seven-point stencils),
                             each shifted solve eliminates one colour exactly and the
                             Krylov method runs on the other: (G + p' I) x_b =
                             F b_r - (d + p) b_b, G = F E, p' = -(d + p)^2, then
                             x_r = (b_r - E x_b) / (d + p) (the red-black block
                             factorisation behind a multicolour ILU of the stencil,
                             with the black block's fill kept); 0: never        */
  int32_t krylov_precond; /* 1: the restarted GMRES solves (krylov_method = 1) are right-
                             preconditioned by ILU(0) of A^T + p I in a multicolour
                             order (care_ilu0_factor), the inner solver of Sec. 5
                             ("Performance Analysis on GPU"); with krylov_rb = 1 and
                             a two-colourable A, GMRES runs on the reduced system
                             G + p' I, preconditioned by ILU(0) of that matrix;
                             krylov_rb = 0 gives the paper's setting.  0 (default):
                             no preconditioner                                     */
} care_opts;

/* Statistics written by the solvers (host struct). */
typedef struct {
  int32_t iter0_outer, iter0_inner;   /* initial solve "outer(inner)" (Sec. 5 tables)  */
  int32_t iter_outer, iter_inner;     /* refinement "outer(inner)"                     */
  int32_t rank;                       /* columns of the returned factor               */
  int32_t stagnated;
  double res_rel;                     /* ||R(Z)||_F / ||C^T C||_F of the result (FP64)  */
  double res_paper;                   /* the paper's normalised residual "Res" (Sec. 5) */
  double eta_n;                       /* ||P-||_F / ||P||_F of the last Alg. 2 (Lemma 1) */
  double t_total, t_stage0, t_refine, t_setup;   /* seconds, host wall clock          */
  int64_t spmm_calls;                 /* sparse product launches                       */
  double spmm_bytes;                  /* algorithmic bytes of those launches           */
  double t_spmm;                      /* summed kernel time (profile = 1), seconds      */
  int64_t krylov_iters;               /* BiCGStab iterations summed over columns' solves */
  int32_t hist_len;                   /* entries of res_hist used                      */
  double res_hist[48];                /* relative residual after each outer step      */
  int32_t inner_prec;                 /* inner precision used (CARE_AUTO resolved)     */
  int32_t krylov_compactions;         /* BiCGStab column compactions (krylov_compact)  */
  int32_t adi_rotations;              /* rotations of an LR-ADI residual factor group  */
} care_stats;

/* ---------------------------------------------------------------------- */
/* Context                                                                  */
/* ---------------------------------------------------------------------- */

/* Device-memory hooks of a context (the caller's allocator, e.g. a caching
 * allocator of the framework that owns the device).  alloc returns `bytes`
 * bytes of device memory of the context's device, usable in work queued on
 * `stream` (the context's own stream, a hipStream_t passed as void*), or
 * NULL when it cannot; dealloc returns a block obtained from alloc (same
 * bytes and stream).  `user` is passed through unchanged.  The hooks are
 * only called from the thread that calls an entry point with the context
 * (never from threads the library creates: the worker contexts of
 * care_solve_batch allocate their workspace with hipMalloc). */
typedef void* (*care_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*care_dealloc_fn)(void* ptr, size_t bytes, void* stream, void* user);

/* Create a context on `device` that orders all work on `stream` (a
 * hipStream_t passed as void*; NULL = the default stream).  *ctx receives a
 * handle owned by the caller, released with care_ctx_destroy.
 * Workspace (the boundary passage of the problem statement: the caller owns
 * inputs and outputs, the library only its workspace): with alloc = dealloc =
 * NULL the library allocates its device workspace with hipMalloc; with both
 * set, every device workspace block the library uses is drawn through alloc
 * and handed back through dealloc (blocks are cached by the context between
 * calls and all returned by care_ctx_destroy, or earlier when a solve trims
 * its cache).  The vendor BLAS/LAPACK handle of the context keeps its own
 * internal scratch.  Exactly one of alloc, dealloc NULL is CARE_ERR_ARG. */
care_status care_ctx_create(care_ctx** ctx, int32_t device, void* stream, care_alloc_fn alloc,
                            care_dealloc_fn dealloc, void* user);
void care_ctx_destroy(care_ctx* ctx);

/* Default options for inner precision `inner_prec`.  Taken from Sec. 5:
 * eta_r = 1e-4 max|lambda(H)|, eta_s = 10 u max|lambda(P)|, tau_L = 1e-12
 * for FP64, k_max = 20, j_max = 50, stagnation ratio 0.999, GMRES restart
 * 30 (FP32) / 50 (FP64) when krylov_method = 1.  Departures from Sec. 5:
 *   - tau_L = 1e-6 for FP32 (paper 1e-5), 1e-4 / 1e-3 for FP16 / BF16
 *     products (not in the paper);
 *   - inner solver: column-batched BiCGStab on the red-black reduced
 *     operator where A is two-colourable with a constant diagonal
 *     (krylov_rb = 1), unpreconditioned BiCGStab otherwise (paper:
 *     ILU(0)-preconditioned restarted GMRES, available as krylov_method = 1,
 *     krylov_precond = 1, krylov_rb = 0); Krylov tolerance 1e-7 for
 *     FP32 (paper 1e-5), max(1e-13, min(1e-10, tol / 10)) for FP64 (paper
 *     1e-10); iteration cap 4000 (paper 100 / 200 GMRES steps);
 *   - refinement forcing theta = 0.25 (refine_forcing; paper: fixed
 *     tolerances) with residual-budget truncation in Algorithms 1 and 2;
 *   - inexact LR-ADI (krylov_relax = 1), column deflation (adi_deflate = 1),
 *     rotation of the FP32 residual factor (adi_rotate = 1), block-relative
 *     Krylov accuracy for FP32 (krylov_block_tol = -1), column compaction
 *     (krylov_compact = 1), panel-width autotuning (spmm_tune = 1): none is
 *     in the paper, each leaves the solution within the tolerance;
 *   - heuristic shifts (nshifts = 0): Penzl's procedure with l0 = 16,
 *     kp = 20, km = 10 computed once from A (shift_update = 0); the paper
 *     says only that its shifts come from Krylov subspaces. */
void care_opts_default(care_opts* opts, int32_t inner_prec);

/* Message describing the last error of the calling thread ("" if none). */
const char* care_last_error(void);

/* Library version string (static storage). */
const char* care_version(void);

/* sizeof of the ABI structs as this library was compiled, for bindings to
 * check their own layouts: sizes[0..count) receives care_csr, care_shift,
 * care_opts, care_stats, care_instance, care_instance_result (count <= 6).
 * sizes is HOST memory.  Needs no device. */
care_status care_struct_sizes(int64_t* sizes, int32_t count);

/* ---------------------------------------------------------------------- */
/* Building blocks of the LR-ADI inner loop (Sec. 4)                        */
/* ---------------------------------------------------------------------- */

/* Shifted sparse product Y = (A^T + p I) X in precision `prec` (the
 * operator M_alpha of the SMW formula, Sec. 4).  X: n x k column-major FP64
 * (ldx >= n); Y: n x k (ldy >= n).  For a complex shift, X and Y hold k
 * complex columns as [Re(X) | Im(X)] (2k real columns).  X is rounded to
 * the working precision first and Y is returned in FP64.  k = 0 is a no-op. */
care_status care_spmm(care_ctx* ctx, const care_csr* A, int32_t prec, care_shift p,
                      const double* X, int64_t ldx, int32_t k, double* Y, int64_t ldy);

/* Timing of the shifted sparse product alone (the SpMM of the inner solves,
 * Sec. 4): builds `nsets` copies of the SELL operator of A^T in precision
 * `prec`, fills nsets input panels of k columns (complex shift: k complex
 * columns), runs one warm-up round and then `reps` rounds of
 * Y_s = (A^T + p I) X_s over the sets in turn (rotating the sets keeps the
 * operands out of the caches once their total exceeds them), and returns the
 * mean time per product in microseconds (HIP events on the context's stream)
 * and the algorithmic bytes of one product, nnz (s_v + 4) + 4 (n + 1) +
 * 2 n k s_x, in *bytes_per_product (both HOST).  panel = 8 or 16 fixes the
 * column panel of products wider than 8 columns, 0 uses the default;
 * panels_per_block > 0 fixes how many column panels one workgroup runs (the
 * operator's entries are loaded once for all of them), 0 uses the default.
 * The library allocates the operator copies and panels itself. */
care_status care_spmm_timing(care_ctx* ctx, const care_csr* A, int32_t prec, care_shift p, int32_t k,
                             int32_t nsets, int32_t reps, int32_t panel, int32_t panels_per_block,
                             double* us_per_product, double* bytes_per_product);

/* Shifted block solve (A_k^T + p I) V = W with A_k = A - B K^T, by the
 * Sherman-Morrison-Woodbury formula of Sec. 4: solve (A^T + p I)[Vh, S] = [W, K]
 * with column-batched BiCGStab in precision `prec`, then
 * V = Vh + S (I_m - B^T S)^{-1} B^T Vh.  B, K: n x m column-major (ldb, ldk
 * >= n; K = NULL or m = 0 means A_k = A).  W, V: n x w (complex shifts: [Re|Im]
 * layout as in care_spmm for V; W is real).  tol <= 0 / maxit <= 0 select the
 * precision's defaults.  *iters (host, may be NULL) receives the largest
 * per-column iteration count.  Returns CARE_WARN_MAXIT if a column did not
 * reach tol. */
care_status care_shifted_solve(care_ctx* ctx, const care_csr* A, const double* B, int64_t ldb,
                               const double* K, int64_t ldk, int32_t m, care_shift p,
                               const double* W, int64_t ldw, int32_t w, int32_t prec,
                               double tol, int32_t maxit, double* V, int64_t ldv, int32_t* iters);

/* care_shifted_solve with the Krylov method of `opts` (NULL: as
 * care_shifted_solve): krylov_method, krylov_restart, krylov_compact,
 * krylov_rb and krylov_precond are read, nothing else.  With krylov_method = 1,
 * krylov_precond = 1 and krylov_rb = 0 the solve is the paper's restarted
 * GMRES right-preconditioned by ILU(0) (Sec. 5, "Performance Analysis on
 * GPU"); maxit then counts Arnoldi steps.  A zero ILU(0) pivot returns
 * CARE_ERR_BREAKDOWN. */
care_status care_shifted_solve_opts(care_ctx* ctx, const care_csr* A, const double* B, int64_t ldb,
                                    const double* K, int64_t ldk, int32_t m, care_shift p, const double* W,
                                    int64_t ldw, int32_t w, int32_t prec, double tol, int32_t maxit,
                                    const care_opts* opts, double* V, int64_t ldv, int32_t* iters);

/* ILU(0) of M = A^T + p I (real p) in precision prec, the preconditioner of
 * the restarted-GMRES inner solves of Sec. 5 ("Performance Analysis on
 * GPU"), in the multicolour order the library uses: rows are coloured
 * first-fit in their natural order over the off-diagonal pattern of A (an
 * edge for a_ij or a_ji nonzero), ordered colour by colour and by index
 * inside a colour; L (unit lower) and U in that order keep the pattern of M
 * and satisfy (L U)_ij = m_ij on it.  Inspection entry point, all outputs
 * HOST: colours[n] the colour of each row; off[noff] the factor value at
 * each off-diagonal nonzero (i, j) of A^T in row-major order (l_ij when j's
 * colour is below i's, u_ij otherwise), noff = the number of off-diagonal
 * nonzeros of A (CARE_ERR_CAPACITY otherwise); udiag[n] the pivots u_ii.
 * CARE_ERR_BREAKDOWN on a zero pivot, CARE_ERR_NOT_IMPLEMENTED when the
 * pattern needs more than 1024 colours. */
care_status care_ilu0_factor(care_ctx* ctx, const care_csr* A, int32_t prec, double p, int32_t* colours,
                             double* off, int64_t noff, double* udiag);

/* The colouring that orders care_ilu0_factor's unknowns, on its own: first-
 * fit in natural row order over the undirected graph of the off-diagonal
 * entries of A (a_ij or a_ji nonzero).  row_ptr, col_idx: HOST CSR pattern of
 * A (n + 1 and nnz int32, checked here); colours: HOST, n entries; ncolours:
 * HOST.  Needs no device.  CARE_ERR_NOT_IMPLEMENTED past 1024 colours. */
care_status care_ilu0_colouring(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                                int32_t* colours, int32_t* ncolours);

/* Z = (L U)^{-1} X with the factors of care_ilu0_factor (the preconditioner
 * solve: one forward and one backward sweep, each one parallel step per
 * colour).  X, Z: device FP64, n x k column-major (ldx, ldz >= n), X rounded
 * to prec, Z converted back; they may not overlap. */
care_status care_ilu0_apply(care_ctx* ctx, const care_csr* A, int32_t prec, double p, const double* X,
                            int64_t ldx, int32_t k, double* Z, int64_t ldz);

/* Batched LU factorisation with partial pivoting of M_s = M0 + p_s I,
 * s < nshifts: the direct shifted solves of the dense problems (Sec. 5.1
 * solves its dense examples with LU; under the Sherman-Morrison-Woodbury form
 * of Sec. 4 the factors of A^T + p I serve every Newton step).  One launch,
 * one workgroup per matrix, matrix-core updates.  prec: CARE_FP32 or
 * CARE_FP64, the element type of M0 and F.  M0: device, n x n column-major,
 * leading dimension n.  shifts: HOST, real, rounded to prec before they are
 * added to the diagonal.  F: device, nshifts consecutive n x n matrices
 * (leading dimension n, not overlapping M0) receiving the LAPACK getrf layout
 * (unit lower L strictly below the diagonal, U on and above it).  perm:
 * device, nshifts x n int32 with (P M_s)[i] = M_s[perm[s n + i]] (the row
 * exchanges composed).  info: HOST, nshifts entries: 0, or the 1-based index
 * of the first zero pivot (the factorisation still completes, as getrf's).
 * 1 <= n <= 2048.  Errors: CARE_ERR_ARG. */
care_status care_shifted_lu_factor(care_ctx* ctx, int32_t prec, int64_t n, const void* M0, const double* shifts,
                                   int32_t nshifts, void* F, int32_t* perm, int32_t* info);

/* X = M_s^{-1} B with one matrix's factors from care_shifted_lu_factor
 * (F: n x n, perm: n entries, both device): the permuted right-hand sides,
 * then the unit lower and the upper triangular solves, in prec (CARE_FP32 or
 * CARE_FP64, the element type of F, B and X).  B, X: device, n x k column-
 * major (ldb, ldx >= n); X may be B (same leading dimension).  One workgroup
 * per 2 (FP32) or 1 (FP64) columns.  1 <= n <= 2048, k >= 0.  Errors:
 * CARE_ERR_ARG. */
care_status care_shifted_lu_solve(care_ctx* ctx, int32_t prec, int64_t n, const void* F, const int32_t* perm,
                                  int32_t k, const void* B, int64_t ldb, void* X, int64_t ldx);

/* Gram product C = X^T Y of tall-skinny FP64 panels (FP64 matrix cores), the
 * Gram step of the thin QR of F in Algorithm 1 and of G in Algorithm 2.  For
 * a * b >= 1024: the library's own 128 x 128-tile MFMA kernel for X^T X (the
 * tiles on and above the diagonal) up to 512 columns or 1.5 GB of X, rocBLAS
 * dgemm over row chunks otherwise (environment variable MPCARE_GRAM, read at
 * context creation: 0 always rocBLAS, 1 always the own kernel); smaller
 * products use the library's 32 x 32-tile MFMA kernel.  X: n x a (ldx >= n), Y: n x b (ldy >= n), C: a x b (ldc >= a).
 * Partial products over row chunks are summed in a fixed order (run-to-run
 * reproducible); X == Y (same pointer and ld) gives an exactly symmetric C. */
care_status care_gram(care_ctx* ctx, int64_t n, const double* X, int64_t ldx, int32_t a, const double* Y,
                      int64_t ldy, int32_t b, double* C, int64_t ldc);

/* care_gram for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same product C = X^T Y with the library's own FP64 MFMA kernel only (no
 * rocBLAS), its row-split partial sums kept in a fixed 32 MiB device array
 * of the library (one per GPU, held until the process ends) instead of
 * allocated workspace; no allocation of any kind.  Arguments as care_gram;
 * limit: ceil(a/32) * ceil(b/32) <= 4096 (e.g. a = b = 2048), larger sizes
 * return CARE_ERR_ARG; n = 0 returns CARE_ERR_ARG.  C is not exactly
 * symmetric for X == Y (every tile is computed).  All calls on one GPU share
 * the array: calls that overlap on one GPU (other threads, other contexts)
 * race on it and must be serialised by the caller.  Returns after the
 * product has completed. */
care_status care_gram_noalloc(care_ctx* ctx, int64_t n, const double* X, int64_t ldx, int32_t a, const double* Y,
                              int64_t ldy, int32_t b, double* C, int64_t ldc);

/* Tall-skinny product Y = alpha X S + beta Y (FP64 matrix cores: rocBLAS
 * dgemm for q * k >= 4096, the library's own MFMA kernel below): X n x q
 * (ldx >= n), S q x k (lds >= q), Y n x k (ldy >= n); beta = 0 does not read
 * Y.  Forms U = F T^{-1}, C+- = U Q+- |Lambda+-|^(1/2) and Z = V Theta+
 * Sigma+^(1/2) in Algorithms 1 and 2. */
care_status care_tsgemm(care_ctx* ctx, int64_t n, const double* X, int64_t ldx, int32_t q, const double* S,
                        int64_t lds, int32_t k, double alpha, double beta, double* Y, int64_t ldy);

/* ---------------------------------------------------------------------- */
/* The four solver entry points                                             */
/* ---------------------------------------------------------------------- */

/* LR-ADI for the Lyapunov equation  A_k^T X + X A_k + W W^T = 0,
 * A_k = A - B K^T (B, K: n x m; B = K = NULL or m = 0 means A_k = A), the
 * inner solver of Sec. 4 (residual-based LR-ADI; real shifts and
 * complex-conjugate pairs).  nshifts = 0 with opts->shift_update = 2 runs
 * on projection shifts (see care_opts).  W: n x w.  Runs in opts->inner_prec until
 * ||W_j^T W_j||_F <= tol ||W^T W||_F (tol <= 0 selects opts' tau_L) or
 * opts->j_max steps.  Output Z: n x (*r_out) FP64, ldz >= n, capacity rmax
 * columns; block j of w columns keeps the column order of W (a complex pair
 * gives two blocks).  stats may be NULL. */
care_status lyap_lradi(care_ctx* ctx, const care_csr* A, const double* B, const double* K, int32_t m,
                       const double* W, int64_t ldw, int32_t w, const care_shift* shifts,
                       int32_t nshifts, double tol, const care_opts* opts, double* Z, int64_t ldz,
                       int32_t rmax, int32_t* r_out, care_stats* stats);

/* Algorithm 1 (Residual Factor Decomposition) in FP64:
 * R(Z Z^T) = C+ C+^T - C- C-^T with thresholds +-eta_r, eta_r = eta_r_rel
 * max|lambda(H)| (eta_r_rel = 0: no truncation).  Z: n x r (ldz >= n).
 * Cp: n x (*rp), Cm: n x (*rm), leading dimension ldc >= n, each with
 * capacity `cap` columns.  *res_fro (host) = ||R(Z Z^T)||_F = ||H||_F,
 * taken from the eigenvalues of H before truncation. */
care_status care_residual_factor(care_ctx* ctx, const care_csr* A, const double* B, int32_t m,
                                 const double* C, int32_t p, const double* Z, int64_t ldz, int32_t r,
                                 double eta_r_rel, double* Cp, int32_t* rp, double* Cm, int32_t* rm,
                                 int64_t ldc, int32_t cap, double* res_fro);

/* Algorithm 2 (Solution Factor Decomposition) for a general signature:
 * given G (n x s, ldg >= n) and host sign[s] in {+1, -1} (N = diag(sign)),
 * returns Z (n x *r_out, ldz >= n, capacity cap) with Z Z^T the positive
 * spectral part of G N G^T above eta_s = eta_s_rel max|lambda(P)|.
 * sign = all +1 gives plain column compression.  *eta_n (host, may be
 * NULL) receives ||P-||_F / ||P||_F. */
care_status lowrank_truncate(care_ctx* ctx, int64_t n, const double* G, int64_t ldg, int32_t s, const int8_t* sign,
                             double eta_s_rel, double* Z, int64_t ldz, int32_t cap, int32_t* r_out,
                             double* eta_n);

/* Framework 1 (Factorization-based Mixed Precision Newton Iterative
 * Refinement): initial NLR-ADI solve in opts->inner_prec (Sec. 4), then
 * FP64 Algorithm 1, inner LR-ADI corrections on [C+, C-] in inner_prec and
 * FP64 Algorithm 2, until ||R||_F <= tol ||C^T C||_F.  B: n x m, C: p x n
 * row-major.  shifts: host array of nshifts shifts; nshifts = 0 computes
 * them with the Penzl heuristic (Ritz values of A^T and A^-T).  Z: n x *r_out
 * FP64 (ldz >= n, capacity rmax).  Warnings: CARE_WARN_STAGNATED,
 * CARE_WARN_MAXIT (Z holds the best factor so far). */
care_status care_solve(care_ctx* ctx, const care_csr* A, const double* B, int32_t m, const double* C,
                       int32_t p, double tol, const care_shift* shifts, int32_t nshifts,
                       const care_opts* opts, double* Z, int64_t ldz, int32_t rmax, int32_t* r_out,
                       care_stats* stats);

/* One CARE instance of a batch: the arguments care_solve takes for it. */
typedef struct {
  const care_csr* A;            /* device CSR of A (n x n), or NULL for a dense A  */
  const double* A_dense;        /* dense A (device, column-major) when A is NULL   */
  int64_t n_dense, lda_dense;
  const double* B;              /* device, n x m column-major (ld n)              */
  int32_t m;
  const double* C;              /* device, p x n row-major                        */
  int32_t p;
  const care_shift* shifts;     /* host; nshifts = 0 selects the heuristic shifts */
  int32_t nshifts;
  double* Z;                    /* device output, n x rmax, ld ldz >= n           */
  int64_t ldz;
  int32_t rmax;
} care_instance;

/* Outcome of one instance of care_solve_batch (host). */
typedef struct {
  int32_t status;               /* what care_solve returns for this instance      */
  int32_t r;                    /* columns of Z (CARE_ERR_CAPACITY: needed)       */
  care_stats stats;
  char message[128];            /* error text of a failed instance, else ""       */
} care_instance_result;

/* Batched Framework 1 over `count` independent CAREs of uneven sizes (the
 * paper solves one instance at a time): every instance is solved exactly as
 * care_solve would, with the same tol and opts; `workers` concurrent solves
 * (<= 0: min(count, 8)), each on its own non-blocking stream of the ctx's
 * device with its own host thread, pick instances largest n first, so that
 * the kernels of small instances fill the GPU together.  results: HOST array
 * of count entries.  Returns CARE_OK when every instance returned a status
 * >= 0, else the error of the first failed instance in input order (the
 * other instances are still solved).  Each instance's Z must be its own
 * buffer. */
care_status care_solve_batch(care_ctx* ctx, int32_t count, const care_instance* instances, double tol,
                             const care_opts* opts, int32_t workers, care_instance_result* results);

/* care_solve for a dense A (device, n x n column-major, leading dimension
 * lda >= n), e.g. the dense test CAREs of Sec. 5.1.  The shifted solves
 * factor A^T + p I once per real shift (partially pivoted LU in the inner
 * precision: for n <= 2048 every shift of a set in one launch of
 * care_shifted_lu_factor's kernel, solved by care_shifted_lu_solve's; beyond,
 * rocSOLVER getrf / getrs) and reuse the factors for every right-hand side
 * block; products with A^T are GEMMs.  Real shifts only
 * (CARE_ERR_NOT_IMPLEMENTED for complex ones) and inner precision FP64 or
 * FP32.  Other arguments, outputs and statuses as care_solve. */
care_status care_solve_dense(care_ctx* ctx, const double* A, int64_t n, int64_t lda, const double* B, int32_t m,
                             const double* C, int32_t p, double tol, const care_shift* shifts, int32_t nshifts,
                             const care_opts* opts, double* Z, int64_t ldz, int32_t rmax, int32_t* r_out,
                             care_stats* stats);

/* Penzl-type heuristic shifts (Sec. 5 takes its shifts from Krylov
 * subspaces; one reading is Penzl's procedure): Ritz values of kp Arnoldi steps with A^T and
 * of km steps with A^-T (inverted), FP64 on the GPU from ones / sqrt(n);
 * those in the open left half-plane are the candidates of the greedy min-max
 * choice of care_penzl_select.  real_only = 1 replaces each Ritz value by its
 * real part first.  shifts_out: HOST array with room for l0 + 1 entries (a
 * conjugate pair is never split); *count receives the number written.
 * Errors: CARE_ERR_UNSTABLE if no Ritz value has a negative real part,
 * CARE_ERR_BREAKDOWN if a solve with A^T fails. */
care_status care_penzl_shifts(care_ctx* ctx, const care_csr* A, int32_t l0, int32_t kp, int32_t km,
                              int32_t real_only, care_shift* shifts_out, int32_t* count);

/* Projection shifts (Benner, Kuerschner and Saak, ETNA 43, 2014; the other
 * reading of the Krylov-subspace shifts of Sec. 5): the Ritz values of
 * F = A^T - K B^T (K = NULL or m = 0: A^T) on span(V), V: n x s FP64
 * (ldv >= n), restricted to the dominant directions of V (eigenvalues of
 * V^T V above 1e-10 of the largest, at most 64), computed in precision
 * `prec` (CARE_FP64, or an FP32 variant: V, B, K rounded to FP32 and the
 * product in that variant); Ritz values in the right half-plane are
 * mirrored into the left one, and at most l0 shifts are chosen among them
 * by the greedy min-max rule of care_penzl_select.  B, K: n x m FP64 device
 * (ld n).  shifts_out: HOST array with room for l0 + 1 entries; *count
 * receives the number written.  Fails with CARE_ERR_UNSTABLE when no Ritz
 * value has a nonzero real part. */
care_status care_projection_shifts(care_ctx* ctx, const care_csr* A, const double* B, const double* K,
                                   int32_t m, const double* V, int64_t ldv, int32_t s, int32_t l0, int32_t prec,
                                   care_shift* shifts_out, int32_t* count);

/* Host step of the shift heuristic: the eigenvalues (re[i], im[i]) of the
 * k x k upper Hessenberg matrix H (HOST, column-major, ldh >= k; entries
 * below the subdiagonal are ignored), i.e. the Ritz values of an Arnoldi
 * run, by the Francis double-shift QR iteration.  Complex eigenvalues come
 * in adjacent conjugate pairs.  No device work. */
care_status care_ritz_values(const double* H, int32_t k, int64_t ldh, double* re, double* im);

/* Host step of the shift heuristic: greedy min-max choice among nr candidate
 * values (re[i], im[i]) (HOST; im may be NULL for real candidates).  Only
 * candidates with Re < 0 take part, in ascending (Re, Im) order.  The first
 * shift p minimises max_t |(t - p) / (t + p)|; then the candidate t that
 * maximises prod_{p chosen} |(t - p) / (t + p)| is added until l0 shifts are
 * chosen or every candidate is chosen.  A complex choice adds the pair
 * (Im > 0 first).  out: HOST, room for l0 + 1.  No device work. */
care_status care_penzl_select(const double* re, const double* im, int32_t nr, int32_t l0, care_shift* out,
                              int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* MPCARE_H */
