/*
 * hsvd.h -- C ABI of libhsvd.so: one-sided Jacobi hyperbolic SVD on MI355X (gfx950).
 *
 * Method: Novakovic & Singer, "A GPU-based hyperbolic SVD algorithm".
 * For a square factor G (n x n, full column rank) and J = diag(+1 x p, -1 x (n-p))
 * the library computes G = U Sigma V^T with U orthogonal and V^T J V = J
 * (Sec. 1, eq. 1.1), and the eigenvalues Sigma^2 J of M = G J G^T (Sec. 1).
 *
 * Conventions shared by every entry point:
 *  - Matrices are column-major FP64.  Every pointer argument named as "device"
 *    is a device pointer on the context's device (e.g. a torch tensor's
 *    data_ptr()); "host" pointers are ordinary host memory.
 *  - The caller owns and allocates every input and output.  The library owns
 *    its workspace (allocated on first use, grown on demand, released by
 *    hsvd_destroy) and never frees or retains caller memory.
 *  - All device work is enqueued on the context's stream.  Entry points that
 *    return an hsvd_info synchronise with that stream before returning.
 *  - Errors are returned as hsvd_status; nothing is thrown across the ABI.
 *    On HSVD_E_INVAL nothing is launched.  On HSVD_E_NOCONV and HSVD_E_RANK
 *    the outputs hold the current iterate.
 *  - A context is not thread-safe: one host thread at a time per context.
 */
#ifndef HSVD_H
#define HSVD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsvd_ctx hsvd_ctx;

typedef enum {
    HSVD_OK = 0,
    HSVD_E_INVAL = -1,   /* bad argument, non-finite input                          */
    HSVD_E_NOCONV = -2,  /* max_sweeps reached without meeting the stop rule        */
    HSVD_E_RANK = -3,    /* zero column, or a hyperbolic pair with |tanh 2phi| >= 1
                            (G, or G J G^T, numerically rank deficient; Sec. 1)     */
    HSVD_E_NOMEM = -4,   /* workspace allocation failed                             */
    HSVD_E_DEVICE = -5,  /* a HIP runtime call failed                               */
    HSVD_E_SIZE = -6     /* hsvd_solve_noalloc: the solve needs more workspace than
                            the fixed scratch array (HSVD_NOALLOC_BYTES) holds    */
} hsvd_status;

/* Size in bytes of the fixed device scratch array of hsvd_solve_noalloc (per
   device, held from library load to process exit).  It holds the workspace of
   a solve of order n <= 1024 on every path (FP64 pairwise or block, mixed). */
#define HSVD_NOALLOC_BYTES (64u << 20)

typedef enum { HSVD_FP64 = 0, HSVD_MIXED = 1 } hsvd_precision;
typedef enum { HSVD_AUTO = 0, HSVD_PAIRWISE = 1, HSVD_BLOCK = 2 } hsvd_algo;
typedef enum { HSVD_ORD_MODMOD = 0, HSVD_ORD_ROUNDROBIN = 1 } hsvd_ordering;

typedef struct {
    int precision;   /* hsvd_precision: HSVD_FP64, or HSVD_MIXED = FP32 block sweeps on
                        FP32 MFMA until they stop paying (the largest rotation
                        tangent or the rotating fraction stops falling, or falls
                        below FP32 reach), FP64 J-re-orthogonalisation of V, then
                        FP64 block sweeps.  If an FP32 sweep flags a pair as rank deficient, or
                        the re-orthogonalisation ends above reorth_accept, the solve
                        starts again from G in FP64 (hsvd_info.fp64_restart)           */
    int algo;        /* hsvd_algo                                                        */
    int ordering;    /* hsvd_ordering: modified modulus (Sec. 2, Algs. 4.3-4.4) or the
                        round-robin circle method starting on the same antidiagonal      */
    int block;       /* block width b of the block path: 0 or 32; or 64 (FP64 single solves
                        only: the wide block path, Gram and update on the FP64 MFMA GEMM,
                        working copies in sorted position order)                        */
    int sort;        /* 1: sort the diagonal before sweep 0 and after every sweep (Alg. 4.1) */
    int want_v;      /* 1: accumulate V (V^{-T} of the paper, eq. 2.1)                   */
    int max_sweeps;  /* <= 0: 100                                                        */
    double tol;      /* threshold of the relative orthogonality test (eq. 2.3); <= 0: 1e-15 n */
    double t_thresh; /* T of eq. (4.2); <= 0: sqrt(tol) / 2 (Sec. 2)                     */
    int graph;       /* 1 = capture one sweep's launches as a HIP graph and replay it
                        every sweep: the step launches of the pairwise path (timed per
                        sweep as before), and a whole sweep of a batched group (no
                        per-kernel timing in hsvd_info then); 0 = stream launches     */
    int inner_sweeps; /* block path.  0: block-oriented method (Sec. 5) -- each outer step
                        annihilates the pivot block's off-diagonal entries once (all pairs
                        of the 2b columns in the first outer step of a sweep, the cross
                        pairs in the others).  k in [1, 100]: full-block method (Sec. 6)
                        -- each outer step diagonalises the pivot block by sweeps of the
                        pointwise method over its 2b columns until one rotates nothing, at
                        most k.  k > 0 makes HSVD_AUTO take the block path; the pairwise
                        path rejects k > 0 with HSVD_E_INVAL                           */
    double reorth_accept; /* mixed path: largest accepted max |J X^T J X - I| after the
                        Newton-Schulz J-re-orthogonalisation of V (above it the
                        solve restarts from G in FP64); <= 0: 16384 n u, u = 2^-53  */
    int batch_mode;  /* hsvd_solve_batched, the sweep schedule: 0 = every
                        block-oriented problem with n <= 256, FP64 or mixed, in
                        one persistent launch (the others, and the full-block
                        method, in launches grouped by bordered order); 1 =
                        grouped launches for every problem; 2 (default) = the
                        schedule hsvd_autotune_batched chose for the precision,
                        0 before tuning.  FP64: 0 and 1 give bit-identical
                        results.  Mixed: each gives a valid mixed trajectory (the
                        FP64 sweeps of a problem start at the stepper phase its
                        own FP32 sweeps left, in the grouped launches at the
                        group's)                                               */
    int persistent;  /* pairwise path: 0 = one launch per parallel step (replayed from a
                        HIP graph when graph = 1) and the stop rule checked on the host
                        after every sweep; 1 = all sweeps in one persistent cooperative
                        launch: a pair waits only for the two visits of the previous
                        step that last held its columns (per-column visit counts), and
                        the diagonal sort and the stop rule (eq. 4.2) run on the device
                        at every sweep's end; 2 = the same launch with a grid barrier
                        between steps.  All three give bit-identical results; the
                        block path ignores it.  Other values: HSVD_E_INVAL          */
} hsvd_params;

/* Kernel classes timed in hsvd_info (index into the kernel_* arrays). */
enum {
    HSVD_K_PAIR_STEP = 0,      /* pairwise path: one parallel step of pivot pairs          */
    HSVD_K_BLOCK_GRAM = 1,     /* block path, FP64: Gram matrices G_P^T G_P                */
    HSVD_K_BLOCK_INNER = 2,    /* block path, FP64: inner rotations of each block pair     */
    HSVD_K_BLOCK_UPDATE = 3,   /* block path, FP64: [G_P | V_P] <- [G_P | V_P] W           */
    HSVD_K_BLOCK_GRAM32 = 4,   /* mixed path, FP32 sweeps: Gram on FP32 MFMA               */
    HSVD_K_BLOCK_INNER32 = 5,  /* mixed path, FP32 sweeps: inner rotations, parameters in   */
                               /* FP64, applied to the FP32-held blocks                     */
    HSVD_K_BLOCK_UPDATE32 = 6, /* mixed path, FP32 sweeps: update on FP32 MFMA             */
    HSVD_K_REORTH = 7,         /* mixed path: J-re-orthogonalisation of V and G1 = G X     */
                               /* (FP64 MFMA products, gemm_kernels)                       */
    HSVD_NKERNELS = 8
};

typedef struct {
    int status;              /* same value as returned                                   */
    int sweeps;              /* sweeps executed (the last one met the stop rule)         */
    int code;                /* OR of the eq. (4.2) codes of the last sweep              */
    int r;                   /* bordered order (eq. 4.1)                                 */
    int block;               /* block width b used; 0 = pairwise path                    */
    int ldg;                 /* padded leading dimension of the working copies           */
    int sweeps_fp32;         /* mixed path: FP32 sweeps before the FP64 refinement       */
    int reorth_iters;        /* mixed path: Newton-Schulz iterations on V                */
    double max_t_last;       /* largest |t| of the last sweep                            */
    double reorth_resid;     /* mixed path: final max |J X^T J X - I|                    */
    int fp64_restart;        /* mixed path: 1 when the FP32 phase was abandoned and the
                                solve ran again in FP64 from G (rank flag in an FP32
                                sweep, or reorth_resid above reorth_accept)            */
    int pad_;
    long long rotations;     /* rotations applied                                        */
    long long skips;         /* pair visits skipped by eq. (2.3)                         */
    long long steps;         /* parallel (outer) steps executed                          */
    long long active_pairs;  /* block pair steps with at least one rotation              */
    double ms_total;         /* device time of the solve (event pair on the stream)      */
    double kernel_ms[HSVD_NKERNELS];         /* device time per kernel class (HIP events);
                                                block sweeps time the first step of each
                                                sweep and every 8th step after it and
                                                count the other steps of that sweep at
                                                the mean of its timed ones              */
    long long kernel_launches[HSVD_NKERNELS];
    double kernel_bytes[HSVD_NKERNELS];      /* algorithmic bytes: the columns of G
                                                and V a kernel class must read and
                                                write (Gram: 2b columns per block
                                                pair; update: the touched columns,
                                                read and written; pairwise: two
                                                columns per visit)                  */
    double kernel_flops[HSVD_NKERNELS];      /* algorithmic flops                        */
    long long kernel_timed[HSVD_NKERNELS];   /* launches that were timed by events      */
} hsvd_info;

/* Creates a context bound to HIP device `device` and stream `hip_stream`
   (a hipStream_t; NULL = the device's null stream).  *ctx receives the
   handle.  Errors: HSVD_E_INVAL (ctx NULL, bad device), HSVD_E_DEVICE. */
hsvd_status hsvd_init(hsvd_ctx **ctx, int device, void *hip_stream);

/* Releases the workspace and the handle (synchronises with the stream first). */
hsvd_status hsvd_destroy(hsvd_ctx *ctx);

/* Fills *prm with the defaults: FP64, AUTO, modified modulus, sort on, V on,
   max_sweeps 100, tol and t_thresh from n at solve time, graph replay on. */
void hsvd_default_params(hsvd_params *prm);

/* One-sided Jacobi HSVD of a square G (Sec. 2 and Sec. 4, Algs. 4.1-4.5).
 *   G       device, n x n, leading dimension lda >= n; read only (copied).
 *   jsig    device, n signed chars (+1 or -1): J's diagonal in the column
 *           order of G, with exactly p entries +1 in any order; or NULL for
 *           J = diag(I_p, -I_{n-p}).  A signature that is not already in that
 *           canonical order is handled by stably partitioning the columns (+1
 *           first), solving, and mapping the outputs back to the input column
 *           order (V = P V_p P^T, so G V = U Sigma and V^T J V = J with the
 *           caller's J); this copies G once more and reads jsig to the host.
 *   n, p    order and number of +1 signs in J (0 <= p <= n).
 *   prm     host; NULL = defaults.
 * Outputs (device, caller-allocated; any may be NULL except sigma):
 *   sigma[n]   hyperbolic singular values, physical (input) column order.
 *   U          n x n, ldu >= n: U = G_final Sigma^{-1} (Sec. 2).
 *   V          n x n, ldv >= n: the accumulated V^{-T} of eq. (2.1), so that
 *              G V = U Sigma and V^T J V = J; the paper's V is J V J.
 *   lambda[n]  eigenvalues of G J G^T: sigma_c^2 times the sign of column c.
 *   perm[n]    physical column index by final sorted position (rho of Fig. 4.1).
 *   info       host; may be NULL.
 * Odd n is bordered by a unit column with a negative sign (eq. 4.1); the
 * border never appears in the outputs.  Errors: see hsvd_status; HSVD_E_INVAL
 * also for a jsig entry other than +-1 or a count of +1 entries other than p.
 * Synchronises with the context's stream before returning. */
hsvd_status hsvd_solve(hsvd_ctx *ctx, const double *G, int lda, const signed char *jsig, int n, int p,
                       const hsvd_params *prm, double *sigma, double *U, int ldu, double *V, int ldv,
                       double *lambda, int *perm, hsvd_info *info);

/* hsvd_solve without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Computes what hsvd_solve computes with jsig = NULL
 * (J = diag(I_p, -I_{n-p})), the same arguments otherwise, by the same kernels
 * and launches: the results are identical to hsvd_solve's for the same G and
 * parameters.  Differences:
 *  - The workspace is a fixed array of HSVD_NOALLOC_BYTES in device memory
 *    that the library reserves per device; no hipMalloc, hipFree, event or
 *    graph is created.  A solve whose workspace does not fit returns
 *    HSVD_E_SIZE before launching anything (its size grows as 16 n^2 bytes
 *    for FP64, about 54 n^2 for HSVD_MIXED; every path fits for n <= 1024).
 *  - prm->graph is ignored (stream launches), and hsvd_info carries no times
 *    (ms_total and kernel_ms are zero).
 *  - prm->persistent must be 0 (HSVD_E_INVAL otherwise): the persistent
 *    pairwise kernel is a cooperative launch, which the runtime may back
 *    with allocations of its own.
 *  - Every call on one device uses that device's one array, whatever the
 *    context: calls that overlap on one device (two host threads, or two
 *    contexts on different streams) race and corrupt each other.  Calls on one
 *    context are ordered by its stream, and each call initialises all of the
 *    workspace it reads; the array keeps the last call's contents.
 * Errors: as hsvd_solve, plus HSVD_E_SIZE.  Synchronises. */
hsvd_status hsvd_solve_noalloc(hsvd_ctx *ctx, const double *G, int lda, int n, int p, const hsvd_params *prm,
                               double *sigma, double *U, int ldu, double *V, int ldv, double *lambda, int *perm,
                               hsvd_info *info);

/* Batched solves: `batch` independent problems G_k (n[k] x n[k], 1 <= n[k] <= 1024,
 * J_k = diag(I_p[k], -I_{n[k]-p[k]})), each solved as by hsvd_solve with the block
 * path and its own tolerance (prm->tol <= 0: 1e-15 n[k]) and stop rule, in FP64
 * or (prm->precision = HSVD_MIXED) with FP32 sweeps first, each problem leaving
 * them by its own switch rule, then the J-re-orthogonalisation of its V and
 * FP64 refinement sweeps (or, per problem, the FP64 restart of hsvd_solve).
 *   n, p, off, voff  device (or host) arrays of `batch` entries: order, number of
 *                    +1 signs, element offset of G_k / U_k / V_k in the packed
 *                    matrices (column-major, leading dimension n[k]), element
 *                    offset of sigma_k / lambda_k in the packed vectors.  The
 *                    library reads them to the host once, to plan the launches.
 *   G                device, packed inputs (read only).
 *   sigma, U, V, lambda  device, packed outputs (U, V, lambda may be NULL;
 *                    V requires prm->want_v).
 *   info             device or host array of `batch` hsvd_info, or NULL: per
 *                    problem status, sweeps (FP64), sweeps_fp32, code, r, block,
 *                    ldg, reorth_iters, reorth_resid, fp64_restart, rotations,
 *                    skips, active_pairs; ms_total is the device time of the
 *                    whole batched call; the kernel_* arrays are zero.
 * Problems of the block-oriented method with n <= 256 run in one persistent
 * launch (prm->batch_mode = 0; with the default 2, before tuning or when
 * hsvd_autotune_batched chose it for the precision; captured as a HIP graph
 * when prm->graph is set): each workgroup takes problems from a device work queue,
 * largest n first, and solves each one completely -- Gram, inner rotations
 * and update of every block pair, sort and the stop rule of eq. (4.2) per
 * sweep; with mixed precision first the FP32 sweeps, the switch rule and the
 * J-re-orthogonalisation of V -- then output extraction, with no host round
 * trip.  The other problems (n > 256, the full-block method, batch_mode = 1,
 * or 2 when tuning chose the grouped launches) are grouped by their bordered
 * order (a multiple of 2b); each
 * group runs as one sequence of launches that covers all of its problems,
 * with the stop rule decided per problem on the device.  In FP64 both forms
 * give bit-identical results (in mixed precision see batch_mode).  Returns
 * HSVD_OK when every problem converged, else the status of the first problem
 * that did not.  Synchronises. */
hsvd_status hsvd_solve_batched(hsvd_ctx *ctx, int batch, const int *n, const int *p, const long long *off,
                               const long long *voff, const double *G, const hsvd_params *prm, double *sigma,
                               double *U, double *V, double *lambda, hsvd_info *info);

/* Autotuner.  Times the speed-only choices of the library on a seeded synthetic
 * problem of order n (uniform entries in [-1, 1) from a counter-based hash,
 * p = n/2; two sweeps per candidate): the path (pairwise, or block with the
 * Gram's rows split for 256 / 512 / 1024 / 2048 workgroups per step).  The
 * fastest is kept for n's size bucket (n rounded up to a power of two) in the
 * context; later hsvd_solve calls with algo = HSVD_AUTO and block = 0 in that
 * bucket use it.  A solve's result depends on the choice only through the
 * pivot ordering of the chosen path and the Gram's summation order.  When the
 * environment variable HSVD_AUTOTUNE_CACHE names a file, hsvd_init reads the
 * table from it (JSON written by this call) and this call writes it back.
 *   best_algo, best_wg   host, may be NULL: the chosen path and workgroup target.
 * Errors: HSVD_E_INVAL (n < 2 or n > 16382).  Synchronises. */
hsvd_status hsvd_autotune(hsvd_ctx *ctx, int n, int *best_algo, int *best_wg);

/* Autotuner of the batched solver.  Block-oriented problems with n <= 256 run
 * in one persistent launch in which each workgroup solves whole problems;
 * its width (256, 512 or 1024 threads per problem: the inner rotations and the
 * column updates of a block pair spread over all of them) is a speed-only
 * choice.  This call times the three widths on a sample of at most 4096 of the
 * given problems (every k-th, the ones with n <= 256; seeded synthetic entries,
 * uniform in [-1, 1) from a counter-based hash; V accumulated) and keeps the
 * fastest for the bucket of the sample's largest order ((0, 64], (64, 128],
 * (128, 192], (192, 256]) in the context; later hsvd_solve_batched calls whose
 * persistent problems fall in that bucket use it (default before tuning: 256).
 * The results of a batched solve do not depend on the width (bit-identical).
 * Then, with the chosen width, it times the two sweep schedules (one persistent
 * launch, launches grouped by order; batch_mode 0 and 1) in FP64 and in mixed
 * precision on the orders of all the given problems with n <= 256, up to
 * 16384 of them (every k-th beyond; seeded synthetic entries as above: the
 * grouped launches gain with the number of problems per group, so a small
 * sample would not tell) and keeps the faster per precision for
 * hsvd_solve_batched calls with batch_mode = 2 (hsvd_batched_schedule reports
 * the choice).  Its inputs and outputs take three times their packed size in
 * the context's auxiliary device buffer, kept until hsvd_destroy.  With HSVD_AUTOTUNE_CACHE
 * set the choices are written to that file too.
 *   n, p          device or host arrays of `batch` entries (as hsvd_solve_batched).
 *   best_threads  host, may be NULL: the chosen width.
 *   ms            host, may be NULL: 3 floats, the time of each width (ms).
 * Errors: HSVD_E_INVAL (no problem with n <= 256, or bad n / p).  Synchronises. */
hsvd_status hsvd_autotune_batched(hsvd_ctx *ctx, int batch, const int *n, const int *p, int *best_threads,
                                  float *ms);

/* The sweep schedule hsvd_solve_batched takes with batch_mode = 2 for
 * `precision` (HSVD_FP64 or HSVD_MIXED): *mode = 0 (one persistent launch),
 * 1 (launches grouped by order), or -1 (not tuned: the persistent launch).
 * Errors: HSVD_E_INVAL (ctx or mode NULL, another precision). */
hsvd_status hsvd_batched_schedule(const hsvd_ctx *ctx, int precision, int *mode);

/* ---- Diagnostics: the individual steps of the path on caller data ---- */

/* Elementwise skip test (eq. 2.3), rotation parameters (Sec. 2: t = tan / tanh
 * of the angle that annihilates a_ij under eqs. 2.4/2.5, c = cos / cosh) and
 * convergence code (eq. 4.2), computed by the device routine the solver uses.
 *   m                      number of items.
 *   aii, ajj, aij (device) m doubles each; hyp (device) m ints, -1 trig, +1 hyperbolic.
 *   skip, status, code     (device) m ints out: 1 = skipped; 1 = rank failure; code.
 *   t, c                   (device) m doubles out (t = 0, c = 1 when skipped).
 * Synchronises.  Errors: HSVD_E_INVAL (m < 0, NULL arrays). */
hsvd_status hsvd_pair_params(hsvd_ctx *ctx, long long m, const double *aii, const double *ajj,
                             const double *aij, const int *hyp, double tol, double t_thresh,
                             int *skip, double *t, double *c, int *status, int *code);

/* As hsvd_pair_params, with the rotation routine of the block path's inner
 * solves (the same rotation in a shorter dependency chain: one square root and
 * Newton-refined hardware reciprocal and reciprocal square root; within a few
 * ulps of hsvd_pair_params; for a_ii = a_jj trigonometric pairs it takes
 * t = sgn(a_ij)).  Same arguments, errors and synchronisation. */
hsvd_status hsvd_block_pair_params(hsvd_ctx *ctx, long long m, const double *aii, const double *ajj,
                                   const double *aij, const int *hyp, double tol, double t_thresh,
                                   int *skip, double *t, double *c, int *status, int *code);

/* Pivot pairs produced by the device stepper (Algs. 4.3-4.4, or round-robin)
 * for `steps` consecutive steps starting at the first step of sweep 0.
 *   r          even order (2 <= r).
 *   pairs      device, steps x (r/2) x 2 ints out: (i, j), i < j, per slot.
 * Synchronises.  Errors: HSVD_E_INVAL. */
hsvd_status hsvd_pivot_trace(hsvd_ctx *ctx, int ordering, int r, int steps, int *pairs);

/* Block-path pivot positions of `steps` consecutive outer steps from the
 * start of sweep 0 (outer ordering over nb = r/b blocks; inner ordering of
 * each block pair as used by the solver).
 *   r, b       r a multiple of 2b; b = 32 or 64 (the block widths the library runs).
 *   pairs      device ints out, concatenated over the steps: step s contributes
 *              (nb/2) x inner(s) x b pairs (i, j), i < j, ordered by block pair,
 *              inner step, slot; inner(s) = 2b - 1 at the first step of a sweep,
 *              else b.
 * Synchronises.  Errors: HSVD_E_INVAL. */
hsvd_status hsvd_block_trace(hsvd_ctx *ctx, int ordering, int r, int b, int steps, int *pairs);

/* Device diagonal sort (Sec. 4, Sort_Diagonal): stable; positions [0, p) by
 * d decreasing, [p, r) by d increasing; rho travels with d.  In place on
 *   d (device, r doubles), rho (device, r ints).  r <= 16384.  Keys are
 *   compared in the IEEE-754 total order of their bit patterns: the numeric
 *   order on the non-negative values the solver produces (it separates -0.0
 *   from +0.0 and places NaN beyond +inf), and a permutation for any input.
 * Synchronises.  Errors: HSVD_E_INVAL. */
hsvd_status hsvd_sort_diag(hsvd_ctx *ctx, int r, int p, double *d, int *rho);

/* Library version string (static storage). */
const char *hsvd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HSVD_H */
