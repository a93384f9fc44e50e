/*
 * Reference (oracle) implementation of the one-sided Jacobi hyperbolic SVD.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential-by-definition
 * FP64 CPU implementation used to check the HIP library.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * Method: Novakovic & Singer, "A GPU-based hyperbolic SVD algorithm".
 *   - HSVD definition G = U [Sigma; 0] V^T, V^T J V = J           (Sec. 1, eq. 1.1)
 *   - one-sided recurrence G_k = G_{k-1} V_k^{-T}                   (Sec. 2, eq. 2.1)
 *   - trigonometric / hyperbolic rotations in tangent-cosine form    (Sec. 2, eq. 2.2)
 *   - relative orthogonality skip test                               (Sec. 2, eq. 2.3)
 *   - column updates                                                 (Sec. 2, eqs. 2.4, 2.5)
 *   - convergence code per sweep                                     (Sec. 4, eq. 4.2)
 *   - modified modulus pivot strategy                                (Sec. 2 and Sec. 4, Algs. 4.3, 4.4)
 *   - diagonal sorting                                               (Sec. 4, Alg. 4.1, Fig. 4.1 text)
 *   - bordering of odd orders                                        (Sec. 4, eq. 4.1)
 *   - block-column ordering (inner pass over a pivot block)          (Sec. 5, block-oriented algorithm)
 *
 * Where the paper is ambiguous or garbled, the reading taken is restated
 * where it is used in the .c file.
 */
#ifndef HSVD_ORACLE_H
#define HSVD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_NOCONV = -2, ORC_E_RANK = -3 };
enum { ORC_MODMOD = 0, ORC_ROUNDROBIN = 1 };

typedef struct {
    int ordering;     /* ORC_MODMOD or ORC_ROUNDROBIN (outer ordering)                  */
    int sort;         /* 1: sort the diagonal before sweep 0 and after every sweep      */
    int want_v;       /* 1: accumulate V (V^{-T} of the paper)                          */
    int max_sweeps;   /* stop with ORC_E_NOCONV after this many sweeps                  */
    double tol;       /* threshold of the skip test (eq. 2.3)                           */
    double tthresh;   /* T: |t| above it keeps the process going (eq. 4.2)              */
    int block;        /* 0: pairwise; b > 0: block-column ordering with blocks of b     */
    long max_steps;   /* > 0: stop after this many outer steps (bounded timing sample)  */
    int nthreads;     /* OpenMP threads over the independent pairs of one step          */
    int inner_sweeps; /* block > 0: 0 = block-oriented (each outer step annihilates the
                         pivot block's off-diagonal once, Sec. 5); k > 0 = full-block
                         (each outer step diagonalises the pivot block by sweeps of the
                         pointwise method over its 2b columns until one applies no
                         rotation, at most k, Sec. 6)                                  */
} orc_params;

typedef struct {
    int sweeps;       /* sweeps executed                                                */
    int code;         /* OR of the per-pair convergence codes of the last sweep         */
    long rotations;   /* rotations applied in total                                     */
    long skips;       /* pair visits skipped by eq. 2.3                                 */
    long steps;       /* outer steps executed                                           */
    int r;            /* bordered order                                                 */
    long inner;       /* full-block: inner sweeps executed, over all pivot blocks       */
} orc_info;

/* 2x2 pieces (exposed for pinning tests and bit-exact comparisons). */
int  orc_skip(double aii, double ajj, double aij, double tol);
int  orc_rotation(double aii, double ajj, double aij, int hyp, double *t, double *c);
int  orc_conv_code(int code, int rotated, double t, double tthresh);
void orc_pair_params_batch(long m, const double *aii, const double *ajj, const double *aij,
                           const int *hyp, double tol, double tthresh,
                           int *skip, double *t, double *c, int *status, int *code);

/* Orderings.  pairs receives r/2 pairs (i, j), i < j, as 2 ints each. */
int  orc_bordered_order(int n, int block);
int  orc_steps_per_sweep(int ordering, int r);
void orc_modmod_init(int r, int *state);             /* state: 4 ints per slot, r/2 slots */
void orc_modmod_pairs(int r, const int *state, int *pairs);
void orc_modmod_advance(int r, int *state);
void orc_roundrobin_pairs(int r, int step, int *pairs);
/* All pairs of sweep-relative outer step `step` of the block ordering, flattened in
   order: for each block pair, for each inner step, b pairs.  Returns pair count. */
int  orc_block_step_pairs(int r, int b, const int *outer_pairs, int step_in_sweep, int *pairs);

/* Stable diagonal sort (positive part decreasing, negative part increasing). */
void orc_sort(int r, int p, double *d, int *rho);

/* Full solve.  G is n x n column-major with leading dimension ldg (read only).
   Outputs (any except sigma may be NULL): sigma[n], U (n x n, ld n),
   V (n x n, ld n), lambda[n], perm[n].                                          */
int  orc_hsvd(int n, int p, const double *G, int ldg, const orc_params *prm,
              double *sigma, double *U, double *V, double *lambda, int *perm,
              orc_info *info);

#ifdef __cplusplus
}
#endif
#endif
