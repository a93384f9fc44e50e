/*
 * Oracle: plain FP64 one-sided Jacobi hyperbolic SVD on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY -- loaded by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark; never by the library.  It shares no
 * code with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math).  Every floating
 * point operation below is a separately rounded IEEE-754 binary64 operation
 * except the explicit fma() calls; sqrt() and '/' are correctly rounded.
 *
 * Paper: Novakovic & Singer, "A GPU-based hyperbolic SVD algorithm".
 */
#include "hsvd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* 2x2 pieces                                                                 */
/* ------------------------------------------------------------------------- */

/* Relative orthogonality test, eq. (2.3): the pair is skipped when
   |a_ij| < tol * sqrt(a_ii a_jj).  The square root of the product is taken as
   sqrt(a_ii) * sqrt(a_jj) so that it cannot overflow or underflow. */
int orc_skip(double aii, double ajj, double aij, double tol)
{
    return fabs(aij) < tol * (sqrt(aii) * sqrt(ajj));
}

/* Rotation parameters (Sec. 2, eq. 2.2 and the definitions of hyp, theta, t).
 *
 * The rotation must annihilate a_ij under the update rules (2.4) / (2.5):
 *   trigonometric (hyp = -1): tan(2 phi)  =  2 a_ij / (a_jj - a_ii)
 *   hyperbolic    (hyp = +1): tanh(2 phi) = -2 a_ij / (a_ii + a_jj)
 * i.e. theta = 2 a_ij / (-a_ii - hyp a_jj).  (The printed denominator
 * -a_ii + hyp a_jj does not annihilate a_ij under (2.4)/(2.5); this sign is
 * the reading adopted.)  With zeta = 1/theta, t = tan(phi) resp. tanh(phi) is
 * the root of smaller magnitude of
 *   trig: t^2 + 2 zeta t - 1 = 0  ->  t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2))
 *   hyp:  t^2 - 2 zeta t + 1 = 0  ->  t = sgn(zeta) / (|zeta| + sqrt(zeta^2 - 1))
 * and c = cos(phi) = 1/sqrt(1 + t^2) resp. cosh(phi) = 1/sqrt((1 - t)(1 + t)).
 * sgn(0) = +1.  For |zeta| > 2^500 the root is t = 1/(2 zeta) to working
 * precision.  A hyperbolic pair needs |zeta| > 1 (|tanh 2phi| < 1); otherwise
 * the pair is numerically rank deficient and 1 is returned. */
int orc_rotation(double aii, double ajj, double aij, int hyp, double *t, double *c)
{
    const double big = 0x1p500;
    double two_aij = 2.0 * aij;
    if (hyp < 0) {
        double zeta = (ajj - aii) / two_aij;
        double az = fabs(zeta);
        double sg = (zeta < 0.0) ? -1.0 : 1.0;
        double tt;
        if (az > big) {
            tt = 0.5 / zeta;
        } else {
            double zz = zeta * zeta;
            double s = sqrt(1.0 + zz);
            tt = sg / (az + s);
        }
        double tsq = tt * tt;
        *t = tt;
        *c = 1.0 / sqrt(1.0 + tsq);
        return 0;
    } else {
        double num = aii + ajj;
        double zeta = -num / two_aij;
        double az = fabs(zeta);
        if (!(az > 1.0)) {
            *t = 0.0;
            *c = 1.0;
            return 1;
        }
        double sg = (zeta < 0.0) ? -1.0 : 1.0;
        double tt;
        if (az > big) {
            tt = 0.5 / zeta;
        } else {
            double s = sqrt(az - 1.0) * sqrt(az + 1.0);
            tt = sg / (az + s);
        }
        double omt = 1.0 - tt;
        double opt = 1.0 + tt;
        *t = tt;
        *c = 1.0 / sqrt(omt * opt);
        return 0;
    }
}

/* Per-pair convergence code, eq. (4.2): unchanged when no rotation was
   applied; (11)_2 when |t| > T; otherwise (01)_2 OR the previous code. */
int orc_conv_code(int code, int rotated, double t, double tthresh)
{
    if (!rotated) return code;
    if (fabs(t) > tthresh) return 3;
    return code | 1;
}


/* Element-wise skip test, rotation parameters and convergence code for m
   independent (a_ii, a_jj, a_ij, hyp) items.  For comparisons on identical
   inputs; skip[k] = 1 means eq. (2.3) held and no rotation is formed. */
void orc_pair_params_batch(long m, const double *aii, const double *ajj, const double *aij,
                           const int *hyp, double tol, double tthresh,
                           int *skip, double *t, double *c, int *status, int *code)
{
    for (long k = 0; k < m; ++k) {
        skip[k] = orc_skip(aii[k], ajj[k], aij[k], tol);
        t[k] = 0.0;
        c[k] = 1.0;
        status[k] = 0;
        code[k] = 0;
        if (skip[k]) continue;
        status[k] = orc_rotation(aii[k], ajj[k], aij[k], hyp[k], &t[k], &c[k]);
        if (status[k] == 0) code[k] = orc_conv_code(0, 1, t[k], tthresh);
    }
}

/* ------------------------------------------------------------------------- */
/* Orderings                                                                  */
/* ------------------------------------------------------------------------- */

/* Order after bordering (eq. 4.1): pairwise needs an even order; the block
   ordering needs a multiple of 2b.  Added columns are unit vectors with a
   negative sign in J. */
int orc_bordered_order(int n, int block)
{
    int m = (block > 0) ? 2 * block : 2;
    return ((n + m - 1) / m) * m;
}

int orc_steps_per_sweep(int ordering, int r)
{
    return (ordering == ORC_ROUNDROBIN) ? r - 1 : r;
}

/* Modified modulus strategy, Alg. 4.3: slot k starts on the antidiagonal
   (k, r-1-k).  state[4k..4k+3] = (ip, jp, iblk, jblk). */
void orc_modmod_init(int r, int *state)
{
    for (int k = 0; k < r / 2; ++k) {
        state[4 * k + 0] = k;
        state[4 * k + 1] = r - k - 1;
        state[4 * k + 2] = k;
        state[4 * k + 3] = r - k - 1;
    }
}

void orc_modmod_pairs(int r, const int *state, int *pairs)
{
    for (int k = 0; k < r / 2; ++k) {
        pairs[2 * k + 0] = state[4 * k + 2];
        pairs[2 * k + 1] = state[4 * k + 3];
    }
}

/* Alg. 4.4, with the comparison read as ip + jp >= r - 1 (the printed strict
   comparison sends every slot past the last column on the first transition,
   because all slots start on the antidiagonal ip + jp = r - 1). */
void orc_modmod_advance(int r, int *state)
{
    for (int k = 0; k < r / 2; ++k) {
        int *s = state + 4 * k;
        if (s[0] + s[1] >= r - 1) {
            s[0] += 1;
            if (s[0] == s[1]) {
                s[0] -= r / 2;
                s[1] = s[0];
            }
            s[2] = s[0];
        } else {
            s[1] += 1;
            s[3] = s[1];
        }
    }
}

/* Round-robin (circle method) ordering over r indices: index 0 is fixed and
   the other r-1 rotate by one place per step; slot k pairs the k-th and the
   (r-1-k)-th entries of the arrangement.  r-1 steps cover every pair once. */
void orc_roundrobin_pairs(int r, int step, int *pairs)
{
    int *L = (int *)malloc(sizeof(int) * (size_t)r);
    L[0] = 0;
    for (int m = 1; m < r; ++m) L[m] = 1 + ((m - 1 + step) % (r - 1));
    for (int k = 0; k < r / 2; ++k) {
        int a = L[k], b = L[r - 1 - k];
        pairs[2 * k + 0] = a < b ? a : b;
        pairs[2 * k + 1] = a < b ? b : a;
    }
    free(L);
}

/* Inner pairs of one block pair (I, J), I < J, in local indices x in [0, 2b):
   x < b is position I*b + x, x >= b is position J*b + x - b.
   First outer step of a sweep: every pair of the 2b columns once, by the
   circle method over 2b indices (2b - 1 inner steps).  Other outer steps:
   only the cross pairs between the two blocks, b inner steps, inner step u
   pairing x with b + ((x + u) mod b).  Returns the number of inner pairs
   written to loc (2 ints each, local indices, first < second). */
static int block_inner_pairs(int b, int first_step, int *loc)
{
    int cnt = 0;
    if (first_step) {
        int m = 2 * b;
        int *tmp = (int *)malloc(sizeof(int) * (size_t)m);
        for (int u = 0; u < m - 1; ++u) {
            orc_roundrobin_pairs(m, u, tmp);
            for (int k = 0; k < b; ++k) {
                loc[2 * cnt + 0] = tmp[2 * k + 0];
                loc[2 * cnt + 1] = tmp[2 * k + 1];
                ++cnt;
            }
        }
        free(tmp);
    } else {
        for (int u = 0; u < b; ++u)
            for (int x = 0; x < b; ++x) {
                loc[2 * cnt + 0] = x;
                loc[2 * cnt + 1] = b + ((x + u) % b);
                ++cnt;
            }
    }
    return cnt;
}

static int loc_to_pos(int b, int I, int J, int x)
{
    return (x < b) ? I * b + x : J * b + (x - b);
}

int orc_block_step_pairs(int r, int b, const int *outer_pairs, int step_in_sweep, int *pairs)
{
    int nb = r / b;
    int *loc = (int *)malloc(sizeof(int) * (size_t)(2 * b * (2 * b - 1)));
    int cnt = block_inner_pairs(b, step_in_sweep == 0, loc);
    int out = 0;
    for (int k = 0; k < nb / 2; ++k) {
        int I = outer_pairs[2 * k], J = outer_pairs[2 * k + 1];
        for (int q = 0; q < cnt; ++q) {
            int a = loc_to_pos(b, I, J, loc[2 * q]);
            int c = loc_to_pos(b, I, J, loc[2 * q + 1]);
            pairs[2 * out + 0] = a < c ? a : c;
            pairs[2 * out + 1] = a < c ? c : a;
            ++out;
        }
    }
    free(loc);
    return out;
}

/* ------------------------------------------------------------------------- */
/* Diagonal sorting                                                           */
/* ------------------------------------------------------------------------- */

/* Stable sort of the positions: [0, p) by d decreasing, [p, r) by d
   increasing; rho travels with its key; equal keys keep their order.  The
   partition between the two signs of J is never crossed. */
void orc_sort(int r, int p, double *d, int *rho)
{
    for (int q = 1; q < p; ++q) {
        double key = d[q];
        int val = rho[q];
        int m = q - 1;
        while (m >= 0 && d[m] < key) {
            d[m + 1] = d[m];
            rho[m + 1] = rho[m];
            --m;
        }
        d[m + 1] = key;
        rho[m + 1] = val;
    }
    for (int q = p + 1; q < r; ++q) {
        double key = d[q];
        int val = rho[q];
        int m = q - 1;
        while (m >= p && d[m] > key) {
            d[m + 1] = d[m];
            rho[m + 1] = rho[m];
            --m;
        }
        d[m + 1] = key;
        rho[m + 1] = val;
    }
}

/* ------------------------------------------------------------------------- */
/* The sweep loop                                                             */
/* ------------------------------------------------------------------------- */

static double dot(int len, const double *x, const double *y)
{
    double s = 0.0;
    for (int q = 0; q < len; ++q) s = fma(x[q], y[q], s);
    return s;
}

typedef struct {
    int r, p;
    double *G, *V, *d;
    int *rho;
    double tol, tthresh;
} orc_state;

typedef struct {
    int code;
    long rot, skip;
    int rank;
} orc_acc;

/* One pivot pair (i, j), i < j, positions: Alg. 4.5.
   a_ii, a_jj are the kept diagonal, a_ij a fresh dot product of the physical
   columns rho(i), rho(j).  Update (2.4)/(2.5) with the parenthesised part as
   one FMA:  g_i' = (g_i + hyp t g_j) c,  g_j' = (t g_i + g_j) c.
   New diagonal entries are fresh dot products of the new columns. */
static void pair_rotate(const orc_state *st, int i, int j, orc_acc *acc)
{
    int r = st->r;
    int ci = st->rho[i], cj = st->rho[j];
    double *gi = st->G + (size_t)ci * r;
    double *gj = st->G + (size_t)cj * r;
    double aii = st->d[i], ajj = st->d[j];
    double aij = dot(r, gi, gj);
    if (orc_skip(aii, ajj, aij, st->tol)) {
        acc->skip += 1;
        return;
    }
    int hyp = ((i < st->p) == (j < st->p)) ? -1 : 1;
    double t, c;
    if (orc_rotation(aii, ajj, aij, hyp, &t, &c)) {
        acc->rank = 1;
        return;
    }
    double ht = (hyp < 0) ? -t : t;
    for (int q = 0; q < r; ++q) {
        double x = gi[q], y = gj[q];
        gi[q] = fma(ht, y, x) * c;
        gj[q] = fma(t, x, y) * c;
    }
    st->d[i] = dot(r, gi, gi);
    st->d[j] = dot(r, gj, gj);
    if (st->V) {
        double *vi = st->V + (size_t)ci * r;
        double *vj = st->V + (size_t)cj * r;
        for (int q = 0; q < r; ++q) {
            double x = vi[q], y = vj[q];
            vi[q] = fma(ht, y, x) * c;
            vj[q] = fma(t, x, y) * c;
        }
    }
    acc->rot += 1;
    acc->code = orc_conv_code(acc->code, 1, t, st->tthresh);
}

int orc_hsvd(int n, int p, const double *G, int ldg, const orc_params *prm,
             double *sigma, double *U, double *V, double *lambda, int *perm,
             orc_info *info)
{
    if (n < 1 || p < 0 || p > n || ldg < n || !G || !prm || !sigma) return ORC_E_INVAL;
    if (!(prm->tol > 0.0) || !(prm->tthresh >= 0.0) || prm->max_sweeps < 0) return ORC_E_INVAL;
    if (prm->block < 0 || prm->ordering < 0 || prm->ordering > 1) return ORC_E_INVAL;
    for (int c = 0; c < n; ++c)
        for (int q = 0; q < n; ++q)
            if (!isfinite(G[(size_t)c * ldg + q])) return ORC_E_INVAL;

#ifdef _OPENMP
    if (prm->nthreads > 0) omp_set_num_threads(prm->nthreads);
#endif
    const int b = prm->block;
    const int r = orc_bordered_order(n, b);

    /* Working copies, bordered by unit columns (eq. 4.1). */
    double *Gw = (double *)calloc((size_t)r * r, sizeof(double));
    double *Vw = prm->want_v ? (double *)calloc((size_t)r * r, sizeof(double)) : NULL;
    double *d = (double *)malloc(sizeof(double) * (size_t)r);
    int *rho = (int *)malloc(sizeof(int) * (size_t)r);
    for (int c = 0; c < n; ++c) memcpy(Gw + (size_t)c * r, G + (size_t)c * ldg, sizeof(double) * n);
    for (int c = n; c < r; ++c) Gw[(size_t)c * r + c] = 1.0;
    if (Vw)
        for (int c = 0; c < r; ++c) Vw[(size_t)c * r + c] = 1.0;

    /* Alg. 4.2: d = diag(G^T G), rho = id, j = diag(I_p, -I_{r-p}). */
    int status = ORC_OK;
    for (int c = 0; c < r; ++c) {
        d[c] = dot(r, Gw + (size_t)c * r, Gw + (size_t)c * r);
        rho[c] = c;
        if (!(d[c] > 0.0)) status = ORC_E_RANK;
    }

    const int outer_r = b > 0 ? r / b : r;
    const int S = orc_steps_per_sweep(prm->ordering, outer_r);
    int *mm_state = (int *)malloc(sizeof(int) * (size_t)(2 * outer_r));
    int *outer = (int *)malloc(sizeof(int) * (size_t)outer_r);
    int *pairs = NULL;
    int maxpairs = outer_r / 2;
    if (b > 0) maxpairs = (outer_r / 2) * b * (2 * b - 1);
    pairs = (int *)malloc(sizeof(int) * (size_t)(2 * maxpairs));
    orc_modmod_init(outer_r, mm_state);

    orc_state st = {r, p, Gw, Vw, d, rho, prm->tol, prm->tthresh};
    int sweeps = 0, code = 0;
    long rot = 0, skp = 0, steps = 0, inner = 0;
    int converged = 0, stopped = 0;

    if (status == ORC_OK) {
        if (prm->sort) orc_sort(r, p, d, rho);
        for (int sw = 0; sw < prm->max_sweeps && !stopped; ++sw) {
            code = 0;
            int rank = 0;
            for (int s = 0; s < S; ++s) {
                if (prm->ordering == ORC_MODMOD) orc_modmod_pairs(outer_r, mm_state, outer);
                else orc_roundrobin_pairs(outer_r, s, outer);
                int scode = 0, srank = 0;
                long srot = 0, sskp = 0;
                if (b == 0) {
                    int np = r / 2;
#pragma omp parallel for schedule(static) reduction(|:scode, srank) reduction(+:srot, sskp)
                    for (int k = 0; k < np; ++k) {
                        orc_acc acc = {0, 0, 0, 0};
                        pair_rotate(&st, outer[2 * k], outer[2 * k + 1], &acc);
                        scode |= acc.code; srank |= acc.rank;
                        srot += acc.rot; sskp += acc.skip;
                    }
                } else if (prm->inner_sweeps > 0) {
                    /* full-block: every pair of the 2b columns by the circle
                       method, repeated until an inner sweep rotates nothing */
                    int cnt = orc_block_step_pairs(r, b, outer, 0, pairs);
                    int per = cnt / (outer_r / 2);
                    int nbp = outer_r / 2;
                    long sinner = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(|:scode, srank) reduction(+:srot, sskp, sinner)
                    for (int k = 0; k < nbp; ++k) {
                        orc_acc acc = {0, 0, 0, 0};
                        for (int it = 0; it < prm->inner_sweeps; ++it) {
                            long before = acc.rot;
                            for (int q = 0; q < per; ++q) {
                                int *pq = pairs + 2 * ((size_t)k * per + q);
                                pair_rotate(&st, pq[0], pq[1], &acc);
                            }
                            ++sinner;
                            if (acc.rot == before) break;
                        }
                        scode |= acc.code; srank |= acc.rank;
                        srot += acc.rot; sskp += acc.skip;
                    }
                    inner += sinner;
                } else {
                    int cnt = orc_block_step_pairs(r, b, outer, s, pairs);
                    int per = cnt / (outer_r / 2);
                    int nbp = outer_r / 2;
#pragma omp parallel for schedule(dynamic, 1) reduction(|:scode, srank) reduction(+:srot, sskp)
                    for (int k = 0; k < nbp; ++k) {
                        orc_acc acc = {0, 0, 0, 0};
                        for (int q = 0; q < per; ++q) {
                            int *pq = pairs + 2 * ((size_t)k * per + q);
                            pair_rotate(&st, pq[0], pq[1], &acc);
                        }
                        scode |= acc.code; srank |= acc.rank;
                        srot += acc.rot; sskp += acc.skip;
                    }
                }
                code |= scode; rank |= srank; rot += srot; skp += sskp;
                if (prm->ordering == ORC_MODMOD) orc_modmod_advance(outer_r, mm_state);
                ++steps;
                if (prm->max_steps > 0 && steps >= prm->max_steps) { stopped = 1; break; }
            }
            if (prm->sort) orc_sort(r, p, d, rho);
            ++sweeps;
            if (rank) { status = ORC_E_RANK; break; }
            if (stopped) break;
            /* Stop when no rotation had |t| > T: code 00 (no rotation at all)
               or 01 (only small tangents), eq. (4.2). */
            if ((code & 2) == 0) { converged = 1; break; }
        }
        if (status == ORC_OK && !converged) status = ORC_E_NOCONV;
    }

    /* Sigma, U = G Sigma^{-1}, lambda = Sigma^2 J, in physical column order;
       perm lists physical columns by sorted position (border columns dropped). */
    int m = 0;
    for (int q = 0; q < r; ++q) {
        int c = rho[q];
        if (c >= n) continue;
        double s = sqrt(d[q]);
        sigma[c] = s;
        if (lambda) lambda[c] = (q < p) ? d[q] : -d[q];
        if (perm) perm[m] = c;
        ++m;
        if (U)
            for (int row = 0; row < n; ++row) U[(size_t)c * n + row] = Gw[(size_t)c * r + row] / s;
    }
    if (V && Vw)
        for (int c = 0; c < n; ++c) memcpy(V + (size_t)c * n, Vw + (size_t)c * r, sizeof(double) * n);

    if (info) {
        info->sweeps = sweeps;
        info->code = code;
        info->rotations = rot;
        info->skips = skp;
        info->steps = steps;
        info->r = r;
        info->inner = inner;
    }
    free(Gw); free(Vw); free(d); free(rho); free(mm_state); free(outer); free(pairs);
    return status;
}
