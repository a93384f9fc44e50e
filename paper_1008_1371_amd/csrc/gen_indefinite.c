/* Seeded symmetric indefinite test matrices with a prescribed spectrum, as
 * the paper builds its test inputs (Sec. 5): M = Q diag(lam) Q^T with Q a
 * product of Householder reflectors, then the symmetric indefinite
 * factorisation with complete pivoting of Bunch and Parlett,
 * M = P L D L^T P^T, both carried out in x87 extended precision (long
 * double, 64-bit significand).  Each 2 x 2 pivot block of D is diagonalised
 * by a symmetric Schur rotation, which gives M = G J G^T with J = diag(+-1),
 * and G is rounded to double.
 *
 * This is workload generation (the step before the HSVD): none of the HSVD
 * method's arithmetic is here.  Host C, OpenMP over columns; the random
 * numbers come in from the caller.  Reductions that pick a pivot combine the
 * per-thread candidates in a fixed order, so the result does not depend on
 * the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double xr;

/* A = Q diag(lam) Q^T, Q = H_0 H_1 ... H_{n-2}; H_i = I - 2 w w^T acts on
 * indices i..n-1 with w the normalised vec[i*n + i .. i*n + n-1].  Applied
 * innermost first, so each two-sided application touches only the trailing
 * block A[i:, i:] (the leading part is still diagonal).  Full symmetric
 * storage, column-major. */
static void form_matrix(int n, const double *lam, const double *vec, xr *A, xr *w, xr *y, int nt)
{
    memset(A, 0, sizeof(xr) * (size_t)n * n);
    for (int i = 0; i < n; ++i) A[(size_t)i * n + i] = lam[i];
    for (int i = n - 2; i >= 0; --i) {
        const int m = n - i;
        const double *v = vec + (size_t)i * n + i;
        xr s = 0.0L;
        for (int k = 0; k < m; ++k) {
            w[k] = v[k];
            s += w[k] * w[k];
        }
        if (s == 0.0L) continue;
        s = sqrtl(s);
        for (int k = 0; k < m; ++k) w[k] /= s;
        /* y = A_t w */
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int j = 0; j < m; ++j) {
            const xr *col = A + (size_t)(i + j) * n + i;
            xr t = 0.0L;
            for (int k = 0; k < m; ++k) t += col[k] * w[k];
            y[j] = t;
        }
        /* H A_t H = A_t - 2 (w z^T + z w^T), z = y - (w^T y) w */
        xr wy = 0.0L;
        for (int j = 0; j < m; ++j) wy += w[j] * y[j];
        for (int j = 0; j < m; ++j) y[j] -= wy * w[j];
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int j = 0; j < m; ++j) {
            xr *col = A + (size_t)(i + j) * n + i;
            const xr wj = 2.0L * w[j], zj = 2.0L * y[j];
            for (int k = 0; k < m; ++k) col[k] -= w[k] * zj + y[k] * wj;
        }
    }
}

/* Symmetric interchange of indices a and b of the trailing matrix: rows in
 * every column (this also permutes the rows of the computed columns of L),
 * then columns. */
static void swap_sym(int n, xr *A, int *perm, int a, int b)
{
    if (a == b) return;
    for (int j = 0; j < n; ++j) {
        xr *c = A + (size_t)j * n;
        const xr t = c[a];
        c[a] = c[b];
        c[b] = t;
    }
    xr *ca = A + (size_t)a * n, *cb = A + (size_t)b * n;
    for (int i = 0; i < n; ++i) {
        const xr t = ca[i];
        ca[i] = cb[i];
        cb[i] = t;
    }
    const int t = perm[a];
    perm[a] = perm[b];
    perm[b] = t;
}

typedef struct {
    xr v;
    int i, j;
} cand;

/* a before b: larger value, then smaller column, then smaller row */
static int better(const cand *a, const cand *b)
{
    if (a->v != b->v) return a->v > b->v;
    if (a->j != b->j) return a->j < b->j;
    return a->i < b->i;
}

/* Largest |a_ij| over i >= j >= k and largest |a_ii| over i >= k. */
static void find_pivots(int n, const xr *A, int k, cand *off, cand *dia, cand *scratch, int nt)
{
    for (int t = 0; t < 2 * nt; ++t) scratch[t] = (cand){-1.0L, n, n};
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cand bo = {-1.0L, n, n}, bd = {-1.0L, n, n};
#pragma omp for schedule(static)
        for (int j = k; j < n; ++j) {
            const xr *c = A + (size_t)j * n;
            const cand d = {fabsl(c[j]), j, j};
            if (better(&d, &bd)) bd = d;
            for (int i = j; i < n; ++i) {
                const xr v = fabsl(c[i]);
                if (v > bo.v) bo = (cand){v, i, j};
            }
        }
        scratch[2 * tid] = bo;
        scratch[2 * tid + 1] = bd;
    }
    *off = scratch[0];
    *dia = scratch[1];
    for (int t = 1; t < nt; ++t) {
        if (better(&scratch[2 * t], off)) *off = scratch[2 * t];
        if (better(&scratch[2 * t + 1], dia)) *dia = scratch[2 * t + 1];
    }
}

/* Bunch-Parlett: Pi M Pi^T = L D L^T in place (L below the diagonal of the
 * pivot columns, D's blocks on the diagonal); bsz[k] = 1 or 2 at the start of
 * each pivot block, 0 for the second index of a 2 x 2 block.  Returns 0, or
 * -1 when the trailing matrix is zero (M singular). */
static int bunch_parlett(int n, xr *A, int *perm, int *bsz, int nt)
{
    const xr alpha = (1.0L + sqrtl(17.0L)) / 8.0L;
    cand *scratch = (cand *)malloc(sizeof(cand) * 2 * (size_t)nt);
    if (!scratch) return -2;
    for (int i = 0; i < n; ++i) perm[i] = i;
    int k = 0;
    while (k < n) {
        cand off, dia;
        find_pivots(n, A, k, &off, &dia, scratch, nt);
        if (off.v <= 0.0L) {
            free(scratch);
            return -1;
        }
        if (dia.v >= alpha * off.v || k == n - 1) {
            swap_sym(n, A, perm, k, dia.i);
            xr *lk = A + (size_t)k * n;
            const xr d = lk[k];
            for (int i = k + 1; i < n; ++i) lk[i] /= d;
#pragma omp parallel for schedule(static) num_threads(nt)
            for (int j = k + 1; j < n; ++j) {
                xr *cj = A + (size_t)j * n;
                const xr f = cj[k];  /* a_jk before the division (row k copy) */
                for (int i = k + 1; i < n; ++i) cj[i] -= lk[i] * f;
            }
            bsz[k] = 1;
            k += 1;
        } else {
            /* 2 x 2 pivot on (off.j, off.i), off.j < off.i */
            const int s = off.j, r = off.i;
            swap_sym(n, A, perm, k, s);
            swap_sym(n, A, perm, k + 1, r == k ? s : r);
            xr *l0 = A + (size_t)k * n, *l1 = A + (size_t)(k + 1) * n;
            const xr e11 = l0[k], e21 = l0[k + 1], e22 = l1[k + 1];
            const xr det = e11 * e22 - e21 * e21;
            for (int i = k + 2; i < n; ++i) {
                const xr a0 = l0[i], a1 = l1[i];
                l0[i] = (a0 * e22 - a1 * e21) / det;
                l1[i] = (a1 * e11 - a0 * e21) / det;
            }
#pragma omp parallel for schedule(static) num_threads(nt)
            for (int j = k + 2; j < n; ++j) {
                xr *cj = A + (size_t)j * n;
                const xr f0 = cj[k], f1 = cj[k + 1];
                for (int i = k + 2; i < n; ++i) cj[i] -= l0[i] * f0 + l1[i] * f1;
            }
            bsz[k] = 2;
            bsz[k + 1] = 0;
            k += 2;
        }
    }
    free(scratch);
    return 0;
}

/* G (n x n, column-major, leading dimension n) and jsig such that
 * M = G diag(jsig) G^T for M = Q diag(lam) Q^T (see form_matrix), and the
 * block counts.  lam: n doubles; vec: n x n doubles (the reflector of index i
 * is vec[i*n + i .. i*n + n-1]); nthreads <= 0 uses the OpenMP default.
 * Returns 0; -1 if M is singular; -2 on allocation failure. */
int hsvd_gen_indefinite(int n, const double *lam, const double *vec, int nthreads, double *G,
                        signed char *jsig, int *n2x2)
{
    int nt = nthreads;
#ifdef _OPENMP
    if (nt <= 0) nt = omp_get_max_threads();
#else
    nt = 1;
#endif
    if (nt < 1) nt = 1;
    xr *A = (xr *)malloc(sizeof(xr) * (size_t)n * n);
    xr *w = (xr *)malloc(sizeof(xr) * (size_t)n);
    xr *y = (xr *)malloc(sizeof(xr) * (size_t)n);
    int *perm = (int *)malloc(sizeof(int) * (size_t)n);
    int *bsz = (int *)malloc(sizeof(int) * (size_t)n);
    if (!A || !w || !y || !perm || !bsz) {
        free(A), free(w), free(y), free(perm), free(bsz);
        return -2;
    }
    form_matrix(n, lam, vec, A, w, y, nt);
    const int st = bunch_parlett(n, A, perm, bsz, nt);
    if (st == 0) {
        int blocks2 = 0;
        memset(G, 0, sizeof(double) * (size_t)n * n);
        for (int k = 0; k < n; ++k) {
            if (bsz[k] == 1) {
                const xr *lk = A + (size_t)k * n;
                const xr d = lk[k];
                const xr sc = sqrtl(fabsl(d));
                double *g = G + (size_t)k * n;
                g[perm[k]] = (double)sc;
                for (int i = k + 1; i < n; ++i) g[perm[i]] = (double)(lk[i] * sc);
                jsig[k] = d > 0.0L ? 1 : -1;
            } else if (bsz[k] == 2) {
                /* E = Z diag(mu1, mu2) Z^T, Z = [c s; -s c] (symmetric Schur) */
                const xr *l0 = A + (size_t)k * n, *l1 = A + (size_t)(k + 1) * n;
                const xr e11 = l0[k], e21 = l0[k + 1], e22 = l1[k + 1];
                const xr tau = (e22 - e11) / (2.0L * e21);
                const xr t = (tau >= 0.0L ? 1.0L : -1.0L) / (fabsl(tau) + sqrtl(1.0L + tau * tau));
                const xr c = 1.0L / sqrtl(1.0L + t * t), s = t * c;
                const xr mu1 = e11 - t * e21, mu2 = e22 + t * e21;
                const xr s1 = sqrtl(fabsl(mu1)), s2 = sqrtl(fabsl(mu2));
                double *g0 = G + (size_t)k * n, *g1 = G + (size_t)(k + 1) * n;
                /* columns (c L0 - s L1) s1 and (s L0 + c L1) s2, L0 = e_k + l0,
                 * L1 = e_{k+1} + l1 below the block */
                g0[perm[k]] = (double)(c * s1);
                g0[perm[k + 1]] = (double)(-s * s1);
                g1[perm[k]] = (double)(s * s2);
                g1[perm[k + 1]] = (double)(c * s2);
                for (int i = k + 2; i < n; ++i) {
                    g0[perm[i]] = (double)((c * l0[i] - s * l1[i]) * s1);
                    g1[perm[i]] = (double)((s * l0[i] + c * l1[i]) * s2);
                }
                jsig[k] = mu1 > 0.0L ? 1 : -1;
                jsig[k + 1] = mu2 > 0.0L ? 1 : -1;
                ++blocks2;
            }
        }
        if (n2x2) *n2x2 = blocks2;
    }
    free(A), free(w), free(y), free(perm), free(bsz);
    return st;
}
