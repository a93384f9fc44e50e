// Internal declarations of libhsvd: context, workspace layout, device helpers.
//
// Every floating point expression in the library is compiled with
// -ffp-contract=off: an FMA appears only where fma() is written.  The rotation
// parameter routine therefore rounds every operation separately, in the order
// written, with correctly rounded division and square root.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/hsvd.h"

namespace hsvd {

constexpr int kMaxOrder = 16384;   // largest bordered order r

// Per-solve control block in device memory; copied to pinned host memory once per sweep.
struct Ctl {
    int code;          // OR of the eq. (4.2) codes of the sweep just reduced
    int rank;          // set when a pair is numerically rank deficient
    int inval;         // set when the input holds a non-finite value
    int pad;
    unsigned long long rot;    // rotations, cumulative
    unsigned long long skip;   // skipped pair visits, cumulative
    unsigned long long act;    // block pair steps with a rotation, cumulative
    unsigned long long tcol;   // columns touched by a rotation, summed over block pair steps, cumulative
    double maxt;               // largest |t| of the sweep just reduced
    double nsres;              // Newton-Schulz residual max |J X^T J X - I| (mixed path)
};

// Control block of the persistent pairwise kernel (device memory, zeroed
// before its launch).
struct PersistCtl {
    unsigned int count;  // grid barrier: arrivals at the current barrier
    unsigned int gen;    // grid barrier: completed barriers
    int err;             // a wait passed its time limit: every workgroup leaves
    int stop;            // set at a sweep's end: 1 converged (eq. 4.2), 2 rank deficient
    int sweeps;          // sweeps completed
    int pad[3];
};

struct Workspace {
    double *G = nullptr;      // ldg x r, working copy of G (bordered, zero-padded rows)
    double *V = nullptr;      // ldg x r, accumulated V^{-T}
    double *d = nullptr;      // r: kept diagonal, by position
    int *rho = nullptr;       // r: physical column at each position
    double *dtmp = nullptr;   // r: sort scratch
    int *rtmp = nullptr;      // 2r: sort scratch (moved rho, ranks)
    int4 *S = nullptr;        // r/2: modified modulus stepper state per slot (ip, jp, iblk, jblk)
    int *C = nullptr;         // r/2: per-slot convergence code of the current sweep (eq. 4.2)
    unsigned int *nrot = nullptr;   // r/2: per-slot rotations in the current sweep
    unsigned int *nskip = nullptr;  // r/2: per-slot skips in the current sweep
    unsigned int *nact = nullptr;   // r/2: per-slot steps with at least one rotation (block path)
    unsigned int *ntc = nullptr;    // r/2: per-slot columns touched by rotations, summed over steps (block path)
    double *maxt = nullptr;         // r/2: per-slot largest |t| of the current sweep
    Ctl *ctl = nullptr;
    unsigned int *ver = nullptr;  // r: completed visits per position (persistent pairwise kernel)
    PersistCtl *pctl = nullptr;
    // block path
    double *P = nullptr;      // pairs x splits x (2b)^2 partial Gram matrices
    double *W = nullptr;      // pairs x (2b)^2 accumulated inner transformations
    unsigned long long *active = nullptr;  // pairs: mask of the 2b local columns W changes (0: W = I)
    int4 *S2 = nullptr;       // 2 x pairs: outer stepper state, double-buffered across steps
    // mixed path
    float *G32 = nullptr, *V32 = nullptr, *P32 = nullptr, *W32 = nullptr;
    double *T1 = nullptr, *T2 = nullptr;  // ldg x r FP64 scratch of the J-re-orthogonalisation
    // wide block path (b = 64): second working copies (column moves after a
    // sort), block pairs of the step, position payload of the sort, moved rho,
    // per-pair rotation flags
    double *G2 = nullptr, *V2 = nullptr;
    int2 *blk = nullptr;
    int *pl = nullptr, *rho2 = nullptr, *wact = nullptr;
};

struct Layout {
    int n = 0, r = 0, ldg = 0, pairs = 0, splits = 0, b2 = 0;
    size_t bytes = 0;
    size_t off_G, off_V, off_d, off_rho, off_dtmp, off_rtmp, off_S, off_C, off_nrot, off_nskip,
        off_nact, off_ntc, off_maxt, off_ctl, off_ver, off_pctl, off_P, off_W, off_active, off_S2, off_G32, off_V32, off_P32, off_W32,
        off_T1, off_T2, off_G2, off_V2, off_blk, off_pl, off_rho2, off_wact;
    bool mixed = false, wide = false;
};

// pairs/splits/b2 > 0 adds the block path buffers, mixed the FP32 copies and
// the FP64 scratch of the mixed path.
Layout make_layout(int n, int r, int ldg, bool want_v, int pairs = 0, int splits = 0, int b2 = 0,
                   bool mixed = false);
Workspace carve(void *base, const Layout &L);

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Rotation parameters (Sec. 2): the angle annihilates a_ij under the column
// updates (2.4) trig / (2.5) hyperbolic, i.e.
//   tan 2phi = 2 a_ij / (a_jj - a_ii),   tanh 2phi = -2 a_ij / (a_ii + a_jj).
// zeta = 1 / tan(h) 2phi; t is the root of smaller magnitude of
// t^2 + 2 zeta t - 1 = 0 (trig) or t^2 - 2 zeta t + 1 = 0 (hyperbolic);
// c = 1/sqrt(1 + t^2) or 1/sqrt((1 - t)(1 + t)).  sgn(0) = +1; for
// |zeta| > 2^500, t = 0.5 / zeta.  Returns 1 (rank failure) for a hyperbolic
// pair with |zeta| <= 1.
__device__ __forceinline__ int rotation_params(double aii, double ajj, double aij, int hyp,
                                               double &t, double &c)
{
    // Both cases run the same instruction stream (selects instead of branches,
    // so a wavefront holding both kinds of pair does not serialise); each case
    // still rounds exactly the operations listed above, in that order: the
    // trigonometric root is sqrt(1 + zeta^2) * 1, the hyperbolic one
    // sqrt(|zeta| - 1) * sqrt(|zeta| + 1).
    const double big = 0x1p500;
    const bool trig = hyp < 0;
    const double two_aij = 2.0 * aij;
    const double num = trig ? (ajj - aii) : -(aii + ajj);
    const double zeta = num / two_aij;
    const double az = fabs(zeta);
    const double sg = zeta < 0.0 ? -1.0 : 1.0;
    const double r1 = sqrt(trig ? 1.0 + zeta * zeta : az - 1.0);
    const double r2 = trig ? 1.0 : sqrt(az + 1.0);
    const double root = r1 * r2;
    double tt = az > big ? 0.5 / zeta : sg / (az + root);
    const double cin = trig ? 1.0 + tt * tt : (1.0 - tt) * (1.0 + tt);
    double cc = 1.0 / sqrt(cin);
    const int bad = (!trig && !(az > 1.0)) ? 1 : 0;
    if (bad) {
        tt = 0.0;
        cc = 1.0;
    }
    t = tt;
    c = cc;
    return bad;
}

// Reciprocal and reciprocal square root from the hardware estimates refined by
// two Newton steps each (the estimate's relative error e becomes ~e^4, far below
// one ulp); results within about one ulp, not correctly rounded.
__device__ __forceinline__ double rcp_nr(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-(h * y), y, 0.5);
    y = fma(y, e, y);
    e = fma(-(h * y), y, 0.5);
    return fma(y, e, y);
}

// The same rotation as rotation_params with a shorter dependency chain, for
// the latency-bound inner solves of the block path.  With d = a_jj - a_ii,
// w = 2 a_ij and S = a_ii + a_jj the smaller-magnitude roots are
//   trig: t = sgn(d) w / (|d| + sqrt(d^2 + w^2)),          c = (1 + t^2)^(-1/2)
//   hyp:  t = -w / (S + sqrt((S - |w|)(S + |w|))),          c = (1 - t^2)^(-1/2)
// (one square root, one reciprocal and one reciprocal square root instead of
// three divisions and two or three square roots), rank failure iff S <= |w|.
// Both cases run as one select-driven sequence, q = X Y + Z with (X, Y, Z) =
// (|d|, |d|, w^2) or (S - |w|, S + |w|, 0), so a wave holding pairs of both
// kinds issues it once.  Results agree with rotation_params to within a few
// ulps; for d = 0 the trig case takes t = sgn(a_ij) (both signs annihilate
// a_ij).  Entries outside [2^-480, 2^480], where the squares could leave the
// exponent range, use rotation_params.
__device__ __forceinline__ bool fast_range(double aii, double ajj)
{
    const double lo = 0x1p-480, hi = 0x1p480;
    return aii >= lo && aii <= hi && ajj >= lo && ajj <= hi;
}

__device__ __forceinline__ int rotation_params_fast(double aii, double ajj, double aij, int hyp, double &t,
                                                    double &c)
{
    if (!fast_range(aii, ajj)) return rotation_params(aii, ajj, aij, hyp, t, c);
    const bool trig = hyp < 0;
    const double w = 2.0 * aij, aw = fabs(w);
    const double d = ajj - aii, S = aii + ajj;
    const double m = S - aw;
    const double X = trig ? fabs(d) : m, Y = trig ? fabs(d) : S + aw, Z = trig ? w * w : 0.0;
    const double q = fma(X, Y, Z);
    const double s = q * rsq_nr(q);
    const double num = (trig && !(d < 0.0)) ? w : -w;
    const double tt = num * rcp_nr((trig ? fabs(d) : S) + s);
    const double cc = rsq_nr(fma(trig ? tt : -tt, tt, 1.0));
    const int bad = (!trig && !(m > 0.0)) ? 1 : 0;
    t = bad ? 0.0 : tt;
    c = bad ? 1.0 : cc;
    return bad;
}

// Relative orthogonality, eq. (2.3), strict: |a_ij| < tol sqrt(a_ii) sqrt(a_jj).
__device__ __forceinline__ bool rel_orthogonal(double aii, double ajj, double aij, double tol)
{
    return fabs(aij) < tol * (sqrt(aii) * sqrt(ajj));
}

// The same test squared, a_ij^2 < tol^2 a_ii a_jj (tol2 = tol^2), for the
// block path: no square roots; equal to rel_orthogonal up to rounding at the
// threshold itself.  Where the right-hand side is not a normal number (tiny
// entries or tolerance) or the entries leave [2^-480, 2^480], rel_orthogonal
// decides.
__device__ __forceinline__ bool rel_orthogonal_sq(double aii, double ajj, double aij, double tol, double tol2)
{
    const double rhs = tol2 * (aii * ajj);
    if (!fast_range(aii, ajj) || !(rhs >= 0x1p-1000)) return rel_orthogonal(aii, ajj, aij, tol);
    return aij * aij < rhs;
}

// Sort key of a diagonal entry: the IEEE-754 total order of its bit pattern,
// as a signed integer.  On the non-negative values of d (sums of squares,
// never -0) it orders exactly as the values; on any input, NaN included, it
// is a total order, so the ranks of the sort always form a permutation and
// rho stays one.
__device__ __forceinline__ long long sort_key(double x)
{
    const long long k = __double_as_longlong(x);
    return k < 0 ? (k ^ 0x7fffffffffffffffLL) : k;
}

// Eq. (4.2) code of one applied rotation, to be OR-ed into the slot's code.
__device__ __forceinline__ int rotation_code(double t, double tthresh)
{
    return fabs(t) > tthresh ? 3 : 1;
}

// Modified modulus strategy: state (ip, jp, iblk, jblk) of one slot.
// Start on the antidiagonal, slot k -> (k, r-1-k) (Alg. 4.3).
__host__ __device__ __forceinline__ int4 modmod_start(int k, int r)
{
    return make_int4(k, r - 1 - k, k, r - 1 - k);
}

// Transition (Alg. 4.4) with the test read as ip + jp >= r - 1.
__host__ __device__ __forceinline__ int4 modmod_next(int4 s, int r)
{
    if (s.x + s.y >= r - 1) {
        s.x += 1;
        if (s.x == s.y) {
            s.x -= r / 2;
            s.y = s.x;
        }
        s.z = s.x;
    } else {
        s.y += 1;
        s.w = s.y;
    }
    return s;
}

// Round-robin circle method: arrangement A_s[0] = 0,
// A_s[m] = 1 + ((m - 1 + s) mod (r - 1)); slot k pairs A_s[k] with A_s[r-1-k].
__host__ __device__ __forceinline__ int2 roundrobin_pair(int k, int r, int s)
{
    const int a = (k == 0) ? 0 : 1 + ((k - 1 + s) % (r - 1));
    const int b = 1 + ((r - 2 - k + s) % (r - 1));
    return a < b ? make_int2(a, b) : make_int2(b, a);
}

// Inner ordering of a block pair, local indices x < y in [0, 2b), slot q < b,
// inner step u: first outer step of a sweep -> circle method over 2b indices
// (2b - 1 inner steps); otherwise the cross pair (q, b + ((q + u) mod b)).
__host__ __device__ __forceinline__ int2 block_inner_pair(int q, int u, bool first, int b)
{
    if (first) return roundrobin_pair(q, 2 * b, u);
    return make_int2(q, b + ((q + u) % b));
}

// Sum over a 64-lane wavefront by an xor butterfly; every lane ends with the
// same bits (each stage adds the same two operands, in either order).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sum over a workgroup of WG threads; all threads return the same bits.
// `sh` holds WG/64 doubles.
template <int WG>
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    if (WG == 64) return v;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
#pragma unroll
    for (int q = 1; q < WG / 64; ++q) s += sh[q];
    __syncthreads();
    return s;
}

template <int WG>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *sh)
{
    a = wave_sum(a);
    b = wave_sum(b);
    if (WG == 64) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[2 * w] = a;
        sh[2 * w + 1] = b;
    }
    __syncthreads();
    double sa = sh[0], sb = sh[1];
#pragma unroll
    for (int q = 1; q < WG / 64; ++q) {
        sa += sh[2 * q];
        sb += sh[2 * q + 1];
    }
    __syncthreads();
    a = sa;
    b = sb;
}

// ---------------------------------------------------------------------------
// Kernel launchers (pairwise path), all on `st`.
// ---------------------------------------------------------------------------
struct StepArgs {
    double *G;
    double *V;       // nullptr: no V accumulation
    int ldg, r, p;
    double *d;
    const int *rho;
    int4 *S;
    int *C;
    unsigned int *nrot, *nskip;
    double *maxt;
    Ctl *ctl;
    int ordering;    // HSVD_ORD_MODMOD / HSVD_ORD_ROUNDROBIN
    int step;        // step index inside the sweep (round-robin)
    double tol, tthresh;
};

// The persistent pairwise kernel: every sweep of a solve in one cooperative
// launch.  Steps are separated either by a grid barrier or, per column, by
// the completed-visit counts in ver (a pair waits only for the two pairs that
// last held its columns); at a sweep's end a grid barrier, the sort and the
// convergence test (eq. 4.2) run on the device.
struct PairPersistArgs {
    StepArgs a;
    int steps;        // steps per sweep
    int max_sweeps;
    int sort;         // sort the diagonal after every sweep
    int dataflow;     // 1: per-column readiness between steps; 0: a grid barrier
    double *dtmp;     // r: sort scratch
    int *rtmp;        // 2r: sort scratch (moved rho, then ranks)
    unsigned int *nact, *ntc;  // per-slot counters the reduction resets
    unsigned int *ver;
    PersistCtl *pc;
    long long spin_limit;  // wall-clock ticks one wait may take before the launch gives up
};

template <typename T>
struct BlockArgsT {
    T *G;
    T *V;                    // nullptr: no V accumulation
    int ldg, r, p, nb;
    const int *rho;
    const int4 *S_in;        // outer stepper state of this step
    int4 *S_out;             // state of the next step (written by the update kernel)
    int ordering, step;      // step: outer step index inside the sweep
    int inner_sweeps = 0;    // 0: block-oriented; k > 0: full-block, at most k inner sweeps per pivot block
    // Update kernel: blockIdx.y + tile0 is the tile (G tiles first, then V's).
    int tile0 = 0;
    // Inner kernels of a single problem: vprev_wgs extra workgroups apply the
    // previous outer step's W (W_prev, active_prev, its outer pairs from S_prev
    // or step_prev) to V.
    int vprev_wgs = 0;
    int vrows = 0;           // rows of V per V-update workgroup
    T *W_prev = nullptr;
    unsigned long long *active_prev = nullptr;
    const int4 *S_prev = nullptr;
    int step_prev = 0;
    T *partial;
    int splits, rows_per_split;
    T *W;
    unsigned long long *active;  // per pair: mask of the 2b local columns W changes (0: W = I)
    int *C;
    unsigned int *nrot, *nskip, *nact, *ntc;
    double *maxt;            // per slot: largest |t| of the sweep
    Ctl *ctl;
    double tol, tthresh;
    // Batched solves: problem z = blockIdx.z of a group of problems with the
    // same bordered order r.  Per-problem arrays are laid out back to back
    // (G and V every ldg * r elements, rho every r, slots every nb / 2, partial
    // Grams and W per pair); pvec / tolvec / tthvec give each problem's p and
    // tolerances and done[z] != 0 skips a problem that has converged.
    int nprob = 1;
    const int *done = nullptr;
    const int *pvec = nullptr;
    const double *tolvec = nullptr, *tthvec = nullptr;
};
typedef BlockArgsT<double> BlockArgs;

int block_width();
hipError_t launch_block_stepper_init(hipStream_t st, int4 *S, int nb);
template <typename T>
hipError_t launch_block_gram(hipStream_t st, const BlockArgsT<T> &a);
template <typename T>
hipError_t launch_block_inner(hipStream_t st, const BlockArgsT<T> &a);
// Which tiles an update launch covers.
enum { UPD_BOTH = 0, UPD_G = 1, UPD_V = 2 };
template <typename T>
hipError_t launch_block_update(hipStream_t st, const BlockArgsT<T> &a, int which = UPD_BOTH);
// Rows per workgroup and workgroups that the V update of one outer step takes
// inside an inner launch (cus: compute units of the device).
int v_update_role_rows(int pairs, int ldg, int cus, bool fp64);
int v_update_role_wgs(int pairs, int ldg, int vrows);
template <typename T>
hipError_t launch_colnorm_pos(hipStream_t st, const T *G, int ldg, const int *rho, double *d, int r);
hipError_t launch_block_trace(hipStream_t st, int ordering, int r, int b, int step, int4 *S, int *out,
                              bool advance);

hipError_t launch_setup(hipStream_t st, const double *G, int lda, int n, const Workspace &w,
                        int r, int ldg, bool want_v);
hipError_t launch_precompute(hipStream_t st, const Workspace &w, int r, int ldg);
hipError_t launch_pair_step(hipStream_t st, const StepArgs &a);
hipError_t launch_sort(hipStream_t st, double *d, int *rho, double *dtmp, int *rtmp, int r, int p);
hipError_t launch_sweep_reduce(hipStream_t st, const Workspace &w, int slots);
// Cooperative launch of the persistent pairwise kernel; *grid receives the
// workgroup count (at most one per slot, at most what the device holds at once).
hipError_t launch_pair_persist(hipStream_t st, const PairPersistArgs &a, int *grid);
hipError_t launch_finalize(hipStream_t st, const Workspace &w, int n, int r, int p, int ldg,
                           double *sigma, double *U, int ldu, double *V, int ldv, double *lambda,
                           int *perm);
hipError_t launch_pair_params(hipStream_t st, long long m, const double *aii, const double *ajj,
                              const double *aij, const int *hyp, double tol, double tthresh,
                              int *skip, double *t, double *c, int *status, int *code, bool fast);
hipError_t launch_pivot_trace(hipStream_t st, int ordering, int r, int steps, int *pairs);
hipError_t launch_zero_ctl(hipStream_t st, Ctl *ctl);

// Batched solves (one group of problems with a common bordered order r).
struct BatchGroup {
    int nprob, r, ldg, pairs, max_sweeps;
    const int *ids;            // group slot -> problem index
    const int *n, *p;          // per group slot
    const long long *off, *voff;
    const double *tol, *tth;
    int *done, *status, *sweeps;
    int *active_count;
    double *G, *V, *d, *dtmp;
    int *rho, *rtmp;
    int *C;
    unsigned int *nrot, *nskip, *nact, *ntc;
    double *maxt;
    Ctl *ctl;
    // set-up of a subset (the FP64 restart of mixed solves): the set-up
    // launches touch only the problems with only[z] != 0
    const int *only = nullptr;
};
hipError_t launch_batch_setup(hipStream_t st, const BatchGroup &g, const double *G, bool want_v);
hipError_t launch_batch_colnorm(hipStream_t st, const BatchGroup &g, bool init);
hipError_t launch_batch_sort(hipStream_t st, const BatchGroup &g);
hipError_t launch_batch_reduce_decide(hipStream_t st, const BatchGroup &g);
hipError_t launch_batch_finalize(hipStream_t st, const BatchGroup &g, double *sigma, double *U, double *V,
                                 double *lambda);

// Mixed precision over a group of a batched solve: FP32 sweeps on FP32 copies
// of G and V, each problem leaving them by the switch rule of a single mixed
// solve, then its V J-re-orthogonalised in FP64 and G1 = G X.
struct BatchMixed {
    float *G32, *V32;      // per problem ldg * r
    int *done32;           // FP32 phase over for the problem
    int *sweeps32;
    double *prev_maxt, *prev_frac;
    double *tol32, *tth32;
    double *T1, *T2;       // per problem ldg * r (FP64)
    int *apply;            // the Newton-Schulz correction of this iteration applies; after it, G1 = G X applies
    int *nsdone;
    double *nsprev;        // latest residual max |J X^T J X - I| (the final one once nsdone)
    int *nsiters;          // corrections applied
    int *restart;          // the problem starts again from G in FP64
    double accept = 0.0;   // accepted final residual (<= 0: 16384 n u)
};
hipError_t launch_batch_mixed_init(hipStream_t st, const BatchGroup &g, const BatchMixed &m);
hipError_t launch_batch_colnorm32(hipStream_t st, const BatchGroup &g, const BatchMixed &m);
hipError_t launch_batch_decide32(hipStream_t st, const BatchGroup &g, const BatchMixed &m);
hipError_t launch_batch_promote(hipStream_t st, const BatchGroup &g, const BatchMixed &m);
hipError_t launch_batch_ns_form(hipStream_t st, const BatchGroup &g, const BatchMixed &m);
// last: the iteration cap, every problem stops after this residual
hipError_t launch_batch_ns_decide(hipStream_t st, const BatchGroup &g, const BatchMixed &m, int iter, bool last);
hipError_t launch_batch_ns_accept(hipStream_t st, const BatchGroup &g, const BatchMixed &m);
// dst_z <- src_z (ldg x r) for the problems with flag[z] != 0 (invert: == 0)
hipError_t launch_batch_copy_if(hipStream_t st, const BatchGroup &g, const double *src, double *dst,
                                const int *flag, bool invert);

// Batched solves in one persistent launch (batch_persist.hip): FP64,
// block-oriented method, problems with n <= kPersistMaxOrder.  Workgroups
// take problems from a work queue (order[], counter *next) and solve each one
// completely; per-problem results go to status / sweeps / code / maxt / rot /
// skip / act, indexed by problem.  slots: one slot of persist_slot_bytes()
// per workgroup.
constexpr int kPersistMaxOrder = 256;
constexpr int kPersistDefaultThreads = 256;  // before the autotuner has chosen
struct PersistArgs {
    int batch = 0;
    const int *order = nullptr;  // problem indices, largest n first
    int *next = nullptr;         // work counter (zeroed by the launcher)
    const int *n = nullptr, *p = nullptr;
    const long long *off = nullptr, *voff = nullptr;
    const double *Gin = nullptr;
    double *sigma = nullptr, *U = nullptr, *V = nullptr, *lambda = nullptr;
    int want_v = 1, ordering = 0, sort = 1, max_sweeps = 100;
    double tol = 0.0, tthresh = 0.0;  // <= 0: 1e-15 n and sqrt(tol) / 2 per problem
    int *status = nullptr, *sweeps = nullptr, *code = nullptr;
    double *maxt = nullptr;
    unsigned long long *rot = nullptr, *skip = nullptr, *act = nullptr;
    // mixed precision (FP32 block sweeps, J-re-orthogonalisation, FP64
    // refinement, per problem): FP32 sweeps, Newton-Schulz corrections, final
    // residual, FP64 restart flag per problem
    int mixed = 0;
    double reorth_accept = 0.0;  // <= 0: 16384 n u
    int *sweeps32 = nullptr, *nsiters = nullptr, *restart = nullptr;
    double *nsres = nullptr;
    char *slots = nullptr;
};
size_t persist_slot_bytes();
// threads per workgroup: 256, 512 or 1024 (the block pair's inner solve and
// update spread over all of them); 0 for another count
int persist_blocks_per_cu(int threads);
hipError_t launch_batch_persist(hipStream_t st, const PersistArgs &pa, int threads, int workgroups);

// The wide block path (wide_kernels.hip): column blocks of kWideB = 64, FP64,
// working copies in position order.
constexpr int kWideB = 64;
struct WideArgs {
    const double *partial = nullptr;  // pairs x splits x 128 x 128, column-major (both triangles)
    int splits = 1;
    double *W = nullptr;              // pairs x 128 x 128, column-major
    const int2 *blk = nullptr;        // per pair: its blocks (I, J)
    int p = 0;
    double tol = 0.0, tthresh = 0.0;
    int first = 0;                    // first outer step of a sweep (circle inner ordering)
    int inner_sweeps = 0;             // full-block method: circle sweeps per outer step, at most
    int *active = nullptr;            // per pair: 1 when a rotation was applied (W != I)
    int *C = nullptr;
    unsigned int *nrot = nullptr, *nskip = nullptr, *nact = nullptr, *ntc = nullptr;
    double *maxt = nullptr;
    Ctl *ctl = nullptr;
};
hipError_t launch_wide_blk(hipStream_t st, int ordering, int nb, int step, const int4 *S_in, int4 *S_out,
                           int2 *blk);
hipError_t launch_wide_inner(hipStream_t st, const WideArgs &a, int pairs);
// gather: dst[:, q] = src[:, idx[q]] (and rho_out[q] = rho_in[idx[q]] when
// rho_out is set); scatter: dst[:, idx[q]] = src[:, q]; q < r
hipError_t launch_wide_move(hipStream_t st, const double *src, double *dst, int ldg, int r, const int *idx,
                            bool scatter, const int *rho_in, int *rho_out);
hipError_t launch_wide_iota(hipStream_t st, int *v, int r);

// mixed path helpers
hipError_t launch_to_fp32(hipStream_t st, const double *G, float *G32, float *V32, int ldg, int r);
hipError_t launch_promote(hipStream_t st, const float *X32, double *X, int ldg, int r);
hipError_t launch_ns_form(hipStream_t st, double *B, int p, int ldg, int r, Ctl *ctl);
hipError_t launch_copy(hipStream_t st, const double *src, double *dst, int ldg, int r);
hipError_t launch_synth(hipStream_t st, double *G, int n, unsigned long long seed);
// FP64 products of the J-re-orthogonalisation (gemm_kernels.hip):
// C = op(A) S B, column-major, C M x N, K the inner dimension; op(A) = A
// (A M x K) or A^T (A K x M); S = diag(+1 x p, -1 x (K - p)) on the rows of B
// when signed.  The symmetric form (op(A) = A^T, M = N) forms the upper
// tiles only and writes each to both triangles.  M and N multiples of 16, K
// of 16, leading dimensions and strides even.  Batched (nprob > 1): problem
// z = blockIdx.z at offsets z * (sa, sb, sc), p = pvec[z] when pvec is set,
// and with flag set only the problems with (flag[z] != 0) == want run.
//
// Block-pair form (the wide block path): with `blk` set, problem z belongs to
// block pair g = z / ksplit and to K split s = z % ksplit.  The operands named
// in `map` (1 = A, 2 = B, 4 = C) are not offset by z but address the columns
// of a position-ordered matrix through the pair's two blocks of bw columns:
// column c is column blk[g].x * bw + c for c < bw, blk[g].y * bw + c - bw
// otherwise (for A: its M index when transposed, its K index otherwise; for B
// and C: their N index).  A K split s reads rows [s K, (s + 1) K) of the
// transposed A and of B.  flag and pvec are then indexed by g.  In-place
// products (A and C the same matrix, N = its mapped width) are allowed: a
// workgroup reads all of its rows before it writes them.
struct GemmArgs {
    const double *A = nullptr, *B = nullptr;
    double *C = nullptr;
    int M = 0, N = 0, K = 0;
    int lda = 0, ldb = 0, ldc = 0;
    const int2 *blk = nullptr;
    int bw = 0, map = 0, ksplit = 1;
    long long sa = 0, sb = 0, sc = 0;
    int p = 0;
    const int *pvec = nullptr;
    const int *flag = nullptr;
    int want = 1;
};
hipError_t launch_gemm(hipStream_t st, const GemmArgs &g, int nprob, bool trans_a, bool signed_b, bool symmetric);

hipError_t launch_gather_cols(hipStream_t st, const double *G, int lda, const int *pi, double *Gp, int n);
hipError_t launch_scatter_outputs(hipStream_t st, const int *pi, int n, const double *sp, const double *Up,
                                  const double *Vp, const double *lp, const int *permp, double *sigma, double *U,
                                  int ldu, double *V, int ldv, double *lambda, int *perm);

}  // namespace hsvd
