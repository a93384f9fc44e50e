// Batched solves in one persistent launch.
//
// Each workgroup takes whole problems from a device work queue (problem
// indices ordered by n, largest first, so that the long solves start first
// and the short ones fill in at the end) and runs the complete block-oriented
// solve of each one on its own: set-up and bordering (eq. 4.1), the kept
// diagonal and the sort (Alg. 4.1), then sweeps of outer steps -- for every
// block pair the Gram on MFMA, the inner rotations (eqs. 2.2-2.5), the
// update of the pair's columns of G and V on MFMA -- each sweep closed by
// fresh column norms, the sort and the stop rule of eq. (4.2), decided in the
// workgroup; finally Sigma, U, lambda and V into the caller's packed outputs.
// No host round trip and no other launch happens between the first problem
// and the last.
//
// Several workgroups share a compute unit, so while one runs the
// latency-bound inner solve of its block pair the others keep the matrix
// cores busy with their Gram and update products.
//
// The building blocks are those of the per-launch kernels (block_device.h),
// called with the same arguments and the same thread counts as the grouped
// batched path (one row split, 256-thread inner solves and updates), and the
// set-up, norm, sort and stop-rule steps repeat its arithmetic in the same
// order: for the same problems the results are bit-identical to it.
//
// Mixed precision runs the whole mixed solve of a problem in its workgroup
// too: FP32 block sweeps on FP32 copies (the same building blocks with
// T = float) until the problem's own switch rule, the Newton-Schulz
// J-re-orthogonalisation of V on FP64 MFMA inside the workgroup, G1 = G X,
// then the FP64 sweeps (or, after a rank flag in FP32 or a residual above
// the accepted bound, the FP64 sweeps from G).
//
// Each workgroup works in a slot of device memory of its own (working copies
// of G and V, partial Grams, W, the kept diagonal, rho, stepper state and
// counters; FP32 copies and FP64 product scratch for mixed precision), sized
// for the largest order the kernel takes (n <= 256).
#include "block_device.h"
#include "gemm_device.h"

namespace hsvd {

namespace {

constexpr int kPMaxR = kPersistMaxOrder;       // largest bordered order
constexpr int kPMaxPairs = kPMaxR / kB2;        // block pairs per step at most
// The update re-reads W from LDS for every 16-row strip (the register-resident
// W of the per-launch FP64 update would take the registers that let two
// workgroups share a compute unit); the arithmetic is the same.
constexpr int kPUpdLd = kB2 + 8;                // LDS row stride of W in the update

// LDS of one workgroup: the phases of a problem run one after the other, so
// they share one area.
union PersistLds {
    CircleLds circle;
    CrossLds<double> cross;
    CrossLds<float> cross32;
    gemm::GemmLds gemm;
    double red[kGramRed];
    struct {
        double Wl[kB2 * kPUpdLd];
        int cols[kB2];
        int tl[kB2];
    } upd;
    struct {
        long long key[kPMaxR];
        double dv[kPMaxR];
        int val[kPMaxR];
    } sort;
    double colsum[4][kPMaxR];
};

// The workgroup's LDS and the block pair arguments of the problem it works
// on.  The phases below are separate (not inlined) functions that reach both
// by name: compiled as one function, the whole solve kept so many values live
// at once that it no longer fitted the registers of two workgroups per
// compute unit; as calls, each phase is allocated on its own.
__shared__ PersistLds g_lds;
// raw storage: the argument struct has default member initialisers
__shared__ __align__(16) unsigned char g_args[sizeof(BlockArgsT<double>)];

__shared__ __align__(16) unsigned char g_args32[sizeof(BlockArgsT<float>)];
__shared__ __align__(16) unsigned char g_gemm[sizeof(GemmArgs)];

__device__ __forceinline__ BlockArgsT<double> &pargs() { return *reinterpret_cast<BlockArgsT<double> *>(g_args); }
__device__ __forceinline__ BlockArgsT<float> &pargs32() { return *reinterpret_cast<BlockArgsT<float> *>(g_args32); }
__device__ __forceinline__ GemmArgs &pgemm() { return *reinterpret_cast<GemmArgs *>(g_gemm); }

// NT threads per workgroup (256, 512 or 1024): the inner solves and the
// update spread over all of them, the Gram runs on the first 256.
__device__ __noinline__ void phase_gram(int q) { gram_pair<double>(pargs(), q, 0, g_lds.red); }
template <int NT>
__device__ __noinline__ void phase_circle(int q)
{
    inner_circle_pair<double, NT>(pargs(), q, g_lds.circle);
}
template <int NT>
__device__ __noinline__ void phase_cross(int q)
{
    inner_cross_pair<double, NT>(pargs(), q, g_lds.cross);
}
// M: 0 = G, 1 = V
template <int NT>
__device__ __noinline__ void phase_update(int q, int M, unsigned long long mask)
{
    const BlockArgsT<double> &a = pargs();
    update_rows<double, NT, true, true, kPUpdLd>(a, q, M ? a.V : a.G, 0, a.ldg / 16, mask, g_lds.upd.Wl,
                                               g_lds.upd.cols, g_lds.upd.tl);
}

// The FP32 phases of a mixed solve: the same building blocks on the FP32
// working copies (the rotations still computed in FP64); the FP32 update
// re-reads W from LDS at the FP32 row stride of the per-launch update.
constexpr int kPUpdLd32 = kB2 + 16;
__device__ __noinline__ void phase_gram32(int q)
{
    gram_pair<float>(pargs32(), q, 0, reinterpret_cast<float *>(g_lds.red));
}
template <int NT>
__device__ __noinline__ void phase_circle32(int q)
{
    inner_circle_pair<float, NT>(pargs32(), q, g_lds.circle);
}
template <int NT>
__device__ __noinline__ void phase_cross32(int q)
{
    inner_cross_pair<float, NT>(pargs32(), q, g_lds.cross32);
}
template <int NT>
__device__ __noinline__ void phase_update32(int q, int M, unsigned long long mask)
{
    const BlockArgsT<float> &a = pargs32();
    update_rows<float, NT, true, true, kPUpdLd32>(a, q, M ? a.V : a.G, 0, a.ldg / 16, mask,
                                                reinterpret_cast<float *>(g_lds.upd.Wl), g_lds.upd.cols,
                                                g_lds.upd.tl);
}

// One r x r FP64 product of the re-orthogonalisation, C = op(A) S B
// (arguments in pgemm(); S = diag(+1 x p, -1 x (r - p)) on the rows of B when
// SGN), tile by tile (128 x 128, at most 2 x 2 of them) with the grid-wide
// product kernel's tile code (gemm_device.h) on the first 256 threads: the
// same arithmetic as the grouped launches' products.  SYM: the tiles on and
// above the diagonal, each written to both triangles.
template <bool TA, bool SGN, bool SYM, int NT>
__device__ __noinline__ void phase_gemm()
{
    const GemmArgs &g = pgemm();
    const int tiles = (g.M + gemm::kTM - 1) / gemm::kTM;
    for (int tn = 0; tn < tiles; ++tn)
        for (int tm = 0; tm < tiles; ++tm) {
            if (SYM && tm > tn) continue;
            gemm::gemm_tile<TA, SGN, SYM, (NT > 256)>(g, 0, 0, 0, tm, tn, g_lds.gemm);
        }
    __syncthreads();
}

// Byte offsets of the parts of a slot.
struct SlotLayout {
    size_t G, V, P, W, d, rho, S, C, nrot, nskip, nact, ntc, maxt, active, ctl, G32, V32, T1, T2, bytes;
};

__host__ __device__ inline SlotLayout slot_layout()
{
    SlotLayout s;
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) / 256 * 256;
        return at;
    };
    const size_t mat = sizeof(double) * (size_t)kPMaxR * kPMaxR, bb = sizeof(double) * kB2 * kB2;
    s.G = take(mat);
    s.V = take(mat);
    s.P = take(bb * kPMaxPairs);
    s.W = take(bb * kPMaxPairs);
    s.d = take(sizeof(double) * kPMaxR);
    s.rho = take(sizeof(int) * kPMaxR);
    s.S = take(sizeof(int4) * kPMaxPairs);
    s.C = take(sizeof(int) * kPMaxPairs);
    s.nrot = take(sizeof(unsigned) * kPMaxPairs);
    s.nskip = take(sizeof(unsigned) * kPMaxPairs);
    s.nact = take(sizeof(unsigned) * kPMaxPairs);
    s.ntc = take(sizeof(unsigned) * kPMaxPairs);
    s.maxt = take(sizeof(double) * kPMaxPairs);
    s.active = take(sizeof(unsigned long long) * kPMaxPairs);
    s.ctl = take(sizeof(Ctl));
    // mixed precision: FP32 working copies, FP64 product scratch
    const size_t mat32 = sizeof(float) * (size_t)kPMaxR * kPMaxR;
    s.G32 = take(mat32);
    s.V32 = take(mat32);
    s.T1 = take(mat);
    s.T2 = take(mat);
    s.bytes = o;
    return s;
}

// d[q] = ||G[:, rho[q]]||^2 for q < r: thread `row` (of the first 256)
// squares its entry, the waves add in butterfly order, the four wave sums are
// added in wave order (the order of the grouped path's norm kernel for
// ldg <= 256 rows).
template <int NT, typename T>
__device__ __forceinline__ void persist_colnorm(const T *G, int ldg, int r, const int *rho, bool init,
                                                double *d, PersistLds &L)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int q = 0; q < r; ++q) {
        const int c = init ? q : rho[q];
        const double x = tid < ldg ? (double)G[(size_t)c * ldg + tid] : 0.0;  // ldg <= 256
        const double s = wave_sum(fma(x, x, 0.0));
        if (lane == 0 && wave < 4) L.colsum[wave][q] = s;
    }
    __syncthreads();
    for (int q = tid; q < r; q += NT) {
        double s = L.colsum[0][q];
#pragma unroll
        for (int w = 1; w < 4; ++w) s += L.colsum[w][q];
        d[q] = s;
    }
    __syncthreads();
}

// Stable sort of positions [0, p) by d decreasing and [p, r) by d increasing,
// rho carried along (as the grouped path's sort).
__device__ __forceinline__ void persist_sort(double *d, int *rho, int r, int p, PersistLds &L)
{
    const int q = threadIdx.x;
    if (q < r) {
        L.sort.dv[q] = d[q];
        L.sort.key[q] = sort_key(L.sort.dv[q]);
        L.sort.val[q] = rho[q];
    }
    __syncthreads();
    if (q < r) {
        const long long kq = L.sort.key[q];
        const bool pos = q < p;
        const int lo = pos ? 0 : p, hi = pos ? p : r;
        int cnt = 0;
        for (int u = lo; u < hi; ++u) {
            const long long kv = L.sort.key[u];
            const bool before = pos ? (kv > kq) : (kv < kq);
            cnt += (before || (kv == kq && u < q)) ? 1 : 0;
        }
        d[lo + cnt] = L.sort.dv[q];
        rho[lo + cnt] = L.sort.val[q];
    }
    __syncthreads();
}

// One problem, by the whole workgroup; A is the LDS copy of its block pair
// arguments that the phases read.
template <int NT>
__device__ void persist_solve(const PersistArgs &pa, int z, char *slot, PersistLds &L, BlockArgsT<double> &A)
{
    const int tid = threadIdx.x;
    const SlotLayout sl = slot_layout();
    const int n = pa.n[z], p = pa.p[z];
    const int r = (n + kB2 - 1) / kB2 * kB2, ldg = r, nb = r / kB, pairs = nb / 2;
    const int steps_per_sweep = pa.ordering == HSVD_ORD_MODMOD ? nb : nb - 1;
    const double tol = pa.tol > 0.0 ? pa.tol : 1e-15 * n;
    const double tth = pa.tthresh > 0.0 ? pa.tthresh : sqrt(tol) / 2.0;
    double *G = reinterpret_cast<double *>(slot + sl.G);
    // the mixed path carries V through its FP32 phase even when it is not returned
    double *V = (pa.want_v || pa.mixed) ? reinterpret_cast<double *>(slot + sl.V) : nullptr;
    double *d = reinterpret_cast<double *>(slot + sl.d);
    int *rho = reinterpret_cast<int *>(slot + sl.rho);
    int4 *S = reinterpret_cast<int4 *>(slot + sl.S);
    Ctl *ctl = reinterpret_cast<Ctl *>(slot + sl.ctl);

    if (tid == 0) {
        BlockArgsT<double> a;
        a.G = G;
        a.V = V;
        a.ldg = ldg;
        a.r = r;
        a.p = p;
        a.nb = nb;
        a.rho = rho;
        a.S_in = S;
        a.S_out = S;
        a.ordering = pa.ordering;
        a.step = 0;
        a.partial = reinterpret_cast<double *>(slot + sl.P);
        a.splits = 1;
        a.rows_per_split = ldg;
        a.W = reinterpret_cast<double *>(slot + sl.W);
        a.active = reinterpret_cast<unsigned long long *>(slot + sl.active);
        a.C = reinterpret_cast<int *>(slot + sl.C);
        a.nrot = reinterpret_cast<unsigned *>(slot + sl.nrot);
        a.nskip = reinterpret_cast<unsigned *>(slot + sl.nskip);
        a.nact = reinterpret_cast<unsigned *>(slot + sl.nact);
        a.ntc = reinterpret_cast<unsigned *>(slot + sl.ntc);
        a.maxt = reinterpret_cast<double *>(slot + sl.maxt);
        a.ctl = ctl;
        a.tol = tol;
        a.tthresh = tth;
        a.inner_sweeps = 0;
        a.nprob = 1;
        A = a;
    }
    __syncthreads();
    const BlockArgsT<double> &a = A;

    // set-up: bordered working copy (eq. 4.1), V = I, counters
    const double *src = pa.Gin + pa.off[z];
    for (int e = tid; e < r * ldg; e += NT) {
        const int c = e / ldg, row = e - c * ldg;
        double v;
        if (c < n)
            v = row < n ? src[(size_t)c * n + row] : 0.0;
        else
            v = row == c ? 1.0 : 0.0;
        G[e] = v;
        if (V) V[e] = row == c ? 1.0 : 0.0;
    }
    if (tid < pairs) {
        a.C[tid] = 0;
        a.nrot[tid] = 0;
        a.nskip[tid] = 0;
        a.nact[tid] = 0;
        a.ntc[tid] = 0;
        a.maxt[tid] = 0.0;
        if (pa.ordering == HSVD_ORD_MODMOD) S[tid] = modmod_start(tid, nb);
    }
    if (tid == 0) {
        ctl->code = 0;
        ctl->rank = 0;
        ctl->inval = 0;
        ctl->rot = 0;
        ctl->skip = 0;
        ctl->act = 0;
        ctl->tcol = 0;
        ctl->maxt = 0.0;
    }
    if (tid < r) rho[tid] = tid;
    __syncthreads();
    persist_colnorm<NT>(G, ldg, r, rho, true, d, L);
    // a non-finite entry or a zero column ends the problem at once
    int status = HSVD_OK;
    {
        int bad_inval = 0, bad_rank = 0;
        for (int q = tid; q < r; q += NT) {
            if (!isfinite(d[q])) bad_inval = 1;
            else if (!(d[q] > 0.0)) bad_rank = 1;
        }
        bad_inval = __syncthreads_or(bad_inval);
        bad_rank = __syncthreads_or(bad_rank);
        status = bad_inval ? HSVD_E_INVAL : (bad_rank ? HSVD_E_RANK : HSVD_OK);
    }
    if (pa.sort && status == HSVD_OK) persist_sort(d, rho, r, p, L);

    int sweeps = 0, code = 0;
    double maxt = 0.0;
    unsigned long long rot_all = 0, skip_all = 0, act_all = 0;
    int sweeps32 = 0, nsiters = 0, restart = 0;
    double nsprev = 2.0;
    if (pa.mixed && status == HSVD_OK) {
        // FP32 block sweeps on FP32 copies of G and V = I, each leaving by the
        // switch rule of a single mixed solve; then V promoted and
        // J-re-orthogonalised (Newton-Schulz, FP64 MFMA products) and
        // G1 = G X, or, after a rank flag in FP32 or a residual above the
        // accepted bound, a restart from G in FP64.  The stepper goes on
        // from where the FP32 sweeps left it.
        float *G32 = reinterpret_cast<float *>(slot + sl.G32);
        float *V32 = reinterpret_cast<float *>(slot + sl.V32);
        double *T1 = reinterpret_cast<double *>(slot + sl.T1);
        double *T2 = reinterpret_cast<double *>(slot + sl.T2);
        for (int e = tid; e < r * ldg; e += NT) {
            const int c = e / ldg, row = e - c * ldg;
            G32[e] = (float)G[e];
            V32[e] = row == c ? 1.f : 0.f;
        }
        // the FP32 Gram resolves cosines down to about sqrt(r) FP32 epsilons
        const double tol32 = fmax(tol, sqrt((double)r) * 0x1p-23);
        if (tid == 0) {
            BlockArgsT<float> f;
            f.G = G32;
            f.V = V32;
            f.ldg = ldg;
            f.r = r;
            f.p = p;
            f.nb = nb;
            f.rho = rho;
            f.S_in = S;
            f.S_out = S;
            f.ordering = pa.ordering;
            f.step = 0;
            f.partial = reinterpret_cast<float *>(a.partial);
            f.splits = 1;
            f.rows_per_split = ldg;
            f.W = reinterpret_cast<float *>(a.W);
            f.active = a.active;
            f.C = a.C;
            f.nrot = a.nrot;
            f.nskip = a.nskip;
            f.nact = a.nact;
            f.ntc = a.ntc;
            f.maxt = a.maxt;
            f.ctl = ctl;
            f.tol = tol32;
            f.tthresh = sqrt(tol32) / 2.0;
            f.inner_sweeps = 0;
            f.nprob = 1;
            pargs32() = f;
        }
        __syncthreads();
        double pm = 1.0, pf = 1.0;
        for (int sw = 0; sw < pa.max_sweeps; ++sw) {
            for (int k = 0; k < steps_per_sweep; ++k) {
                if (tid == 0) pargs32().step = k;
                __syncthreads();
                for (int q = 0; q < pairs; ++q) {
                    phase_gram32(q);
                    __syncthreads();
                    if (k == 0)
                        phase_circle32<NT>(q);
                    else
                        phase_cross32<NT>(q);
                    __syncthreads();
                    const unsigned long long mask = a.active[q];
                    if (mask) {
                        phase_update32<NT>(q, 0, mask);
                        __syncthreads();
                        phase_update32<NT>(q, 1, mask);
                        __syncthreads();
                    }
                }
                if (pa.ordering == HSVD_ORD_MODMOD && tid < pairs) S[tid] = modmod_next(S[tid], nb);
                __syncthreads();
            }
            ++sweeps32;
            persist_colnorm<NT>(G32, ldg, r, rho, false, d, L);
            if (pa.sort) persist_sort(d, rho, r, p, L);
            int c = 0;
            unsigned long long rt = 0, sk = 0, ac = 0;
            double mx = 0.0;
            for (int q = 0; q < pairs; ++q) {
                c |= a.C[q];
                rt += a.nrot[q];
                sk += a.nskip[q];
                ac += a.nact[q];
                mx = fmax(mx, a.maxt[q]);
            }
            const int rank = __hip_atomic_load(&ctl->rank, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            if (tid < pairs) {
                a.C[tid] = 0;
                a.nrot[tid] = 0;
                a.nskip[tid] = 0;
                a.nact[tid] = 0;
                a.ntc[tid] = 0;
                a.maxt[tid] = 0.0;
            }
            if (tid == 0 && rank) __hip_atomic_store(&ctl->rank, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            rot_all += rt;
            skip_all += sk;
            act_all += ac;
            if (rank) {
                // a rank failure is final only in FP64
                restart = 1;
                break;
            }
            // leave FP32 at its resolution, on stagnation, when FP32 itself
            // converged, or by the fraction of rotating pair visits
            const double frac = rt + sk > 0 ? (double)rt / (double)(rt + sk) : 0.0;
            const bool stop = mx <= 3e-4 || (c & 2) == 0 || (mx < 0.1 && mx > 0.25 * pm) || frac < 0.01 ||
                              (frac <= 1.0 / 3.0 && frac >= 0.75 * pf) || sweeps32 >= pa.max_sweeps;
            pm = mx;
            pf = frac;
            if (stop) break;
        }
        if (!restart) {
            for (int e = tid; e < r * ldg; e += NT) V[e] = (double)V32[e];
            __syncthreads();
            // Newton-Schulz: X <- X (3I - J X^T J X) / 2 while the residual
            // max |J X^T J X - I| falls quadratically above its rounding floor
            const double floor_ = 16.0 * n * 0x1p-53;
            for (int it = 0; it <= 6; ++it) {
                if (tid == 0) {
                    GemmArgs g;
                    g.A = V;
                    g.B = V;
                    g.C = T2;
                    g.M = g.N = g.K = r;
                    g.lda = g.ldb = g.ldc = ldg;
                    g.p = p;
                    pgemm() = g;
                }
                __syncthreads();
                phase_gemm<true, true, true, NT>();
                double mxr = 0.0;
                for (int e = tid; e < r * ldg; e += NT) {
                    const int c = e / ldg, row = e - c * ldg;
                    const double b = T2[e];
                    const double y = row < p ? b : -b;
                    const double id = row == c ? 1.0 : 0.0;
                    mxr = fmax(mxr, fabs(y - id));
                    T2[e] = (3.0 * id - y) * 0.5;
                }
#pragma unroll
                for (int m = 32; m >= 1; m >>= 1) mxr = fmax(mxr, __shfl_xor(mxr, m, 64));
                if ((tid & 63) == 0) L.red[tid >> 6] = mxr;
                __syncthreads();
                double resid = L.red[0];
                for (int w = 1; w < NT / 64; ++w) resid = fmax(resid, L.red[w]);
                __syncthreads();
                const bool stop = it == 6 || !(resid < 1.0) || resid <= floor_ || (it > 0 && resid > 0.25 * nsprev);
                nsprev = resid;  // the residual of the current X: the final one once stopped
                if (stop) break;
                ++nsiters;
                if (tid == 0) {
                    GemmArgs g;
                    g.A = V;
                    g.B = T2;
                    g.C = T1;
                    g.M = g.N = g.K = r;
                    g.lda = g.ldb = g.ldc = ldg;
                    pgemm() = g;
                }
                __syncthreads();
                phase_gemm<false, false, false, NT>();
                for (int e = tid; e < r * ldg; e += NT) V[e] = T1[e];
                __syncthreads();
            }
            const double bound = pa.reorth_accept > 0.0 ? pa.reorth_accept : 16384.0 * n * 0x1p-53;
            if (!(nsprev <= bound)) restart = 1;
        }
        if (!restart) {
            // G1 = G X
            if (tid == 0) {
                GemmArgs g;
                g.A = G;
                g.B = V;
                g.C = T1;
                g.M = g.N = g.K = r;
                g.lda = g.ldb = g.ldc = ldg;
                pgemm() = g;
            }
            __syncthreads();
            phase_gemm<false, false, false, NT>();
            for (int e = tid; e < r * ldg; e += NT) G[e] = T1[e];
        } else {
            // FP64 from G: the bordered working copy again, V = I, rho = id
            for (int e = tid; e < r * ldg; e += NT) {
                const int c = e / ldg, row = e - c * ldg;
                double v;
                if (c < n)
                    v = row < n ? src[(size_t)c * n + row] : 0.0;
                else
                    v = row == c ? 1.0 : 0.0;
                G[e] = v;
                V[e] = row == c ? 1.0 : 0.0;
            }
            if (tid < r) rho[tid] = tid;
        }
        __syncthreads();
        // the kept diagonal of the FP64 start and the sort, as after a sweep
        persist_colnorm<NT>(G, ldg, r, rho, false, d, L);
        if (pa.sort) persist_sort(d, rho, r, p, L);
    }
    if (status == HSVD_OK) {
        status = HSVD_E_NOCONV;
        for (int sw = 0; sw < pa.max_sweeps; ++sw) {
            for (int k = 0; k < steps_per_sweep; ++k) {
                if (tid == 0) A.step = k;
                __syncthreads();
                for (int q = 0; q < pairs; ++q) {
                    phase_gram(q);
                    __syncthreads();
                    if (k == 0)
                        phase_circle<NT>(q);
                    else
                        phase_cross<NT>(q);
                    __syncthreads();
                    const unsigned long long mask = a.active[q];
                    if (mask) {
                        phase_update<NT>(q, 0, mask);
                        __syncthreads();
                        if (V) {
                            phase_update<NT>(q, 1, mask);
                            __syncthreads();
                        }
                    }
                }
                if (pa.ordering == HSVD_ORD_MODMOD && tid < pairs) S[tid] = modmod_next(S[tid], nb);
                __syncthreads();
            }
            ++sweeps;
            persist_colnorm<NT>(G, ldg, r, rho, false, d, L);
            if (pa.sort) persist_sort(d, rho, r, p, L);
            // the sweep's codes and counters (eq. 4.2)
            int c = 0;
            unsigned long long rt = 0, sk = 0, ac = 0;
            double mx = 0.0;
            for (int q = 0; q < pairs; ++q) {
                c |= a.C[q];
                rt += a.nrot[q];
                sk += a.nskip[q];
                ac += a.nact[q];
                mx = fmax(mx, a.maxt[q]);
            }
            // the inner solves raise the flag with device-scope atomics
            const int rank = __hip_atomic_load(&ctl->rank, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            if (tid < pairs) {
                a.C[tid] = 0;
                a.nrot[tid] = 0;
                a.nskip[tid] = 0;
                a.nact[tid] = 0;
                a.ntc[tid] = 0;
                a.maxt[tid] = 0.0;
            }
            code = c;
            maxt = mx;
            rot_all += rt;
            skip_all += sk;
            act_all += ac;
            if (rank) {
                status = HSVD_E_RANK;
                break;
            }
            if ((c & 2) == 0) {
                status = HSVD_OK;
                break;
            }
        }
    }

    // Sigma, U = G Sigma^{-1}, lambda, V of the real columns
    const int lane = tid & 63, wave = tid >> 6;
    for (int q = wave; q < r; q += NT / 64) {
        const int c = rho[q];
        if (c >= n) continue;
        const double dq = d[q];
        const double s = sqrt(dq);
        const long long vo = pa.voff[z], mo = pa.off[z];
        if (lane == 0) {
            pa.sigma[vo + c] = s;
            if (pa.lambda) pa.lambda[vo + c] = q < p ? dq : -dq;
        }
        const double *gc = G + (size_t)c * ldg;
        if (pa.U)
            for (int row = lane; row < n; row += 64) pa.U[mo + (size_t)c * n + row] = gc[row] / s;
        if (pa.V && V) {
            const double *vc = V + (size_t)c * ldg;
            for (int row = lane; row < n; row += 64) pa.V[mo + (size_t)c * n + row] = vc[row];
        }
    }
    if (tid == 0 && pa.mixed) {
        pa.sweeps32[z] = sweeps32;
        pa.nsiters[z] = nsiters;
        pa.restart[z] = restart;
        pa.nsres[z] = nsprev;
    }
    if (tid == 0) {
        pa.status[z] = status;
        pa.sweeps[z] = sweeps;
        pa.code[z] = code;
        pa.maxt[z] = maxt;
        pa.rot[z] = rot_all;
        pa.skip[z] = skip_all;
        pa.act[z] = act_all;
    }
    __syncthreads();
}

}  // namespace

// Two waves per SIMD at 256 threads (two workgroups per compute unit, some
// registers spilled): 125 ms against 182 ms with the compiler's own
// allocation (248 registers for the FP64 cross phase, 52 accumulation
// registers more) on a 4096-problem sample of n ~ U{8..256}.
template <int NT>
__global__ __launch_bounds__(NT, NT == 1024 ? 4 : 2) void batch_persist_kernel(PersistArgs pa)
{
    __shared__ int s_idx;
    char *slot = pa.slots + (size_t)blockIdx.x * slot_layout().bytes;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(pa.next, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= pa.batch) break;
        persist_solve<NT>(pa, pa.order[idx], slot, g_lds, pargs());
    }
}

__global__ void persist_zero_kernel(int *next) { *next = 0; }

size_t persist_slot_bytes() { return slot_layout().bytes; }

int persist_blocks_per_cu(int threads)
{
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
    if (threads == 256) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_persist_kernel<256>, 256, 0);
    if (threads == 512) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_persist_kernel<512>, 512, 0);
    if (threads == 1024) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_persist_kernel<1024>, 1024, 0);
    return e == hipSuccess ? blocks : 0;
}

hipError_t launch_batch_persist(hipStream_t st, const PersistArgs &pa, int threads, int workgroups)
{
    if (workgroups < 1 || pa.batch < 1) return hipErrorInvalidValue;
    if (threads != 256 && threads != 512 && threads != 1024) return hipErrorInvalidValue;
    persist_zero_kernel<<<1, 1, 0, st>>>(pa.next);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (threads == 256) batch_persist_kernel<256><<<workgroups, 256, 0, st>>>(pa);
    if (threads == 512) batch_persist_kernel<512><<<workgroups, 512, 0, st>>>(pa);
    if (threads == 1024) batch_persist_kernel<1024><<<workgroups, 1024, 0, st>>>(pa);
    return hipGetLastError();
}

}  // namespace hsvd
