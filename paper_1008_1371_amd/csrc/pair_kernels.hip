// Pairwise one-sided Jacobi HSVD kernels for gfx950 (FP64).
//
// One parallel step (Sec. 2: a set of disjoint pivot pairs) is one launch of
// pair_step_kernel with one workgroup per pair slot.  The workgroup keeps the
// two G columns in registers between the dot product and the update, so a
// rotated pair moves exactly 2 reads + 2 writes of G and of V columns, and a
// skipped pair only the 2 G reads.  Columns are column-major with a leading
// dimension padded to a multiple of 64 rows, so every wavefront load is one
// contiguous, aligned 512-byte segment.
#include <algorithm>

#include "internal.h"

namespace hsvd {

// ---------------------------------------------------------------------------
// Set-up: bordered working copy (eq. 4.1) and V = I.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void setup_kernel(const double *__restrict__ G, int lda, int n,
                                                    double *__restrict__ Gw,
                                                    double *__restrict__ Vw, int r, int ldg)
{
    const int c = blockIdx.x;
    double *gc = Gw + (size_t)c * ldg;
    double *vc = Vw ? Vw + (size_t)c * ldg : nullptr;
    for (int row = threadIdx.x; row < ldg; row += blockDim.x) {
        double g;
        if (c < n)
            g = row < n ? G[(size_t)c * lda + row] : 0.0;
        else
            g = row == c ? 1.0 : 0.0;
        gc[row] = g;
        if (vc) vc[row] = row == c ? 1.0 : 0.0;
    }
}

// Precompute (Alg. 4.2): d = diag(G^T G), rho = id, stepper on the antidiagonal.
template <int WG>
__global__ __launch_bounds__(WG) void precompute_kernel(const double *__restrict__ Gw, int ldg, int r,
                                                        double *__restrict__ d, int *__restrict__ rho,
                                                        int4 *__restrict__ S, int *__restrict__ C,
                                                        unsigned int *__restrict__ nrot,
                                                        unsigned int *__restrict__ nskip,
                                                        unsigned int *__restrict__ nact,
                                                        unsigned int *__restrict__ ntc,
                                                        double *__restrict__ maxt, Ctl *ctl)
{
    __shared__ double sh[WG / 64];
    const int c = blockIdx.x;
    const double *gc = Gw + (size_t)c * ldg;
    double s = 0.0;
    for (int row = threadIdx.x; row < ldg; row += WG) {
        const double x = gc[row];
        s = fma(x, x, s);
    }
    s = block_sum<WG>(s, sh);
    if (threadIdx.x == 0) {
        d[c] = s;
        rho[c] = c;
        if (!isfinite(s)) atomicOr(&ctl->inval, 1);
        else if (!(s > 0.0)) atomicOr(&ctl->rank, 1);
        if (c < r / 2) {
            S[c] = modmod_start(c, r);
            C[c] = 0;
            nrot[c] = 0;
            nskip[c] = 0;
            nact[c] = 0;
            ntc[c] = 0;
            maxt[c] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// One parallel step (Alg. 4.5 for every slot of the step).
// WG threads, E rows per thread per column: ldg <= WG * E.
// ---------------------------------------------------------------------------
// The pair of slot k at step `step` of the sweep; st is the slot's modified
// modulus stepper state (unused for round-robin).
__device__ __forceinline__ void pair_of(const StepArgs &a, int k, int step, int4 &st, int &i, int &j)
{
    st = make_int4(0, 0, 0, 0);
    if (a.ordering == HSVD_ORD_MODMOD) {
        st = a.S[k];
        i = st.z;
        j = st.w;
    } else {
        const int2 pr = roundrobin_pair(k, a.r, step);
        i = pr.x;
        j = pr.y;
    }
}

// One visit of slot k to its pair (i, j): the whole Alg. 4.5 step for that
// pair.  Every thread of the workgroup calls it (workgroup barriers).
// kPrefetchV: the V columns are loaded together with G's instead of after the
// rotation decision.  At small orders a step is bound by the dependent chain
// of one pair (loads, reduction, rotation, updates), and this removes one
// memory round trip from it; at large orders, where steps are bandwidth
// bound, skipped pairs would read V for nothing, so it is off there.
template <int WG, int E, bool kPrefetchV>
__device__ __forceinline__ void pair_visit(const StepArgs &a, int k, int4 st, int i, int j, double *sh)
{
    const int ci = a.rho[i], cj = a.rho[j];
    const double aii = a.d[i], ajj = a.d[j];
    double *__restrict__ gi = a.G + (size_t)ci * a.ldg;
    double *__restrict__ gj = a.G + (size_t)cj * a.ldg;

    double x[E], y[E];
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int row = threadIdx.x + e * WG;
        const bool in = (E == 1 || row < a.ldg);
        x[e] = in ? gi[row] : 0.0;
        y[e] = in ? gj[row] : 0.0;
    }
    double vx[E], vy[E];
    if (kPrefetchV && a.V) {
        const double *vi = a.V + (size_t)ci * a.ldg;
        const double *vj = a.V + (size_t)cj * a.ldg;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = threadIdx.x + e * WG;
            const bool in = (E == 1 || row < a.ldg);
            vx[e] = in ? vi[row] : 0.0;
            vy[e] = in ? vj[row] : 0.0;
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) s = fma(x[e], y[e], s);
    const double aij = block_sum<WG>(s, sh);

    int code = 0;
    bool rotated = false;
    double tabs_ = 0.0;
    if (!rel_orthogonal(aii, ajj, aij, a.tol)) {
        const int hyp = ((i < a.p) == (j < a.p)) ? -1 : 1;
        double t, c;
        if (rotation_params(aii, ajj, aij, hyp, t, c)) {
            if (threadIdx.x == 0) atomicOr(&a.ctl->rank, 1);
        } else {
            rotated = true;
            tabs_ = t;
            code = rotation_code(t, a.tthresh);
            const double ht = hyp < 0 ? -t : t;
            double nx = 0.0, ny = 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double xn = fma(ht, y[e], x[e]) * c;
                const double yn = fma(t, x[e], y[e]) * c;
                x[e] = xn;
                y[e] = yn;
                nx = fma(xn, xn, nx);
                ny = fma(yn, yn, ny);
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int row = threadIdx.x + e * WG;
                if (E == 1 || row < a.ldg) {
                    gi[row] = x[e];
                    gj[row] = y[e];
                }
            }
            block_sum2<WG>(nx, ny, sh);
            if (threadIdx.x == 0) {
                a.d[i] = nx;
                a.d[j] = ny;
            }
            if (a.V) {
                double *__restrict__ vi = a.V + (size_t)ci * a.ldg;
                double *__restrict__ vj = a.V + (size_t)cj * a.ldg;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int row = threadIdx.x + e * WG;
                    const bool in = (E == 1 || row < a.ldg);
                    x[e] = kPrefetchV ? vx[e] : (in ? vi[row] : 0.0);
                    y[e] = kPrefetchV ? vy[e] : (in ? vj[row] : 0.0);
                }
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int row = threadIdx.x + e * WG;
                    const double xn = fma(ht, y[e], x[e]) * c;
                    const double yn = fma(t, x[e], y[e]) * c;
                    if (E == 1 || row < a.ldg) {
                        vi[row] = xn;
                        vj[row] = yn;
                    }
                }
            }
        }
    }
    if (threadIdx.x == 0) {
        if (rotated) {
            a.C[k] |= code;
            a.nrot[k] += 1;
            a.maxt[k] = fmax(a.maxt[k], fabs(tabs_));
        } else {
            a.nskip[k] += 1;
        }
        if (a.ordering == HSVD_ORD_MODMOD) a.S[k] = modmod_next(st, a.r);
    }
}

template <int WG, int E, bool kPrefetchV>
__global__ __launch_bounds__(WG) void pair_step_kernel(StepArgs a)
{
    __shared__ double sh[2 * (WG / 64)];
    int4 st;
    int i, j;
    pair_of(a, blockIdx.x, a.step, st, i, j);
    pair_visit<WG, E, kPrefetchV>(a, blockIdx.x, st, i, j, sh);
}

// ---------------------------------------------------------------------------
// Sort_Diagonal
// ---------------------------------------------------------------------------
// Stable diagonal sort (Alg. 4.1): the destination of position q is the
// number of positions of its sign segment that come before it (larger d in
// [0, p), smaller d in [p, r); equal keys by position), keys compared by
// sort_key.  The count runs over a
// 2-D grid of (256 positions) x (256 keys) tiles, each tile adding its exact
// integer count into rank[q]; then every position moves to its rank.
constexpr int kSortWG = 256;
constexpr int kRankTile = 256;

// Rank counts of the NP positions [b0, b0 + NP) against the keys [kb, kb +
// kRankTile).  Every thread of the NP-thread workgroup calls it (barriers);
// `tile` holds kRankTile keys.
template <int NP>
__device__ __forceinline__ void sort_count_tile(const double *__restrict__ d, int *__restrict__ rank, int r, int p,
                                                int b0, int kb, long long *tile)
{
    const int b1 = min(r, b0 + NP), ke = min(r, kb + kRankTile);
    // the keys of this tile's positions' segments (the same in every thread)
    const int need_lo = b0 < p ? 0 : p, need_hi = b1 - 1 < p ? p : r;
    if (ke <= need_lo || kb >= need_hi) return;
    for (int u = threadIdx.x; u < ke - kb; u += NP) tile[u] = sort_key(d[kb + u]);
    __syncthreads();
    const int q = b0 + threadIdx.x;
    if (q < r) {
        const long long kq = sort_key(d[q]);
        const bool pos = q < p;
        const int lo = pos ? 0 : p, hi = pos ? p : r;
        const int u0 = max(lo, kb) - kb, u1 = min(hi, ke) - kb;
        int cnt = 0;
#pragma unroll 8
        for (int u = u0; u < u1; ++u) {
            const long long kv = tile[u];
            const bool before = pos ? (kv > kq) : (kv < kq);
            cnt += (before || (kv == kq && kb + u < q)) ? 1 : 0;
        }
        if (cnt) atomicAdd(&rank[q], cnt);
    }
    __syncthreads();
}

__global__ __launch_bounds__(kSortWG) void sort_count_kernel(const double *__restrict__ d, int *__restrict__ rank,
                                                             int r, int p)
{
    __shared__ long long tile[kRankTile];
    sort_count_tile<kSortWG>(d, rank, r, p, blockIdx.x * kSortWG, blockIdx.y * kRankTile, tile);
}

__global__ __launch_bounds__(256) void sort_scatter_kernel(const double *__restrict__ d, const int *__restrict__ rho,
                                                           int *__restrict__ rank, double *__restrict__ dtmp,
                                                           int *__restrict__ rtmp, int r, int p)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= r) return;
    const int dst = (q < p ? 0 : p) + rank[q];
    dtmp[dst] = d[q];
    rtmp[dst] = rho[q];
}

__global__ __launch_bounds__(256) void sort_zero_kernel(int *__restrict__ rank, int r)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q < r) rank[q] = 0;
}

__global__ __launch_bounds__(256) void sort_copy_kernel(double *__restrict__ d, int *__restrict__ rho,
                                                        const double *__restrict__ dtmp,
                                                        const int *__restrict__ rtmp, int r)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q < r) {
        d[q] = dtmp[q];
        rho[q] = rtmp[q];
    }
}

// Per-sweep reduction of the slot codes and counters (Check_Convergence),
// then reset for the next sweep, by one workgroup of NT threads (every thread
// calls it).  Thread 0 returns the sweep's code.
struct ReduceLds {
    int code[16];
    unsigned long long rot[16], skip[16], act[16], tc[16];
    double mx[16];
};

template <int NT>
__device__ __forceinline__ int sweep_reduce_wg(int *__restrict__ C, unsigned int *__restrict__ nrot,
                                               unsigned int *__restrict__ nskip, unsigned int *__restrict__ nact,
                                               unsigned int *__restrict__ ntc, double *__restrict__ maxt,
                                               int slots, Ctl *ctl, ReduceLds &L)
{
    static_assert(NT % 64 == 0 && NT <= 1024, "workgroup size");
    int code = 0;
    unsigned long long rot = 0, skp = 0, act = 0, tc = 0;
    double mx = 0.0;
    for (int k = threadIdx.x; k < slots; k += NT) {
        code |= C[k];
        rot += nrot[k];
        skp += nskip[k];
        act += nact[k];
        tc += ntc[k];
        mx = fmax(mx, maxt[k]);
        C[k] = 0;
        nrot[k] = 0;
        nskip[k] = 0;
        nact[k] = 0;
        ntc[k] = 0;
        maxt[k] = 0.0;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        code |= __shfl_xor(code, m, 64);
        rot += __shfl_xor(rot, m, 64);
        skp += __shfl_xor(skp, m, 64);
        act += __shfl_xor(act, m, 64);
        tc += __shfl_xor(tc, m, 64);
        mx = fmax(mx, __shfl_xor(mx, m, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        L.code[w] = code;
        L.rot[w] = rot;
        L.skip[w] = skp;
        L.act[w] = act;
        L.tc[w] = tc;
        L.mx[w] = mx;
    }
    __syncthreads();
    int cc = 0;
    if (threadIdx.x == 0) {
        unsigned long long rr = 0, ss = 0, aa = 0, tt = 0;
        double mm = 0.0;
        for (int q = 0; q < NT / 64; ++q) {
            cc |= L.code[q];
            rr += L.rot[q];
            ss += L.skip[q];
            aa += L.act[q];
            tt += L.tc[q];
            mm = fmax(mm, L.mx[q]);
        }
        ctl->code = cc;
        ctl->rot += rr;
        ctl->skip += ss;
        ctl->act += aa;
        ctl->tcol += tt;
        ctl->maxt = mm;
    }
    __syncthreads();
    return cc;
}

__global__ __launch_bounds__(1024) void sweep_reduce_kernel(int *__restrict__ C,
                                                            unsigned int *__restrict__ nrot,
                                                            unsigned int *__restrict__ nskip,
                                                            unsigned int *__restrict__ nact,
                                                            unsigned int *__restrict__ ntc,
                                                            double *__restrict__ maxt,
                                                            int slots, Ctl *ctl)
{
    __shared__ ReduceLds L;
    sweep_reduce_wg<1024>(C, nrot, nskip, nact, ntc, maxt, slots, ctl, L);
}

// ---------------------------------------------------------------------------
// Persistent pairwise kernel: every sweep of a solve in one cooperative
// launch (all workgroups resident at once, so the waits below end).
//
// Workgroup g visits the slots g, g + grid, ... of every step, in step order.
// Between steps, either
//  - a grid barrier, or
//  - per position: ver[i] counts the completed visits of position i (one per
//    step: every step pairs all r positions), and the visit of step s waits
//    until both of its positions have s completed visits.  The order is a
//    perfect matching at every step, so the pair waits exactly for the two
//    visits of step s - 1 that last read and wrote its columns; a workgroup's
//    oldest pending visit always has its predecessors done, so some visit can
//    always proceed.
// A visit publishes its G, V and d writes with a release at device scope
// before its ver increments, and a wait ends with an acquire.  At a sweep's
// end a grid barrier, the diagonal sort (the rank counts spread over all
// workgroups), the counter reduction and the convergence test (eq. 4.2) by
// workgroup 0, and a grid barrier after which every workgroup reads the
// decision.  Every wait is bounded by pa.spin_limit wall-clock ticks: past it
// the workgroup raises pc->err and leaves, and every other wait sees err and
// leaves too, so the launch always ends.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wait_limit_passed(const PairPersistArgs &pa, unsigned long long t0)
{
    return __hip_atomic_load(&pa.pc->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
           (long long)(wall_clock64() - t0) > pa.spin_limit;
}

// Release of the workgroup's writes at device scope: every wave waits for its
// own memory operations, the workgroup meets, then the first wave issues the
// release fence for all of them (one L2 write-back per workgroup rather than
// one per wave).  A release fence followed by a relaxed atomic write is a
// release of that write.
__device__ __forceinline__ void wg_release()
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x < 64) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

// Spin (relaxed loads, so no cache invalidation per poll) until `done()`;
// then one acquire fence.  Thread 0 only.  False when the launch gives up.
template <typename F>
__device__ __forceinline__ bool spin_acquire(const PairPersistArgs &pa, F done)
{
    bool ok = true;
    const unsigned long long t0 = wall_clock64();
    while (!done()) {
        if (wait_limit_passed(pa, t0)) {
            __hip_atomic_fetch_or(&pa.pc->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

// Grid barrier (generation counting).  Returns false in every thread when the
// launch is giving up.
__device__ __forceinline__ bool grid_sync(const PairPersistArgs &pa, unsigned int &gen, int *s_ok)
{
    wg_release();
    if (threadIdx.x == 0) {
        bool ok = true;
        PersistCtl *pc = pa.pc;
        const unsigned int g = gen;
        const unsigned int old = __hip_atomic_fetch_add(&pc->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gridDim.x - 1) {
            // the last arrival: acquire everyone's release, reset, open
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&pc->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&pc->gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = spin_acquire(pa, [&] {
                return __hip_atomic_load(&pc->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != g;
            });
        }
        gen = g + 1;
        *s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Wait until positions i and j have `need` completed visits.
__device__ __forceinline__ bool wait_ready(const PairPersistArgs &pa, int i, int j, unsigned int need, int *s_ok)
{
    if (threadIdx.x == 0) {
        const bool ok = spin_acquire(pa, [&] {
            return __hip_atomic_load(&pa.ver[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need &&
                   __hip_atomic_load(&pa.ver[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        });
        *s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Publish a visit: positions i and j now have `done` completed visits.
__device__ __forceinline__ void publish(const PairPersistArgs &pa, int i, int j, unsigned int done)
{
    wg_release();
    if (threadIdx.x == 0) {
        __hip_atomic_store(&pa.ver[i], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&pa.ver[j], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int WG, int E, bool kPrefetchV>
__global__ __launch_bounds__(WG) void pair_persist_kernel(PairPersistArgs pa)
{
    __shared__ double sh[2 * (WG / 64)];
    __shared__ long long tile[kRankTile];
    __shared__ ReduceLds red;
    __shared__ int s_ok;
    const StepArgs &a = pa.a;
    const int slots = a.r / 2;
    int *const rank = pa.rtmp + a.r;
    unsigned int gen = 0, gstep = 0;
    for (int sw = 0; sw < pa.max_sweeps; ++sw) {
        for (int k = 0; k < pa.steps; ++k, ++gstep) {
            for (int slot = blockIdx.x; slot < slots; slot += gridDim.x) {
                int4 st;
                int i, j;
                pair_of(a, slot, k, st, i, j);
                if (pa.dataflow && !wait_ready(pa, i, j, gstep, &s_ok)) return;
                pair_visit<WG, E, kPrefetchV>(a, slot, st, i, j, sh);
                if (pa.dataflow) publish(pa, i, j, gstep + 1);
            }
            if (!pa.dataflow && !grid_sync(pa, gen, &s_ok)) return;
        }
        if (pa.dataflow && !grid_sync(pa, gen, &s_ok)) return;
        if (pa.sort) {
            // ranks (zero on entry), destinations, moves back
            const int npt = (a.r + WG - 1) / WG, nkt = (a.r + kRankTile - 1) / kRankTile;
            for (int t = blockIdx.x; t < npt * nkt; t += gridDim.x)
                sort_count_tile<WG>(a.d, rank, a.r, a.p, (t / nkt) * WG, (t % nkt) * kRankTile, tile);
            if (!grid_sync(pa, gen, &s_ok)) return;
            for (int q = blockIdx.x * WG + threadIdx.x; q < a.r; q += gridDim.x * WG) {
                const int dst = (q < a.p ? 0 : a.p) + rank[q];
                rank[q] = 0;
                pa.dtmp[dst] = a.d[q];
                pa.rtmp[dst] = a.rho[q];
            }
            if (!grid_sync(pa, gen, &s_ok)) return;
            for (int q = blockIdx.x * WG + threadIdx.x; q < a.r; q += gridDim.x * WG) {
                a.d[q] = pa.dtmp[q];
                const_cast<int *>(a.rho)[q] = pa.rtmp[q];
            }
        }
        if (blockIdx.x == 0) {
            const int code = sweep_reduce_wg<WG>(a.C, a.nrot, a.nskip, pa.nact, pa.ntc, a.maxt, slots, a.ctl, red);
            if (threadIdx.x == 0) {
                const int rank_flag = __hip_atomic_load(&a.ctl->rank, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // eq. (4.2): codes 00 and 01 stop the process
                const int stop = rank_flag ? 2 : ((code & 2) == 0 ? 1 : 0);
                __hip_atomic_store(&pa.pc->sweeps, sw + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&pa.pc->stop, stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (!grid_sync(pa, gen, &s_ok)) return;
        if (__hip_atomic_load(&pa.pc->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
    }
}

__global__ void zero_ctl_kernel(Ctl *ctl)
{
    if (threadIdx.x == 0) {
        ctl->code = 0;
        ctl->rank = 0;
        ctl->inval = 0;
        ctl->pad = 0;
        ctl->rot = 0;
        ctl->skip = 0;
        ctl->act = 0;
        ctl->tcol = 0;
        ctl->maxt = 0.0;
        ctl->nsres = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Finalize: sigma, U = G Sigma^{-1}, lambda = sigma^2 j, V, perm (Sec. 2).
// One workgroup per position.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void finalize_kernel(const double *__restrict__ Gw,
                                                       const double *__restrict__ Vw,
                                                       const double *__restrict__ d,
                                                       const int *__restrict__ rho, int n, int p,
                                                       int ldg, double *__restrict__ sigma,
                                                       double *__restrict__ U, int ldu,
                                                       double *__restrict__ V, int ldv,
                                                       double *__restrict__ lambda)
{
    const int q = blockIdx.x;
    const int c = rho[q];
    if (c >= n) return;
    const double dq = d[q];
    const double s = sqrt(dq);
    if (threadIdx.x == 0) {
        sigma[c] = s;
        if (lambda) lambda[c] = q < p ? dq : -dq;
    }
    const double *gc = Gw + (size_t)c * ldg;
    if (U)
        for (int row = threadIdx.x; row < n; row += blockDim.x) U[(size_t)c * ldu + row] = gc[row] / s;
    if (V && Vw) {
        const double *vc = Vw + (size_t)c * ldg;
        for (int row = threadIdx.x; row < n; row += blockDim.x) V[(size_t)c * ldv + row] = vc[row];
    }
}

// perm: physical columns by position, border columns (index >= n) dropped.
__global__ __launch_bounds__(1024) void perm_kernel(const int *__restrict__ rho, int r, int n,
                                                    int *__restrict__ perm)
{
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < r; base += 1024) {
        const int q = base + threadIdx.x;
        const int c = q < r ? rho[q] : n;
        const int keep = c < n ? 1 : 0;
        // inclusive scan of keep over the 1024 threads
        int v = keep;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            const int u = __shfl_up(v, m, 64);
            if (lane >= m) v += u;
        }
        if (lane == 63) wsum[w] = v;
        __syncthreads();
        int before = carry;
        for (int q2 = 0; q2 < w; ++q2) before += wsum[q2];
        if (keep) perm[before + v - 1] = c;
        __syncthreads();
        if (threadIdx.x == 1023) carry = before + v;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Diagnostics
// ---------------------------------------------------------------------------
template <bool kFast>
__global__ void pair_params_kernel(long long m, const double *__restrict__ aii,
                                   const double *__restrict__ ajj, const double *__restrict__ aij,
                                   const int *__restrict__ hyp, double tol, double tthresh,
                                   int *__restrict__ skip, double *__restrict__ t,
                                   double *__restrict__ c, int *__restrict__ status,
                                   int *__restrict__ code)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    double tt = 0.0, cc = 1.0;
    const bool orth = kFast ? rel_orthogonal_sq(aii[k], ajj[k], aij[k], tol, tol * tol)
                            : rel_orthogonal(aii[k], ajj[k], aij[k], tol);
    int sk = orth ? 1 : 0;
    int stt = 0, cd = 0;
    if (!sk) {
        stt = kFast ? rotation_params_fast(aii[k], ajj[k], aij[k], hyp[k], tt, cc)
                    : rotation_params(aii[k], ajj[k], aij[k], hyp[k], tt, cc);
        if (!stt) cd = rotation_code(tt, tthresh);
    }
    skip[k] = sk;
    t[k] = tt;
    c[k] = cc;
    status[k] = stt;
    code[k] = cd;
}

__global__ void pivot_trace_kernel(int ordering, int r, int steps, int *__restrict__ pairs)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r / 2) return;
    int4 st = modmod_start(k, r);
    for (int s = 0; s < steps; ++s) {
        int2 pr;
        if (ordering == HSVD_ORD_MODMOD) {
            pr = make_int2(st.z, st.w);
            st = modmod_next(st, r);
        } else {
            pr = roundrobin_pair(k, r, s % (r - 1));
        }
        int *o = pairs + ((size_t)s * (r / 2) + k) * 2;
        o[0] = pr.x;
        o[1] = pr.y;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_setup(hipStream_t st, const double *G, int lda, int n, const Workspace &w, int r,
                        int ldg, bool want_v)
{
    setup_kernel<<<r, 256, 0, st>>>(G, lda, n, w.G, want_v ? w.V : nullptr, r, ldg);
    return hipGetLastError();
}

hipError_t launch_precompute(hipStream_t st, const Workspace &w, int r, int ldg)
{
    precompute_kernel<256><<<r, 256, 0, st>>>(w.G, ldg, r, w.d, w.rho, w.S, w.C, w.nrot, w.nskip,
                                              w.nact, w.ntc, w.maxt, w.ctl);
    return hipGetLastError();
}

template <int WG, int E>
static hipError_t step_as(hipStream_t st, const StepArgs &a)
{
    // V prefetch up to 1024 rows (measured: 5% per step at n = 1024)
    if (a.ldg <= 1024)
        pair_step_kernel<WG, E, true><<<a.r / 2, WG, 0, st>>>(a);
    else
        pair_step_kernel<WG, E, false><<<a.r / 2, WG, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_pair_step(hipStream_t st, const StepArgs &a)
{
    const int L = a.ldg;  // multiple of 64
    if (L <= 64) return step_as<64, 1>(st, a);
    if (L <= 128) return step_as<64, 2>(st, a);
    if (L <= 256) return step_as<64, 4>(st, a);
    if (L <= 512) return step_as<128, 4>(st, a);
    if (L <= 1024) return step_as<256, 4>(st, a);
    if (L <= 2048) return step_as<256, 8>(st, a);
    if (L <= 4096) return step_as<256, 16>(st, a);
    if (L <= 8192) return step_as<512, 16>(st, a);
    return step_as<1024, 16>(st, a);
}

// Sort ranks, visit counts and the control block to zero before a launch.
__global__ __launch_bounds__(256) void persist_reset_kernel(int *__restrict__ rank, unsigned int *__restrict__ ver,
                                                            int r, PersistCtl *pc)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q < r) {
        rank[q] = 0;
        ver[q] = 0u;
    }
    if (q == 0) {
        pc->count = 0u;
        pc->gen = 0u;
        pc->err = 0;
        pc->stop = 0;
        pc->sweeps = 0;
    }
}

template <int WG, int E, bool kPrefetchV>
static hipError_t persist_as(hipStream_t st, const PairPersistArgs &a, int *grid)
{
    const void *fn = reinterpret_cast<const void *>(&pair_persist_kernel<WG, E, kPrefetchV>);
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, WG, 0);
    if (e != hipSuccess) return e;
    if (!coop || per_cu < 1) return hipErrorNotSupported;
    const int g = std::min(a.a.r / 2, per_cu * cus);
    *grid = g;
    persist_reset_kernel<<<(a.a.r + 255) / 256, 256, 0, st>>>(a.rtmp + a.a.r, a.ver, a.a.r, a.pc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    PairPersistArgs arg = a;
    void *args[] = {&arg};
    return hipLaunchCooperativeKernel(fn, dim3(g), dim3(WG), args, 0, st);
}

hipError_t launch_pair_persist(hipStream_t st, const PairPersistArgs &a, int *grid)
{
    const int L = a.a.ldg;  // multiple of 64; the same shapes as the per-step launches
    if (L <= 64) return persist_as<64, 1, true>(st, a, grid);
    if (L <= 128) return persist_as<64, 2, true>(st, a, grid);
    if (L <= 256) return persist_as<64, 4, true>(st, a, grid);
    if (L <= 512) return persist_as<128, 4, true>(st, a, grid);
    if (L <= 1024) return persist_as<256, 4, true>(st, a, grid);
    if (L <= 2048) return persist_as<256, 8, false>(st, a, grid);
    if (L <= 4096) return persist_as<256, 16, false>(st, a, grid);
    if (L <= 8192) return persist_as<512, 16, false>(st, a, grid);
    return persist_as<1024, 16, false>(st, a, grid);
}

hipError_t launch_sort(hipStream_t st, double *d, int *rho, double *dtmp, int *rtmp, int r, int p)
{
    // rtmp holds 2r ints: the moved rho, then the ranks
    int *rank = rtmp + r;
    const int blocks = (r + kSortWG - 1) / kSortWG;
    sort_zero_kernel<<<blocks, 256, 0, st>>>(rank, r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sort_count_kernel<<<dim3(blocks, (r + kRankTile - 1) / kRankTile), kSortWG, 0, st>>>(d, rank, r, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    sort_scatter_kernel<<<blocks, 256, 0, st>>>(d, rho, rank, dtmp, rtmp, r, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    sort_copy_kernel<<<blocks, 256, 0, st>>>(d, rho, dtmp, rtmp, r);
    return hipGetLastError();
}

hipError_t launch_sweep_reduce(hipStream_t st, const Workspace &w, int slots)
{
    sweep_reduce_kernel<<<1, 1024, 0, st>>>(w.C, w.nrot, w.nskip, w.nact, w.ntc, w.maxt, slots, w.ctl);
    return hipGetLastError();
}

hipError_t launch_zero_ctl(hipStream_t st, Ctl *ctl)
{
    zero_ctl_kernel<<<1, 64, 0, st>>>(ctl);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t st, const Workspace &w, int n, int r, int p, int ldg,
                           double *sigma, double *U, int ldu, double *V, int ldv, double *lambda,
                           int *perm)
{
    finalize_kernel<<<r, 256, 0, st>>>(w.G, w.V, w.d, w.rho, n, p, ldg, sigma, U, ldu, V, ldv, lambda);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (perm) {
        perm_kernel<<<1, 1024, 0, st>>>(w.rho, r, n, perm);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_pair_params(hipStream_t st, long long m, const double *aii, const double *ajj,
                              const double *aij, const int *hyp, double tol, double tthresh,
                              int *skip, double *t, double *c, int *status, int *code, bool fast)
{
    if (m == 0) return hipSuccess;
    const long long blocks = (m + 255) / 256;
    if (fast)
        pair_params_kernel<true><<<(unsigned)blocks, 256, 0, st>>>(m, aii, ajj, aij, hyp, tol, tthresh, skip,
                                                                   t, c, status, code);
    else
        pair_params_kernel<false><<<(unsigned)blocks, 256, 0, st>>>(m, aii, ajj, aij, hyp, tol, tthresh, skip,
                                                                    t, c, status, code);
    return hipGetLastError();
}

hipError_t launch_pivot_trace(hipStream_t st, int ordering, int r, int steps, int *pairs)
{
    const int slots = r / 2;
    pivot_trace_kernel<<<(slots + 255) / 256, 256, 0, st>>>(ordering, r, steps, pairs);
    return hipGetLastError();
}

}  // namespace hsvd
