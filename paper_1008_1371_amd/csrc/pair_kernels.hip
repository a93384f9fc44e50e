// Pairwise one-sided Jacobi HSVD kernels for gfx950 (FP64).
//
// One parallel step (Sec. 2: a set of disjoint pivot pairs) is one launch of
// pair_step_kernel with one workgroup per pair slot.  The workgroup keeps the
// two G columns in registers between the dot product and the update, so a
// rotated pair moves exactly 2 reads + 2 writes of G and of V columns, and a
// skipped pair only the 2 G reads.  Columns are column-major with a leading
// dimension padded to a multiple of 64 rows, so every wavefront load is one
// contiguous, aligned 512-byte segment.
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
// kPrefetchV: the V columns are loaded together with G's instead of after the
// rotation decision.  At small orders a step is bound by the dependent chain
// of one pair (loads, reduction, rotation, updates), and this removes one
// memory round trip from it; at large orders, where steps are bandwidth
// bound, skipped pairs would read V for nothing, so it is off there.
template <int WG, int E, bool kPrefetchV>
__global__ __launch_bounds__(WG) void pair_step_kernel(StepArgs a)
{
    __shared__ double sh[2 * (WG / 64)];
    const int k = blockIdx.x;
    int4 st = make_int4(0, 0, 0, 0);
    int i, j;
    if (a.ordering == HSVD_ORD_MODMOD) {
        st = a.S[k];
        i = st.z;
        j = st.w;
    } else {
        const int2 pr = roundrobin_pair(k, a.r, a.step);
        i = pr.x;
        j = pr.y;
    }
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

__global__ __launch_bounds__(kSortWG) void sort_count_kernel(const double *__restrict__ d, int *__restrict__ rank,
                                                             int r, int p)
{
    __shared__ long long tile[kRankTile];
    const int b0 = blockIdx.x * kSortWG, b1 = min(r, b0 + kSortWG);
    const int kb = blockIdx.y * kRankTile, ke = min(r, kb + kRankTile);
    // the keys of this workgroup's positions' segments
    const int need_lo = b0 < p ? 0 : p, need_hi = b1 - 1 < p ? p : r;
    if (ke <= need_lo || kb >= need_hi) return;
    for (int u = threadIdx.x; u < ke - kb; u += kSortWG) tile[u] = sort_key(d[kb + u]);
    __syncthreads();
    const int q = b0 + threadIdx.x;
    if (q >= r) return;
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
// then reset for the next sweep.
__global__ __launch_bounds__(1024) void sweep_reduce_kernel(int *__restrict__ C,
                                                            unsigned int *__restrict__ nrot,
                                                            unsigned int *__restrict__ nskip,
                                                            unsigned int *__restrict__ nact,
                                                            unsigned int *__restrict__ ntc,
                                                            double *__restrict__ maxt,
                                                            int slots, Ctl *ctl)
{
    __shared__ int scode[16];
    __shared__ unsigned long long srot[16], sskip[16], sact[16], stc[16];
    __shared__ double smax[16];
    int code = 0;
    unsigned long long rot = 0, skp = 0, act = 0, tc = 0;
    double mx = 0.0;
    for (int k = threadIdx.x; k < slots; k += 1024) {
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
        scode[w] = code;
        srot[w] = rot;
        sskip[w] = skp;
        sact[w] = act;
        stc[w] = tc;
        smax[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int cc = 0;
        unsigned long long rr = 0, ss = 0, aa = 0, tt = 0;
        double mm = 0.0;
        for (int q = 0; q < 16; ++q) {
            cc |= scode[q];
            rr += srot[q];
            ss += sskip[q];
            aa += sact[q];
            tt += stc[q];
            mm = fmax(mm, smax[q]);
        }
        ctl->code = cc;
        ctl->rot += rr;
        ctl->skip += ss;
        ctl->act += aa;
        ctl->tcol += tt;
        ctl->maxt = mm;
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
