// Batched solves: many independent problems of uneven order and signature.
//
// The library groups the problems by their bordered order r (a multiple of 2b)
// and runs the block path over a whole group at once: every launch of the
// Gram / inner / update kernels covers all (problem, block pair) tasks of a
// step, so the latency-bound inner solves of thousands of small problems run
// side by side.  These kernels are the per-problem set-up, the kept diagonal,
// the sort, the per-problem stop rule (eq. 4.2) and the output extraction;
// each problem converges, and stops being worked on, on its own.
#include "internal.h"

namespace hsvd {

// Bordered working copy of problem z (eq. 4.1) and V = I.  grid (r, nprob)
__global__ __launch_bounds__(256) void batch_setup_kernel(BatchGroup g, const double *__restrict__ Gin,
                                                          int want_v)
{
    const int c = blockIdx.x, z = blockIdx.y;
    if (g.only && !g.only[z]) return;
    const int n = g.n[z];
    const size_t mat = (size_t)g.ldg * g.r;
    double *gc = g.G + z * mat + (size_t)c * g.ldg;
    double *vc = want_v ? g.V + z * mat + (size_t)c * g.ldg : nullptr;
    const double *src = Gin + g.off[z] + (size_t)c * n;
    for (int row = threadIdx.x; row < g.ldg; row += 256) {
        double v;
        if (c < n)
            v = row < n ? src[row] : 0.0;
        else
            v = row == c ? 1.0 : 0.0;
        gc[row] = v;
        if (vc) vc[row] = row == c ? 1.0 : 0.0;
    }
}

// d[z][q] = ||G_z[:, rho_z[q]]||^2.  With init: rho = id, per-problem slot
// counters cleared, non-finite / zero columns flagged.  grid (r, nprob)
__global__ __launch_bounds__(256) void batch_colnorm_kernel(BatchGroup g, int init)
{
    __shared__ double sh[4];
    const int q = blockIdx.x, z = blockIdx.y;
    if (!init && g.done[z]) return;
    if (init && g.only && !g.only[z]) return;
    const size_t mat = (size_t)g.ldg * g.r;
    int *rho = g.rho + (size_t)z * g.r;
    const int c = init ? q : rho[q];
    const double *gc = g.G + z * mat + (size_t)c * g.ldg;
    double s = 0.0;
    for (int row = threadIdx.x; row < g.ldg; row += 256) {
        const double x = gc[row];
        s = fma(x, x, s);
    }
    s = block_sum<256>(s, sh);
    if (threadIdx.x == 0) {
        g.d[(size_t)z * g.r + q] = s;
        if (init) {
            rho[q] = q;
            Ctl *ctl = g.ctl + z;
            if (!isfinite(s)) atomicOr(&ctl->inval, 1);
            else if (!(s > 0.0)) atomicOr(&ctl->rank, 1);
            if (q < g.pairs) {
                const size_t k = (size_t)z * g.pairs + q;
                g.C[k] = 0;
                g.nrot[k] = 0;
                g.nskip[k] = 0;
                g.nact[k] = 0;
                g.ntc[k] = 0;
                g.maxt[k] = 0.0;
            }
        }
    }
}

// Stable diagonal sort of each problem (positions [0, p) by d decreasing,
// [p, r) increasing; keys compared by sort_key), one workgroup per problem
// (r <= 1024).  grid nprob
__global__ __launch_bounds__(1024) void batch_sort_kernel(BatchGroup g)
{
    __shared__ long long key[1024];
    __shared__ double dv[1024];
    __shared__ int val[1024];
    const int z = blockIdx.x;
    if (g.done[z]) return;
    const int r = g.r, p = g.p[z];
    double *d = g.d + (size_t)z * r;
    int *rho = g.rho + (size_t)z * r;
    const int q = threadIdx.x;
    if (q < r) {
        dv[q] = d[q];
        key[q] = sort_key(dv[q]);
        val[q] = rho[q];
    }
    __syncthreads();
    if (q < r) {
        const long long kq = key[q];
        const bool pos = q < p;
        const int lo = pos ? 0 : p, hi = pos ? p : r;
        int cnt = 0;
        for (int u = lo; u < hi; ++u) {
            const long long kv = key[u];
            const bool before = pos ? (kv > kq) : (kv < kq);
            cnt += (before || (kv == kq && u < q)) ? 1 : 0;
        }
        d[lo + cnt] = dv[q];
        rho[lo + cnt] = val[q];
    }
}

// After the set-up: problems with a non-finite entry or a zero column stop at once.
__global__ void batch_init_decide_kernel(BatchGroup g)
{
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= g.nprob) return;
    if (g.only && !g.only[z]) return;
    const Ctl *ctl = g.ctl + z;
    g.sweeps[z] = 0;
    if (ctl->inval) {
        g.status[z] = HSVD_E_INVAL;
        g.done[z] = 1;
    } else if (ctl->rank) {
        g.status[z] = HSVD_E_RANK;
        g.done[z] = 1;
    } else {
        g.status[z] = HSVD_OK;
        g.done[z] = 0;
    }
}

// End of a sweep: per problem, OR of the slot codes and the stop rule of
// eq. (4.2); problems still running are counted.  grid nprob, 64 threads
__global__ __launch_bounds__(64) void batch_reduce_decide_kernel(BatchGroup g)
{
    const int z = blockIdx.x;
    if (g.done[z]) return;
    int code = 0;
    unsigned long long rot = 0, skp = 0, act = 0, tc = 0;
    double mx = 0.0;
    for (int q = threadIdx.x; q < g.pairs; q += 64) {
        const size_t k = (size_t)z * g.pairs + q;
        code |= g.C[k];
        rot += g.nrot[k];
        skp += g.nskip[k];
        act += g.nact[k];
        tc += g.ntc[k];
        mx = fmax(mx, g.maxt[k]);
        g.C[k] = 0;
        g.nrot[k] = 0;
        g.nskip[k] = 0;
        g.nact[k] = 0;
        g.ntc[k] = 0;
        g.maxt[k] = 0.0;
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
    if (threadIdx.x == 0) {
        Ctl *ctl = g.ctl + z;
        ctl->code = code;
        ctl->rot += rot;
        ctl->skip += skp;
        ctl->act += act;
        ctl->tcol += tc;
        ctl->maxt = mx;
        const int sw = g.sweeps[z] + 1;
        g.sweeps[z] = sw;
        if (ctl->rank) {
            g.status[z] = HSVD_E_RANK;
            g.done[z] = 1;
        } else if ((code & 2) == 0) {
            g.status[z] = HSVD_OK;
            g.done[z] = 1;
        } else if (sw >= g.max_sweeps) {
            g.status[z] = HSVD_E_NOCONV;
            g.done[z] = 1;
        } else {
            atomicAdd(g.active_count, 1);
        }
    }
}

// sigma, U = G Sigma^{-1}, lambda, V of problem z into the packed outputs.
// grid (r, nprob)
__global__ __launch_bounds__(256) void batch_finalize_kernel(BatchGroup g, double *__restrict__ sigma,
                                                             double *__restrict__ U, double *__restrict__ V,
                                                             double *__restrict__ lambda)
{
    const int q = blockIdx.x, z = blockIdx.y;
    const int n = g.n[z], p = g.p[z];
    const int c = g.rho[(size_t)z * g.r + q];
    if (c >= n) return;
    const double dq = g.d[(size_t)z * g.r + q];
    const double s = sqrt(dq);
    const long long vo = g.voff[z], mo = g.off[z];
    if (threadIdx.x == 0) {
        sigma[vo + c] = s;
        if (lambda) lambda[vo + c] = q < p ? dq : -dq;
    }
    const size_t mat = (size_t)g.ldg * g.r;
    const double *gc = g.G + z * mat + (size_t)c * g.ldg;
    if (U)
        for (int row = threadIdx.x; row < n; row += 256) U[mo + (size_t)c * n + row] = gc[row] / s;
    if (V && g.V) {
        const double *vc = g.V + z * mat + (size_t)c * g.ldg;
        for (int row = threadIdx.x; row < n; row += 256) V[mo + (size_t)c * n + row] = vc[row];
    }
}

__global__ void batch_zero_ctl_kernel(Ctl *ctl, int nprob, int *active_count, const int *only)
{
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z == 0) *active_count = 0;
    if (z >= nprob) return;
    if (only && !only[z]) return;
    ctl[z].code = 0;
    ctl[z].rank = 0;
    ctl[z].inval = 0;
    ctl[z].pad = 0;
    ctl[z].rot = 0;
    ctl[z].skip = 0;
    ctl[z].act = 0;
    ctl[z].tcol = 0;
    ctl[z].maxt = 0.0;
    ctl[z].nsres = 0.0;
}

__global__ void batch_zero_count_kernel(int *active_count) { *active_count = 0; }

// ---------------------------------------------------------------------------
// Mixed precision over a group (the steps of a single mixed solve, per problem)
// ---------------------------------------------------------------------------

// FP32 copies G32 = G, V32 = I and the per-problem FP32 state; problems that
// failed their set-up (done) stay out of both phases.  grid (r, nprob)
__global__ __launch_bounds__(256) void batch_mixed_init_kernel(BatchGroup g, BatchMixed m)
{
    const int c = blockIdx.x, z = blockIdx.y;
    if (c == 0 && threadIdx.x == 0) {
        m.done32[z] = g.done[z];
        m.sweeps32[z] = 0;
        m.prev_maxt[z] = 1.0;
        m.prev_frac[z] = 1.0;
        m.nsdone[z] = g.done[z];
        m.apply[z] = 0;
        m.nsprev[z] = 2.0;
        m.nsiters[z] = 0;
        m.restart[z] = 0;
        g.ctl[z].nsres = 0.0;
        // the FP32 Gram resolves cosines down to about sqrt(r) FP32 epsilons
        const double t32 = fmax(g.tol[z], sqrt((double)g.r) * 0x1p-23);
        m.tol32[z] = t32;
        m.tth32[z] = sqrt(t32) / 2.0;
    }
    if (g.done[z]) return;
    const size_t mat = (size_t)g.ldg * g.r;
    const double *gc = g.G + z * mat + (size_t)c * g.ldg;
    float *g32 = m.G32 + z * mat + (size_t)c * g.ldg;
    float *v32 = m.V32 + z * mat + (size_t)c * g.ldg;
    for (int row = threadIdx.x; row < g.ldg; row += 256) {
        g32[row] = (float)gc[row];
        v32[row] = row == c ? 1.f : 0.f;
    }
}

// d[z][q] = ||G32_z[:, rho_z[q]]||^2 (accumulated in FP64) for the problems in
// their FP32 phase.  grid (r, nprob)
__global__ __launch_bounds__(256) void batch_colnorm32_kernel(BatchGroup g, BatchMixed m)
{
    __shared__ double sh[4];
    const int q = blockIdx.x, z = blockIdx.y;
    if (m.done32[z]) return;
    const size_t mat = (size_t)g.ldg * g.r;
    const int c = g.rho[(size_t)z * g.r + q];
    const float *gc = m.G32 + z * mat + (size_t)c * g.ldg;
    double s = 0.0;
    for (int row = threadIdx.x; row < g.ldg; row += 256) {
        const double x = (double)gc[row];
        s = fma(x, x, s);
    }
    s = block_sum<256>(s, sh);
    if (threadIdx.x == 0) g.d[(size_t)z * g.r + q] = s;
}

// Per problem after an FP32 sweep: reduce the slot counters, then leave FP32
// when the largest tangent is at the FP32 resolution (<= 3e-4), when it
// stagnates below 0.1, when FP32 converged, when the fraction f of the
// sweep's pair visits that rotated is below 1/100, or f <= 1/3 while falling
// by less than a quarter per sweep (the rule of a single mixed solve), or at
// max_sweeps.  A rank flag ends the FP32 phase and marks the problem for a
// restart from G in FP64 (the FP32 Gram resolves S - |w| of a hyperbolic
// pair only to about sqrt(r) FP32 epsilons; a rank failure is final only in
// FP64).  grid nprob, 64 threads
__global__ __launch_bounds__(64) void batch_decide32_kernel(BatchGroup g, BatchMixed m)
{
    const int z = blockIdx.x;
    if (m.done32[z]) return;
    int code = 0;
    unsigned long long rot = 0, skp = 0;
    double mx = 0.0;
    for (int q = threadIdx.x; q < g.pairs; q += 64) {
        const size_t k = (size_t)z * g.pairs + q;
        code |= g.C[k];
        rot += g.nrot[k];
        skp += g.nskip[k];
        mx = fmax(mx, g.maxt[k]);
        g.C[k] = 0;
        g.nrot[k] = 0;
        g.nskip[k] = 0;
        g.nact[k] = 0;
        g.ntc[k] = 0;
        g.maxt[k] = 0.0;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        code |= __shfl_xor(code, s, 64);
        rot += __shfl_xor(rot, s, 64);
        skp += __shfl_xor(skp, s, 64);
        mx = fmax(mx, __shfl_xor(mx, s, 64));
    }
    if (threadIdx.x == 0) {
        Ctl *ctl = g.ctl + z;
        ctl->rot += rot;
        ctl->skip += skp;
        const int sw = m.sweeps32[z] + 1;
        m.sweeps32[z] = sw;
        const double frac = rot + skp > 0 ? (double)rot / (double)(rot + skp) : 0.0;
        if (ctl->rank) {
            ctl->rank = 0;
            m.done32[z] = 1;
            m.nsdone[z] = 1;
            m.restart[z] = 1;
        } else {
            const double pm = m.prev_maxt[z], pf = m.prev_frac[z];
            const bool stop = mx <= 3e-4 || (code & 2) == 0 || (mx < 0.1 && mx > 0.25 * pm) || frac < 0.01 ||
                              (frac <= 1.0 / 3.0 && frac >= 0.75 * pf) || sw >= g.max_sweeps;
            if (stop) m.done32[z] = 1;
            else atomicAdd(g.active_count, 1);
        }
        m.prev_maxt[z] = mx;
        m.prev_frac[z] = frac;
    }
}

// V = V32 promoted.  grid (r, nprob)
__global__ __launch_bounds__(256) void batch_promote_kernel(BatchGroup g, BatchMixed m)
{
    const int c = blockIdx.x, z = blockIdx.y;
    if (g.done[z]) return;
    const size_t mat = (size_t)g.ldg * g.r;
    const float *src = m.V32 + z * mat + (size_t)c * g.ldg;
    double *dst = g.V + z * mat + (size_t)c * g.ldg;
    for (int row = threadIdx.x; row < g.ldg; row += 256) dst[row] = (double)src[row];
}

// T2 holds X^T J X of problem z.  Y = J T2; T2 <- (3I - Y) / 2; the largest
// |Y - I| entry into ctl[z].nsres (non-negative doubles order like their bit
// patterns, so an integer max is exact and order independent).  grid (r, nprob)
__global__ __launch_bounds__(256) void batch_ns_form_kernel(BatchGroup g, BatchMixed m)
{
    __shared__ double sh[256];
    const int c = blockIdx.x, z = blockIdx.y;
    if (m.nsdone[z]) return;
    const int p = g.p[z];
    const size_t mat = (size_t)g.ldg * g.r;
    double *B = m.T2 + z * mat + (size_t)c * g.ldg;
    double mx = 0.0;
    for (int row = threadIdx.x; row < g.r; row += 256) {
        const double b = B[row];
        const double y = row < p ? b : -b;
        const double id = row == c ? 1.0 : 0.0;
        mx = fmax(mx, fabs(y - id));
        B[row] = (3.0 * id - y) * 0.5;
    }
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(&g.ctl[z].nsres),
                  static_cast<unsigned long long>(__double_as_longlong(sh[0])));
}

// Per problem: the correction of this iteration applies unless X is already
// J-orthogonal to working accuracy (residual at the rounding floor of its n
// real columns, or no longer falling quadratically); counts the problems it
// applies to.  grid ceil(nprob / 256)
__global__ void batch_ns_decide_kernel(BatchGroup g, BatchMixed m, int iter, int last)
{
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= g.nprob) return;
    if (m.nsdone[z]) {
        m.apply[z] = 0;
        return;
    }
    const double resid = g.ctl[z].nsres;
    g.ctl[z].nsres = 0.0;
    const double floor_ = 16.0 * g.n[z] * 0x1p-53;
    const bool stop =
        last || !(resid < 1.0) || resid <= floor_ || (iter > 0 && resid > 0.25 * m.nsprev[z]);
    m.nsprev[z] = resid;  // the residual of the current X: the final one once stopped
    if (stop) {
        m.nsdone[z] = 1;
        m.apply[z] = 0;
    } else {
        m.apply[z] = 1;
        m.nsiters[z] += 1;
        atomicAdd(g.active_count, 1);
    }
}

// After the J-re-orthogonalisation: a problem whose final residual is above
// the accepted bound (m.accept, or 16384 n u) restarts from G in FP64, like
// one flagged rank deficient in its FP32 phase; apply[z] marks the problems
// that go on from G1 = G X.  grid ceil(nprob / 256)
__global__ void batch_ns_accept_kernel(BatchGroup g, BatchMixed m)
{
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= g.nprob) return;
    if (g.done[z]) {
        m.apply[z] = 0;
        return;
    }
    const double bound = m.accept > 0.0 ? m.accept : 16384.0 * g.n[z] * 0x1p-53;
    if (!m.restart[z] && !(m.nsprev[z] <= bound)) m.restart[z] = 1;
    m.apply[z] = m.restart[z] ? 0 : 1;
}

// dst_z <- src_z where flag[z] != 0 (invert: == 0).  grid (r, nprob)
__global__ __launch_bounds__(256) void batch_copy_if_kernel(BatchGroup g, const double *__restrict__ src,
                                                            double *__restrict__ dst, const int *__restrict__ flag,
                                                            int invert)
{
    const int c = blockIdx.x, z = blockIdx.y;
    if ((flag[z] != 0) == (invert != 0)) return;
    const size_t mat = (size_t)g.ldg * g.r;
    const size_t o = z * mat + (size_t)c * g.ldg;
    for (int row = threadIdx.x; row < g.ldg; row += 256) dst[o + row] = row < g.r ? src[o + row] : 0.0;
}

hipError_t launch_batch_mixed_init(hipStream_t st, const BatchGroup &g, const BatchMixed &m)
{
    batch_mixed_init_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, m);
    return hipGetLastError();
}

hipError_t launch_batch_colnorm32(hipStream_t st, const BatchGroup &g, const BatchMixed &m)
{
    batch_colnorm32_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, m);
    return hipGetLastError();
}

hipError_t launch_batch_decide32(hipStream_t st, const BatchGroup &g, const BatchMixed &m)
{
    batch_zero_count_kernel<<<1, 1, 0, st>>>(g.active_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    batch_decide32_kernel<<<g.nprob, 64, 0, st>>>(g, m);
    return hipGetLastError();
}

hipError_t launch_batch_promote(hipStream_t st, const BatchGroup &g, const BatchMixed &m)
{
    batch_promote_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, m);
    return hipGetLastError();
}

hipError_t launch_batch_ns_form(hipStream_t st, const BatchGroup &g, const BatchMixed &m)
{
    batch_ns_form_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, m);
    return hipGetLastError();
}

hipError_t launch_batch_ns_decide(hipStream_t st, const BatchGroup &g, const BatchMixed &m, int iter, bool last)
{
    batch_zero_count_kernel<<<1, 1, 0, st>>>(g.active_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    batch_ns_decide_kernel<<<(g.nprob + 255) / 256, 256, 0, st>>>(g, m, iter, last ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_ns_accept(hipStream_t st, const BatchGroup &g, const BatchMixed &m)
{
    batch_ns_accept_kernel<<<(g.nprob + 255) / 256, 256, 0, st>>>(g, m);
    return hipGetLastError();
}

hipError_t launch_batch_copy_if(hipStream_t st, const BatchGroup &g, const double *src, double *dst,
                                const int *flag, bool invert)
{
    batch_copy_if_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, src, dst, flag, invert ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_setup(hipStream_t st, const BatchGroup &g, const double *G, bool want_v)
{
    batch_zero_ctl_kernel<<<(g.nprob + 255) / 256, 256, 0, st>>>(g.ctl, g.nprob, g.active_count, g.only);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    batch_setup_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, G, want_v ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    batch_colnorm_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, 1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    batch_init_decide_kernel<<<(g.nprob + 255) / 256, 256, 0, st>>>(g);
    return hipGetLastError();
}

hipError_t launch_batch_colnorm(hipStream_t st, const BatchGroup &g, bool init)
{
    batch_colnorm_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, init ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_sort(hipStream_t st, const BatchGroup &g)
{
    batch_sort_kernel<<<g.nprob, 1024, 0, st>>>(g);
    return hipGetLastError();
}

hipError_t launch_batch_reduce_decide(hipStream_t st, const BatchGroup &g)
{
    batch_zero_count_kernel<<<1, 1, 0, st>>>(g.active_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    batch_reduce_decide_kernel<<<g.nprob, 64, 0, st>>>(g);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(hipStream_t st, const BatchGroup &g, double *sigma, double *U, double *V,
                                 double *lambda)
{
    batch_finalize_kernel<<<dim3(g.r, g.nprob), 256, 0, st>>>(g, sigma, U, V, lambda);
    return hipGetLastError();
}

}  // namespace hsvd
