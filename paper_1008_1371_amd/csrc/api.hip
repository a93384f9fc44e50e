// C ABI of libhsvd (include/hsvd.h) and the host driver of the sweep loop.
//
// The driver follows the structure of the paper's host routine (Alg. 4.1):
// set-up and Precompute_Data, Sort_Diagonal, then sweeps of parallel steps,
// each sweep ending with the convergence check and another sort.  The only
// host synchronisation inside a solve is one small copy of the control block
// per sweep, which decides whether another sweep is launched.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "internal.h"

struct hsvd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hsvd::Ctl *host_ctl = nullptr;           // pinned
    std::vector<hipEvent_t> events;          // reusable timing events
};

namespace hsvd {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

Layout make_layout(int n, int r, int ldg, bool want_v)
{
    Layout L;
    L.n = n;
    L.r = r;
    L.ldg = ldg;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    const size_t slots = (size_t)r / 2;
    L.off_G = take(sizeof(double) * (size_t)ldg * r);
    L.off_V = take(want_v ? sizeof(double) * (size_t)ldg * r : 0);
    L.off_d = take(sizeof(double) * r);
    L.off_rho = take(sizeof(int) * r);
    L.off_dtmp = take(sizeof(double) * r);
    L.off_rtmp = take(sizeof(int) * r);
    L.off_S = take(sizeof(int4) * slots);
    L.off_C = take(sizeof(int) * slots);
    L.off_nrot = take(sizeof(unsigned int) * slots);
    L.off_nskip = take(sizeof(unsigned int) * slots);
    L.off_ctl = take(sizeof(Ctl));
    L.bytes = o;
    return L;
}

Workspace carve(void *base, const Layout &L)
{
    char *b = static_cast<char *>(base);
    Workspace w;
    w.G = reinterpret_cast<double *>(b + L.off_G);
    w.V = L.off_d > L.off_V ? reinterpret_cast<double *>(b + L.off_V) : nullptr;
    w.d = reinterpret_cast<double *>(b + L.off_d);
    w.rho = reinterpret_cast<int *>(b + L.off_rho);
    w.dtmp = reinterpret_cast<double *>(b + L.off_dtmp);
    w.rtmp = reinterpret_cast<int *>(b + L.off_rtmp);
    w.S = reinterpret_cast<int4 *>(b + L.off_S);
    w.C = reinterpret_cast<int *>(b + L.off_C);
    w.nrot = reinterpret_cast<unsigned int *>(b + L.off_nrot);
    w.nskip = reinterpret_cast<unsigned int *>(b + L.off_nskip);
    w.ctl = reinterpret_cast<Ctl *>(b + L.off_ctl);
    return w;
}

}  // namespace hsvd

using namespace hsvd;

#define HSVD_TRY(expr)                              \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return HSVD_E_DEVICE; \
    } while (0)

static hsvd_status ensure_ws(hsvd_ctx *ctx, size_t bytes)
{
    if (ctx->ws_bytes >= bytes) return HSVD_OK;
    if (ctx->ws) {
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) return HSVD_E_DEVICE;
        hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return HSVD_E_NOMEM;
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    return HSVD_OK;
}

static hsvd_status ensure_events(hsvd_ctx *ctx, size_t count)
{
    while (ctx->events.size() < count) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return HSVD_E_DEVICE;
        ctx->events.push_back(e);
    }
    return HSVD_OK;
}

extern "C" {

const char *hsvd_version(void) { return "hsvd-gfx950 0.1"; }

void hsvd_default_params(hsvd_params *prm)
{
    if (!prm) return;
    prm->precision = HSVD_FP64;
    prm->algo = HSVD_AUTO;
    prm->ordering = HSVD_ORD_MODMOD;
    prm->block = 0;
    prm->sort = 1;
    prm->want_v = 1;
    prm->max_sweeps = 100;
    prm->tol = 0.0;
    prm->t_thresh = 0.0;
}

hsvd_status hsvd_init(hsvd_ctx **out, int device, void *hip_stream)
{
    if (!out) return HSVD_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return HSVD_E_DEVICE;
    if (device < 0 || device >= count) return HSVD_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return HSVD_E_DEVICE;
    hsvd_ctx *ctx = new (std::nothrow) hsvd_ctx();
    if (!ctx) return HSVD_E_NOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    void *h = nullptr;
    if (hipHostMalloc(&h, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return HSVD_E_DEVICE;
    }
    ctx->host_ctl = static_cast<Ctl *>(h);
    *out = ctx;
    return HSVD_OK;
}

hsvd_status hsvd_destroy(hsvd_ctx *ctx)
{
    if (!ctx) return HSVD_E_INVAL;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->events) hipEventDestroy(e);
    if (ctx->ws) hipFree(ctx->ws);
    if (ctx->host_ctl) hipHostFree(ctx->host_ctl);
    delete ctx;
    return HSVD_OK;
}

hsvd_status hsvd_solve(hsvd_ctx *ctx, const double *G, int lda, int n, int p, const hsvd_params *prm_in,
                       double *sigma, double *U, int ldu, double *V, int ldv, double *lambda, int *perm,
                       hsvd_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    if (!ctx || !G || !sigma) return HSVD_E_INVAL;
    hsvd_params prm;
    if (prm_in) prm = *prm_in;
    else hsvd_default_params(&prm);
    if (n < 1 || p < 0 || p > n || lda < n) return HSVD_E_INVAL;
    if (U && ldu < n) return HSVD_E_INVAL;
    if (V && ldv < n) return HSVD_E_INVAL;
    if (prm.ordering != HSVD_ORD_MODMOD && prm.ordering != HSVD_ORD_ROUNDROBIN) return HSVD_E_INVAL;
    if (prm.precision != HSVD_FP64) return HSVD_E_INVAL;
    if (prm.algo != HSVD_AUTO && prm.algo != HSVD_PAIRWISE) return HSVD_E_INVAL;
    if (V && !prm.want_v) return HSVD_E_INVAL;
    const int r = (n + 1) / 2 * 2;  // eq. (4.1): even order
    if (r > kMaxOrder) return HSVD_E_INVAL;
    const int ldg = (r + 63) / 64 * 64;
    const double tol = prm.tol > 0.0 ? prm.tol : 1e-15 * n;
    const double tthresh = prm.t_thresh > 0.0 ? prm.t_thresh : sqrt(tol) / 2.0;
    const int max_sweeps = prm.max_sweeps > 0 ? prm.max_sweeps : 100;
    const bool want_v = prm.want_v != 0;
    if (!isfinite(tol) || !isfinite(tthresh)) return HSVD_E_INVAL;

    HSVD_TRY(hipSetDevice(ctx->device));
    const Layout L = make_layout(n, r, ldg, want_v);
    hsvd_status s = ensure_ws(ctx, L.bytes);
    if (s != HSVD_OK) return s;
    s = ensure_events(ctx, 4);
    if (s != HSVD_OK) return s;
    const Workspace w = carve(ctx->ws, L);
    hipStream_t st = ctx->stream;
    hipEvent_t ev_t0 = ctx->events[0], ev_t1 = ctx->events[1];
    hipEvent_t ev_s0 = ctx->events[2], ev_s1 = ctx->events[3];

    HSVD_TRY(hipEventRecord(ev_t0, st));
    HSVD_TRY(launch_zero_ctl(st, w.ctl));
    HSVD_TRY(launch_setup(st, G, lda, n, w, r, ldg, want_v));
    HSVD_TRY(launch_precompute(st, w, r, ldg));
    if (prm.sort) HSVD_TRY(launch_sort(st, w.d, w.rho, w.dtmp, w.rtmp, r, p));
    HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipStreamSynchronize(st));

    hsvd_status status = HSVD_OK;
    int sweeps = 0, code = 0;
    long long steps = 0, launches = 0;
    double ms_steps = 0.0;
    if (ctx->host_ctl->inval) status = HSVD_E_INVAL;
    else if (ctx->host_ctl->rank) status = HSVD_E_RANK;

    StepArgs a;
    a.G = w.G;
    a.V = want_v ? w.V : nullptr;
    a.ldg = ldg;
    a.r = r;
    a.p = p;
    a.d = w.d;
    a.rho = w.rho;
    a.S = w.S;
    a.C = w.C;
    a.nrot = w.nrot;
    a.nskip = w.nskip;
    a.ctl = w.ctl;
    a.ordering = prm.ordering;
    a.tol = tol;
    a.tthresh = tthresh;
    const int steps_per_sweep = prm.ordering == HSVD_ORD_MODMOD ? r : r - 1;

    bool converged = false;
    if (status == HSVD_OK) {
        for (int sw = 0; sw < max_sweeps; ++sw) {
            HSVD_TRY(hipEventRecord(ev_s0, st));
            for (int k = 0; k < steps_per_sweep; ++k) {
                a.step = k;
                HSVD_TRY(launch_pair_step(st, a));
            }
            HSVD_TRY(hipEventRecord(ev_s1, st));
            steps += steps_per_sweep;
            launches += steps_per_sweep;
            if (prm.sort) HSVD_TRY(launch_sort(st, w.d, w.rho, w.dtmp, w.rtmp, r, p));
            HSVD_TRY(launch_sweep_reduce(st, w, r / 2));
            HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
            HSVD_TRY(hipStreamSynchronize(st));
            float ms = 0.f;
            HSVD_TRY(hipEventElapsedTime(&ms, ev_s0, ev_s1));
            ms_steps += ms;
            ++sweeps;
            code = ctx->host_ctl->code;
            if (ctx->host_ctl->rank) {
                status = HSVD_E_RANK;
                break;
            }
            if ((code & 2) == 0) {  // eq. (4.2): codes 00 and 01 stop the process
                converged = true;
                break;
            }
        }
        if (status == HSVD_OK && !converged) status = HSVD_E_NOCONV;
    }

    HSVD_TRY(launch_finalize(st, w, n, r, p, ldg, sigma, U, ldu, V, ldv, lambda, perm));
    HSVD_TRY(hipEventRecord(ev_t1, st));
    HSVD_TRY(hipStreamSynchronize(st));
    if (info) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ev_t0, ev_t1);
        info->status = status;
        info->sweeps = sweeps;
        info->code = code;
        info->r = r;
        info->rotations = (long long)ctx->host_ctl->rot;
        info->skips = (long long)ctx->host_ctl->skip;
        info->steps = steps;
        info->ms_total = ms;
        info->ms_steps = ms_steps;
        info->step_launches = launches;
        const double rr = (double)r;
        info->step_bytes = (double)info->rotations * 64.0 * rr + (double)info->skips * 16.0 * rr;
        if (!want_v) info->step_bytes -= (double)info->rotations * 32.0 * rr;
        info->step_flops = (double)info->rotations * (want_v ? 18.0 : 12.0) * rr +
                           (double)info->skips * 2.0 * rr;
    }
    return status;
}

hsvd_status hsvd_pair_params(hsvd_ctx *ctx, long long m, const double *aii, const double *ajj,
                             const double *aij, const int *hyp, double tol, double t_thresh, int *skip,
                             double *t, double *c, int *status, int *code)
{
    if (!ctx || m < 0) return HSVD_E_INVAL;
    if (m > 0 && (!aii || !ajj || !aij || !hyp || !skip || !t || !c || !status || !code))
        return HSVD_E_INVAL;
    HSVD_TRY(hipSetDevice(ctx->device));
    HSVD_TRY(launch_pair_params(ctx->stream, m, aii, ajj, aij, hyp, tol, t_thresh, skip, t, c, status,
                                code));
    HSVD_TRY(hipStreamSynchronize(ctx->stream));
    return HSVD_OK;
}

hsvd_status hsvd_pivot_trace(hsvd_ctx *ctx, int ordering, int r, int steps, int *pairs)
{
    if (!ctx || r < 2 || (r & 1) || steps < 0 || (steps > 0 && !pairs)) return HSVD_E_INVAL;
    if (ordering != HSVD_ORD_MODMOD && ordering != HSVD_ORD_ROUNDROBIN) return HSVD_E_INVAL;
    if (steps == 0) return HSVD_OK;
    HSVD_TRY(hipSetDevice(ctx->device));
    HSVD_TRY(launch_pivot_trace(ctx->stream, ordering, r, steps, pairs));
    HSVD_TRY(hipStreamSynchronize(ctx->stream));
    return HSVD_OK;
}

hsvd_status hsvd_sort_diag(hsvd_ctx *ctx, int r, int p, double *d, int *rho)
{
    if (!ctx || r < 1 || r > kMaxOrder || p < 0 || p > r || !d || !rho) return HSVD_E_INVAL;
    HSVD_TRY(hipSetDevice(ctx->device));
    const size_t need = hsvd::make_layout(r, r + (r & 1), 64, false).bytes;
    hsvd_status s = ensure_ws(ctx, need);
    if (s != HSVD_OK) return s;
    const Workspace w = carve(ctx->ws, make_layout(r, r + (r & 1), 64, false));
    HSVD_TRY(launch_sort(ctx->stream, d, rho, w.dtmp, w.rtmp, r, p));
    HSVD_TRY(hipStreamSynchronize(ctx->stream));
    return HSVD_OK;
}

}  // extern "C"
