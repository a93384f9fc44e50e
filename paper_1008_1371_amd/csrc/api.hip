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

Layout make_layout(int n, int r, int ldg, bool want_v, int pairs, int splits, int b2)
{
    Layout L;
    L.n = n;
    L.r = r;
    L.ldg = ldg;
    L.pairs = pairs;
    L.splits = splits;
    L.b2 = b2;
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
    L.off_nact = take(sizeof(unsigned int) * slots);
    L.off_ctl = take(sizeof(Ctl));
    const size_t bb = (size_t)b2 * b2;
    L.off_P = take(sizeof(double) * (size_t)pairs * splits * bb);
    L.off_W = take(sizeof(double) * (size_t)pairs * bb);
    L.off_active = take(sizeof(int) * (size_t)pairs);
    L.off_S2 = take(sizeof(int4) * 2 * (size_t)pairs);
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
    w.nact = reinterpret_cast<unsigned int *>(b + L.off_nact);
    w.ctl = reinterpret_cast<Ctl *>(b + L.off_ctl);
    if (L.pairs > 0) {
        w.P = reinterpret_cast<double *>(b + L.off_P);
        w.W = reinterpret_cast<double *>(b + L.off_W);
        w.active = reinterpret_cast<int *>(b + L.off_active);
        w.S2 = reinterpret_cast<int4 *>(b + L.off_S2);
    }
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
    if (prm.algo != HSVD_AUTO && prm.algo != HSVD_PAIRWISE && prm.algo != HSVD_BLOCK) return HSVD_E_INVAL;
    if (prm.block != 0 && prm.block != block_width()) return HSVD_E_INVAL;
    if (V && !prm.want_v) return HSVD_E_INVAL;
    // The block path needs at least two blocks of b columns; AUTO takes it from n >= 512.
    const bool block = prm.algo == HSVD_BLOCK || (prm.algo == HSVD_AUTO && n >= 512);
    const int b = block ? block_width() : 0;
    const int mult = block ? 2 * b : 2;
    const int r = (n + mult - 1) / mult * mult;  // eq. (4.1) bordering
    if (r > kMaxOrder) return HSVD_E_INVAL;
    const int ldg = block ? (r + 255) / 256 * 256 : (r + 63) / 64 * 64;
    const double tol = prm.tol > 0.0 ? prm.tol : 1e-15 * n;
    const double tthresh = prm.t_thresh > 0.0 ? prm.t_thresh : sqrt(tol) / 2.0;
    const int max_sweeps = prm.max_sweeps > 0 ? prm.max_sweeps : 100;
    const bool want_v = prm.want_v != 0;
    if (!isfinite(tol) || !isfinite(tthresh)) return HSVD_E_INVAL;

    const int nb = block ? r / b : 0;
    const int pairs = nb / 2;
    int splits = 0, rows_per_split = 0;
    if (block) {
        // split the Gram's rows so that about 1024 workgroups run per step
        const int chunks = ldg / 64;
        int want = (1024 + pairs - 1) / pairs;
        want = want < 1 ? 1 : (want > chunks ? chunks : want);
        rows_per_split = (chunks + want - 1) / want * 64;
        splits = (ldg + rows_per_split - 1) / rows_per_split;
    }
    const int steps_per_sweep = block ? (prm.ordering == HSVD_ORD_MODMOD ? nb : nb - 1)
                                      : (prm.ordering == HSVD_ORD_MODMOD ? r : r - 1);

    HSVD_TRY(hipSetDevice(ctx->device));
    const Layout L = make_layout(n, r, ldg, want_v, pairs, splits, block ? 2 * b : 0);
    hsvd_status s = ensure_ws(ctx, L.bytes);
    if (s != HSVD_OK) return s;
    const int nev = block ? 4 + 4 * steps_per_sweep : 4;
    s = ensure_events(ctx, (size_t)nev);
    if (s != HSVD_OK) return s;
    const Workspace w = carve(ctx->ws, L);
    hipStream_t st = ctx->stream;
    hipEvent_t *ev = ctx->events.data();

    HSVD_TRY(hipEventRecord(ev[0], st));
    HSVD_TRY(launch_zero_ctl(st, w.ctl));
    HSVD_TRY(launch_setup(st, G, lda, n, w, r, ldg, want_v));
    HSVD_TRY(launch_precompute(st, w, r, ldg));
    if (block) HSVD_TRY(launch_block_stepper_init(st, w.S2, nb));
    if (prm.sort) HSVD_TRY(launch_sort(st, w.d, w.rho, w.dtmp, w.rtmp, r, p));
    HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HSVD_TRY(hipStreamSynchronize(st));

    hsvd_status status = HSVD_OK;
    int sweeps = 0, code = 0;
    long long steps = 0;
    double kms[HSVD_NKERNELS] = {0, 0, 0, 0};
    long long klaunch[HSVD_NKERNELS] = {0, 0, 0, 0};
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

    BlockArgs ba;
    ba.G = w.G;
    ba.V = want_v ? w.V : nullptr;
    ba.ldg = ldg;
    ba.r = r;
    ba.p = p;
    ba.nb = nb;
    ba.rho = w.rho;
    ba.ordering = prm.ordering;
    ba.partial = w.P;
    ba.splits = splits;
    ba.rows_per_split = rows_per_split;
    ba.W = w.W;
    ba.active = w.active;
    ba.C = w.C;
    ba.nrot = w.nrot;
    ba.nskip = w.nskip;
    ba.nact = w.nact;
    ba.ctl = w.ctl;
    ba.tol = tol;
    ba.tthresh = tthresh;

    bool converged = false;
    long long gstep = 0;
    if (status == HSVD_OK) {
        for (int sw = 0; sw < max_sweeps; ++sw) {
            if (!block) {
                HSVD_TRY(hipEventRecord(ev[2], st));
                for (int k = 0; k < steps_per_sweep; ++k) {
                    a.step = k;
                    HSVD_TRY(launch_pair_step(st, a));
                }
                HSVD_TRY(hipEventRecord(ev[3], st));
                klaunch[HSVD_K_PAIR_STEP] += steps_per_sweep;
            } else {
                for (int k = 0; k < steps_per_sweep; ++k, ++gstep) {
                    ba.step = k;
                    ba.S_in = w.S2 + (gstep & 1) * pairs;
                    ba.S_out = w.S2 + ((gstep + 1) & 1) * pairs;
                    hipEvent_t *e = ev + 4 + 4 * k;
                    HSVD_TRY(hipEventRecord(e[0], st));
                    HSVD_TRY(launch_block_gram(st, ba));
                    HSVD_TRY(hipEventRecord(e[1], st));
                    HSVD_TRY(launch_block_inner(st, ba));
                    HSVD_TRY(hipEventRecord(e[2], st));
                    HSVD_TRY(launch_block_update(st, ba));
                    HSVD_TRY(hipEventRecord(e[3], st));
                }
                klaunch[HSVD_K_BLOCK_GRAM] += steps_per_sweep;
                klaunch[HSVD_K_BLOCK_INNER] += steps_per_sweep;
                klaunch[HSVD_K_BLOCK_UPDATE] += steps_per_sweep;
                // the kept diagonal: fresh column norms of the updated columns
                HSVD_TRY(launch_colnorm_pos(st, w.G, ldg, w.rho, w.d, r));
            }
            steps += steps_per_sweep;
            if (prm.sort) HSVD_TRY(launch_sort(st, w.d, w.rho, w.dtmp, w.rtmp, r, p));
            HSVD_TRY(launch_sweep_reduce(st, w, block ? pairs : r / 2));
            HSVD_TRY(hipMemcpyAsync(ctx->host_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
            HSVD_TRY(hipStreamSynchronize(st));
            float ms = 0.f;
            if (!block) {
                HSVD_TRY(hipEventElapsedTime(&ms, ev[2], ev[3]));
                kms[HSVD_K_PAIR_STEP] += ms;
            } else {
                for (int k = 0; k < steps_per_sweep; ++k) {
                    hipEvent_t *e = ev + 4 + 4 * k;
                    for (int q = 0; q < 3; ++q) {
                        HSVD_TRY(hipEventElapsedTime(&ms, e[q], e[q + 1]));
                        kms[HSVD_K_BLOCK_GRAM + q] += ms;
                    }
                }
            }
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
    HSVD_TRY(hipEventRecord(ev[1], st));
    HSVD_TRY(hipStreamSynchronize(st));
    if (info) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ev[0], ev[1]);
        info->status = status;
        info->sweeps = sweeps;
        info->code = code;
        info->r = r;
        info->block = b;
        info->ldg = ldg;
        info->rotations = (long long)ctx->host_ctl->rot;
        info->skips = (long long)ctx->host_ctl->skip;
        info->steps = steps;
        info->active_pairs = (long long)ctx->host_ctl->act;
        info->ms_total = ms;
        const double rows = (double)ldg;
        const double vmul = want_v ? 2.0 : 1.0;
        for (int q = 0; q < HSVD_NKERNELS; ++q) {
            info->kernel_ms[q] = kms[q];
            info->kernel_launches[q] = klaunch[q];
        }
        if (!block) {
            // a rotated pair reads and writes two columns of G (and of V); a
            // skipped pair reads two columns of G; flops: dot 2, update 6 and
            // new norms 4 per row for G, update 6 per row for V
            const double rot = (double)info->rotations, skp = (double)info->skips;
            info->kernel_bytes[HSVD_K_PAIR_STEP] = rot * 32.0 * rows * vmul + skp * 16.0 * rows;
            info->kernel_flops[HSVD_K_PAIR_STEP] = rot * (12.0 + 6.0 * (vmul - 1.0)) * rows + skp * 2.0 * rows;
        } else {
            // per block pair and step: the Gram reads 2b columns and does a full
            // (2b)^2 x rows product; an active pair's update reads and writes the
            // 2b columns of G (and of V) with (2b)^2 x rows multiply-adds each
            const double b2 = 2.0 * b;
            const double visits = (double)steps * pairs;
            const double act = (double)info->active_pairs;
            info->kernel_bytes[HSVD_K_BLOCK_GRAM] = visits * 8.0 * b2 * rows;
            info->kernel_flops[HSVD_K_BLOCK_GRAM] = visits * 2.0 * b2 * b2 * rows;
            info->kernel_bytes[HSVD_K_BLOCK_UPDATE] = act * 16.0 * b2 * rows * vmul;
            info->kernel_flops[HSVD_K_BLOCK_UPDATE] = act * 2.0 * b2 * b2 * rows * vmul;
            info->kernel_bytes[HSVD_K_BLOCK_INNER] = visits * (double)(splits + 1) * 8.0 * b2 * b2;
            info->kernel_flops[HSVD_K_BLOCK_INNER] = 0.0;
        }
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

hsvd_status hsvd_block_trace(hsvd_ctx *ctx, int ordering, int r, int b, int steps, int *pairs)
{
    if (!ctx || b != block_width() || r < 2 * b || r % (2 * b) || r > kMaxOrder || steps < 0 ||
        (steps > 0 && !pairs))
        return HSVD_E_INVAL;
    if (ordering != HSVD_ORD_MODMOD && ordering != HSVD_ORD_ROUNDROBIN) return HSVD_E_INVAL;
    if (steps == 0) return HSVD_OK;
    HSVD_TRY(hipSetDevice(ctx->device));
    const int nb = r / b;
    const Layout L = make_layout(r, r, 64, false, nb / 2, 1, 2);
    hsvd_status s = ensure_ws(ctx, L.bytes);
    if (s != HSVD_OK) return s;
    const Workspace w = carve(ctx->ws, L);
    HSVD_TRY(launch_block_stepper_init(ctx->stream, w.S2, nb));
    const int per_sweep = ordering == HSVD_ORD_MODMOD ? nb : nb - 1;
    size_t off = 0;
    for (int s_ = 0; s_ < steps; ++s_) {
        const int in_sweep = s_ % per_sweep;
        HSVD_TRY(launch_block_trace(ctx->stream, ordering, r, b, in_sweep, w.S2, pairs + 2 * off,
                                    ordering == HSVD_ORD_MODMOD));
        off += (size_t)(nb / 2) * (in_sweep == 0 ? 2 * b - 1 : b) * b;
    }
    HSVD_TRY(hipStreamSynchronize(ctx->stream));
    return HSVD_OK;
}

hsvd_status hsvd_sort_diag(hsvd_ctx *ctx, int r, int p, double *d, int *rho)
{
    if (!ctx || r < 1 || r > kMaxOrder || p < 0 || p > r || !d || !rho) return HSVD_E_INVAL;
    HSVD_TRY(hipSetDevice(ctx->device));
    const Layout L = make_layout(r, r + (r & 1), 64, false);
    hsvd_status s = ensure_ws(ctx, L.bytes);
    if (s != HSVD_OK) return s;
    const Workspace w = carve(ctx->ws, L);
    HSVD_TRY(launch_sort(ctx->stream, d, rho, w.dtmp, w.rtmp, r, p));
    HSVD_TRY(hipStreamSynchronize(ctx->stream));
    return HSVD_OK;
}

}  // extern "C"
